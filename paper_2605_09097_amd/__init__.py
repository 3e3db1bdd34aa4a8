"""MI355X-native OS-MPM: the implicit per-subdomain MPM step and the
overlapping-Schwarz coarse/fine coupling of arXiv 2605.09097 as hand-written
HIP kernels for gfx950 behind a C ABI (``include/osmpm.h``).

``paper_2605_09097_amd.binding`` loads the built library and exposes its
entry points; ``paper_2605_09097_amd.scenes`` builds seeded synthetic inputs.
"""
