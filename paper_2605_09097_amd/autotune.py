"""Tile-shape autotuner.

The tile shape of a domain (cells per workgroup tile) sets the LDS region of
the P2G, tangent and CG kernels, the number of workgroups per launch and the
halo overhead: small tiles give more workgroups (latency hiding when a domain
is small), large tiles fewer and fuller ones (better when many scenes share a
launch).  The best shape depends on the workload, so it is measured: each
candidate runs the same frames on fresh domains and the fastest wins.  The
timed frames are whole Schwarz frames through the C ABI; only the tile shape
differs between candidates.
"""
import time

from . import binding

CANDIDATES_2D = [(4, 4), (8, 4), (8, 8), (16, 8), (16, 16)]
CANDIDATES_3D = [(4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4)]


def _frames(run_frame, warmup, frames, torch):
    for _ in range(warmup):
        run_frame()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(frames):
        run_frame()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / frames


def tune_pair(ctx, scene, opts, precision=binding.OSMPM_FP64, candidates=None, warmup=1, frames=2):
    """Best (tile_B, tile_S) for one coarse/fine pair, searching the two sides
    one after the other (coarse with the default fine tile, then fine with the
    chosen coarse tile).  Returns (tile_B, tile_S, {description: seconds})."""
    import torch

    cands = candidates or (CANDIDATES_2D if scene.B.dim == 2 else CANDIDATES_3D)
    timings = {}

    def measure(tB, tS):
        key = "B%s S%s" % (tB, tS)
        if key not in timings:
            pair = binding.SchwarzPair(ctx, scene, precision, tile_B=tB, tile_S=tS)
            try:
                timings[key] = _frames(lambda: pair.frame(opts), warmup, frames, torch)
            finally:
                pair.close()
        return timings[key]

    default = cands[len(cands) // 2]
    tB = min(cands, key=lambda t: measure(t, default))
    tS = min(cands, key=lambda t: measure(tB, t))
    return tB, tS, timings


def tune_batch(ctx, scenes, opts, precision=binding.OSMPM_FP64, candidates=None, warmup=1, frames=1):
    """Best single tile shape for every domain of a Schwarz batch of the
    given scenes.  Returns (tile, {tile: seconds per frame})."""
    import torch

    cands = candidates or (CANDIDATES_2D if scenes[0].B.dim == 2 else CANDIDATES_3D)
    timings = {}
    for t in cands:
        sb = binding.SchwarzBatch(ctx, scenes, precision=precision, tile=t)
        try:
            timings[t] = _frames(lambda: sb.frame(opts), warmup, frames, torch)
        finally:
            sb.close()
    return min(timings, key=timings.get), timings
