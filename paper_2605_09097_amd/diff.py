"""Gradients through many Schwarz frames (reverse mode over time).

A thin layer over the library's multi-frame run and its reverse mode
(osmpm_batch_run / osmpm_batch_backward): the library runs the frames, keeps
a checkpoint of every particle state every `checkpoint_every` frames,
reruns each segment in the reverse pass to recover its frame start states,
applies the frame adjoints from the last frame to the first and maps the
Lame-parameter derivatives to Young's moduli.  This module only marshals:
scene boundary-condition tables in, device tensors of the loss adjoint in,
and the per-domain material derivatives out, added onto the scene's
material list (the fine domain's list, whose first entries are the coarse
domain's materials).

adjoint="implicit" applies the fixed-point adjoint of the Schwarz iteration
to every frame instead of the unrolled one (the derivative of the converged
interface data rather than of the k* iterations actually run).

OSMPMStep is the torch.autograd.Function over this: E (the Young's moduli
of the scene's materials) -> final coarse and fine particle positions.
"""
import numpy as np

from . import binding


class SchwarzRun:
    """A scene's coarse/fine pair run over frames, differentiable with respect
    to the Young's moduli of its materials (indexed as in the fine domain,
    whose material list contains the coarse one's as a prefix)."""

    def __init__(self, ctx, scene, precision=binding.OSMPM_FP64, opts=None, checkpoint_every=10, adj_cg_rtol=None,
                 adjoint="unrolled", fp_tol=None, fp_max=400):
        if adjoint not in ("unrolled", "implicit"):
            raise ValueError("adjoint must be 'unrolled' or 'implicit'")
        self.ctx = ctx
        self.torch = ctx.torch
        self.scene = scene
        self.sb = binding.SchwarzBatch(ctx, [scene], precision)
        self.pair = self.sb.pairs[0]
        so = binding.solve_opts(cg_rtol=1e-5 if precision == binding.OSMPM_MIXED else 1e-10)
        self.opts = opts if opts is not None else binding.schwarz_opts(scene.M, eps_tol=scene.eps_tol, coarse=so,
                                                                        fine=so)
        self.every = int(checkpoint_every)
        self.adj_cg_rtol = adj_cg_rtol or (1e-6 if precision == binding.OSMPM_MIXED else 1e-12)
        self.nu = np.asarray(scene.S.nu, dtype=np.float64)
        self.E = np.asarray(scene.S.E, dtype=np.float64).copy()
        self.nB = len(scene.B.E)
        self.iters = []
        self.adjoint = adjoint
        # the adjoint series to the forward's own Schwarz tolerance by default
        self.fp_tol = float(fp_tol) if fp_tol is not None else float(self.opts.eps_conv)
        self.fp_max = int(fp_max)

    def _positions(self, D):
        x, _, _, _, i = D.particles()
        return x[self.torch.argsort(i.long())]

    def set_E(self, E):
        self.E = np.asarray(E, dtype=np.float64).copy()
        self.pair.B.set_materials(self.E[: self.nB], self.nu[: self.nB])
        self.pair.S.set_materials(self.E, self.nu)

    def forward(self, n_frames):
        """Runs frames 0 .. n_frames-1 from the scene's initial state; returns
        the final coarse and fine particle positions ([N_B][d], [N_S][d],
        input order, device tensors)."""
        self.pair.B.set_particles(self.scene.B)
        self.pair.S.set_particles(self.scene.S)
        self.sb.frame_index = 0
        st = self.sb.run(int(n_frames), self.opts, self.every)
        self.iters = [fr[0].iters for fr in st]
        return self._positions(self.pair.B), self._positions(self.pair.S)

    def backward(self, adjB_end, adjS_end=None):
        """dL/dE per material from the adjoint of the final particle positions
        ({"x": tensor [N][d]} per domain, or None)."""
        for a in (adjB_end, adjS_end):
            if a is not None and any(a.get(k) is not None for k in ("v", "B", "F")):
                raise ValueError("the multi-frame reverse mode takes position adjoints only")

        def dev(a):
            if a is None or a.get("x") is None:
                return None
            t = a["x"]
            if not hasattr(t, "device"):
                t = self.torch.as_tensor(np.asarray(t, dtype=np.float64))
            return t.to(device=self.ctx.device, dtype=self.torch.float64).contiguous()

        (dB, dS), = self.sb.backward([dev(adjB_end)], [dev(adjS_end)], adj_cg_rtol=self.adj_cg_rtol,
                                     implicit=self.adjoint == "implicit", fp_tol=self.fp_tol, fp_max=self.fp_max)
        dE = np.zeros_like(self.E)
        dE[: self.nB] += dB
        dE += dS
        return dE

    def close(self):
        self.sb.close()


def _autograd_function():
    import torch

    class OSMPMStep(torch.autograd.Function):
        """E (Young's moduli of the scene's materials, CPU float64) -> final
        coarse and fine particle positions after n_frames (device float64)."""

        @staticmethod
        def forward(fctx, E, run, n_frames):
            run.set_E(E.detach().cpu().numpy())
            fctx.run = run
            return run.forward(int(n_frames))

        @staticmethod
        def backward(fctx, grad_xB, grad_xS):
            aB = {"x": grad_xB.detach().to(torch.float64)} if grad_xB is not None else None
            aS = {"x": grad_xS.detach().to(torch.float64)} if grad_xS is not None else None
            dE = fctx.run.backward(aB, aS)
            return torch.as_tensor(dE, dtype=torch.float64), None, None

    return OSMPMStep


def osmpm_step():
    """The torch.autograd.Function class (created on first use, so importing
    this module does not import torch)."""
    global _OSMPMStep
    try:
        return _OSMPMStep
    except NameError:
        _OSMPMStep = _autograd_function()
        return _OSMPMStep
