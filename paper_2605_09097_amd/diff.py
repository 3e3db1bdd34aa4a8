"""Gradients through many Schwarz frames (reverse mode over time).

The forward pass runs the frames of a coarse/fine pair and keeps a
checkpoint of both particle states every `checkpoint_every` frames.  The
reverse pass walks the segments backwards: it restores a segment's
checkpoint, reruns its frames to recover every frame's start state, and
applies the frame adjoint of the C ABI (osmpm_schwarz_frame_adjoint, which
recomputes one frame with its intermediates stored) from the last frame to
the first, carrying the adjoint of the particle states and accumulating the
derivative with respect to the Lame parameters, converted to Young's moduli
with the textbook relations.  Memory is one checkpoint per segment plus one
segment of frame start states.

adjoint="implicit" applies the fixed-point adjoint of the Schwarz iteration
instead (osmpm_schwarz_frame_adjoint_implicit): the derivative of the
converged interface data rather than of the k* iterations actually run, with
only the last iteration's intermediates stored per frame.

OSMPMStep is the torch.autograd.Function over this: E (the Young's moduli
of the scene's materials) -> final coarse particle positions.
"""
import numpy as np

from . import binding


def _lame_de(E, nu):
    """d mu / dE and d lam / dE per material."""
    nu = np.asarray(nu, dtype=np.float64)
    return 1.0 / (2.0 * (1.0 + nu)), nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


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
        self.pair = binding.SchwarzPair(ctx, scene, precision)
        so = binding.solve_opts(cg_rtol=1e-5 if precision == binding.OSMPM_MIXED else 1e-10)
        self.opts = opts if opts is not None else binding.schwarz_opts(scene.M, eps_tol=scene.eps_tol, coarse=so,
                                                                        fine=so)
        self.every = int(checkpoint_every)
        self.adj_cg_rtol = adj_cg_rtol or (1e-6 if precision == binding.OSMPM_MIXED else 1e-12)
        self.nu = np.asarray(scene.S.nu if scene.S is not None else scene.B.nu, dtype=np.float64)
        self.E = np.asarray(scene.S.E if scene.S is not None else scene.B.E, dtype=np.float64).copy()
        self.nB = len(scene.B.E)
        self.iters = []
        self.ckpt = {}
        self.adjoint = adjoint
        # the adjoint series to the forward's own Schwarz tolerance by default
        self.fp_tol = float(fp_tol) if fp_tol is not None else float(self.opts.eps_conv)
        self.fp_max = int(fp_max)
        self.fp_passes = []

    # ---- state handling (input particle order, device tensors)
    def _save(self, D):
        torch = self.torch
        x, v, B, F, i = D.particles()
        order = torch.argsort(i.long())
        return tuple(t[order].clone() for t in (x, v, B, F))

    def _restore(self, D, st):
        D.set_state(*st)

    def set_E(self, E):
        self.E = np.asarray(E, dtype=np.float64).copy()
        self.pair.B.set_materials(self.E[: self.nB], self.nu[: self.nB])
        self.pair.S.set_materials(self.E, self.nu)

    def _frame(self, f):
        pB, pS = self.scene.bc_params(f)
        self.pair.B.set_bc_params(pB)
        self.pair.S.set_bc_params(pS)
        return binding.schwarz_frame(self.pair.B, self.pair.S, self.scene.dT, self.opts)

    # ---- passes
    def forward(self, n_frames):
        """Runs frames 0 .. n_frames-1 from the scene's initial state; returns
        the final coarse and fine particle positions ([N_B][d], [N_S][d],
        input order)."""
        self.pair.B.set_particles(self.scene.B)
        self.pair.S.set_particles(self.scene.S)
        self.iters, self.ckpt = [], {}
        for f in range(n_frames):
            if f % self.every == 0:
                self.ckpt[f] = (self._save(self.pair.B), self._save(self.pair.S))
            self.iters.append(self._frame(f).iters)
        return self._save(self.pair.B)[0], self._save(self.pair.S)[0]

    def backward(self, adjB_end, adjS_end=None):
        """Reverse sweep from the adjoint of the final particle states; returns
        (dL/dE per material, adjoint of the initial coarse state, of the
        initial fine state)."""
        n = len(self.iters)
        self.fp_passes = [0] * n
        dmu, dlam = _lame_de(self.E, self.nu)
        dE = np.zeros_like(self.E)
        aB, aS = adjB_end, adjS_end
        for s0 in sorted(self.ckpt, reverse=True):
            s1 = min(s0 + self.every, n)
            self._restore(self.pair.B, self.ckpt[s0][0])
            self._restore(self.pair.S, self.ckpt[s0][1])
            starts = []
            for f in range(s0, s1):
                starts.append((self._save(self.pair.B), self._save(self.pair.S)))
                if f + 1 < s1:
                    self._frame(f)
            for f in range(s1 - 1, s0 - 1, -1):
                stB, stS = starts[f - s0]
                self._restore(self.pair.B, stB)
                self._restore(self.pair.S, stS)
                pB, pS = self.scene.bc_params(f)
                self.pair.B.set_bc_params(pB)
                self.pair.S.set_bc_params(pS)
                if self.adjoint == "implicit":
                    aB, aS, mB, lB, mS, lS, self.fp_passes[f] = binding.schwarz_frame_adjoint_implicit(
                        self.pair.B, self.pair.S, self.scene.dT, self.opts, self.iters[f], aB, aS,
                        fp_tol=self.fp_tol, fp_max=self.fp_max, adj_cg_rtol=self.adj_cg_rtol)
                else:
                    aB, aS, mB, lB, mS, lS = binding.schwarz_frame_adjoint(
                        self.pair.B, self.pair.S, self.scene.dT, self.opts, self.iters[f], aB, aS,
                        self.adj_cg_rtol)
                dE[: self.nB] += mB * dmu[: self.nB] + lB * dlam[: self.nB]
                dE += mS * dmu + lS * dlam
        return dE, aB, aS

    def close(self):
        self.pair.close()


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
            dE, _, _ = fctx.run.backward(aB, aS)
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
