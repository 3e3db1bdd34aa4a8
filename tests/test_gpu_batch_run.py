"""GPU parity of the multi-frame run and its reverse mode
(osmpm_batch_run / osmpm_batch_backward) against the oracle's frame-by-frame
run and reverse sweep, scene by scene.

Three inclusion scenes of different grids, radii and moduli run four frames
in one batch with a checkpoint every two frames (so the reverse pass
restores a checkpoint and reruns a segment).  The loss is half the squared
distance of the coarse top-layer particles to a seeded target plus that of
every fine particle to another; its gradient with respect to each material's
Young's modulus (the chain rule from the Lame parameters runs inside the
library) must match the oracle's to 1e-6 (FP64, tight solves: both adjoints
are differentiated at converged solves, whose tolerances set the bar).
Per-frame Schwarz iteration counts must be equal, and the domains must hold
the end-of-run state after the reverse pass."""
import numpy as np
import pytest

import oracle
from helpers import rel_err

pytestmark = pytest.mark.gpu

TIGHT = dict(newton_rtol=1e-12, newton_atol=1e-16, cg_rtol=1e-12)
TIGHT_OR = dict(newton_rtol=1e-12, newton_atol=1e-16, cg_rtol=1e-13, max_newton=60, max_cg=20000)


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09097_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


def _scenes():
    from paper_2605_09097_amd import scenes

    d = scenes.INCLUSION_DELTA
    return [scenes.inclusion_scene(20, 50, r_inc=0.04, E_inc=3e4, seed=21, delta=d, name="r0"),
            scenes.inclusion_scene(30, 60, r_inc=0.07, E_inc=1.5e5, seed=22, delta=d, name="r1"),
            scenes.inclusion_scene(20, 40, r_inc=0.05, E_inc=8e4, seed=23, delta=d, name="r2")]


@pytest.mark.parametrize("mode", ["unrolled", "implicit"])
def test_batch_run_gradient_matches_oracle(ctx, mode):
    import torch

    from paper_2605_09097_amd import binding as b

    n_frames, every = 4, 2
    scs = _scenes()
    so = b.solve_opts(**TIGHT)
    go = b.schwarz_opts(scs[0].M, eps_tol=scs[0].eps_tol, coarse=so, fine=so)
    sb = b.SchwarzBatch(ctx, scs, precision=b.OSMPM_FP64)
    print("batch run,", len(scs), "scenes,", n_frames, "frames,", mode, flush=True)
    st = sb.run(n_frames, go, checkpoint_every=every)
    rng = np.random.default_rng(5)
    adjB, adjS, ref, ends = [], [], [], []
    for i, (sc, p) in enumerate(zip(scs, sb.pairs)):
        sor = oracle.solve_opts(**TIGHT_OR)
        oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=sor, fine=sor)
        E0 = np.asarray(sc.S.E, dtype=np.float64)
        Bd, Sd, starts, iters = oracle.schwarz_run(sc, E0, n_frames, oo)
        assert [fr[i].iters for fr in st] == iters
        xB, _, _, _ = p.B.particles_input_order()
        xS, _, _, _ = p.S.particles_input_order()
        ends.append((xB, xS))
        assert rel_err(xB - sc.B.x, Bd.x - sc.B.x) < 1e-9
        assert rel_err(xS - sc.S.x, Sd.x - sc.S.x) < 1e-9
        idx = np.nonzero(sc.B.flags & 4)[0]
        tB = Bd.x[idx] + 1e-4 * rng.standard_normal((len(idx), 2))
        tS = Sd.x + 1e-4 * rng.standard_normal(Sd.x.shape)
        aB = np.zeros_like(Bd.x)
        aB[idx] = Bd.x[idx] - tB
        aS = Sd.x - tS
        adjB.append(torch.as_tensor(aB, device="cuda"))
        adjS.append(torch.as_tensor(aS, device="cuda"))
        if mode == "unrolled":
            dE, _, _ = oracle.schwarz_run_gradient(sc, E0, Bd, Sd, starts, iters, oo, {"x": aB}, {"x": aS})
            ref.append(dE)
        else:
            ref.append(None)
    grads = sb.backward(adjB, adjS, adj_cg_rtol=1e-12, implicit=(mode == "implicit"), fp_tol=1e-10, fp_max=400)
    for i, (sc, p) in enumerate(zip(scs, sb.pairs)):
        dB, dS = grads[i]
        dE = np.array(dS)
        dE[: len(dB)] += dB
        assert np.all(np.isfinite(dE))
        if ref[i] is not None:
            assert rel_err(dE, ref[i]) < 1e-6, (i, dE, ref[i])
        # the domains hold the end-of-run state again
        assert np.array_equal(p.B.particles_input_order()[0], ends[i][0])
        assert np.array_equal(p.S.particles_input_order()[0], ends[i][1])
    if mode == "implicit":
        # the implicit adjoint to 1e-10 agrees with the unrolled one to the
        # Schwarz tolerance of the forward frames (1e-5)
        g_un = sb.backward(adjB, adjS, adj_cg_rtol=1e-12)
        for (dB, dS), (uB, uS) in zip(grads, g_un):
            assert rel_err(np.concatenate([dB, dS]), np.concatenate([uB, uS])) < 1e-3
    sb.close()


def test_batch_run_without_run_is_refused(ctx):
    from paper_2605_09097_amd import binding as b

    sb = b.SchwarzBatch(ctx, _scenes()[:1], precision=b.OSMPM_FP64)
    with pytest.raises(b.OsmpmError) as e:
        sb.backward([None], [None])
    assert e.value.status == 7  # OSMPM_E_STATE
    sb.close()
