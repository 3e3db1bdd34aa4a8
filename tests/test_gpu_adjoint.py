"""GPU parity of the reverse mode against the oracle's (which is pinned by
finite differences on the CPU): the adjoint of a single-domain frame and of
a Schwarz frame for a random linear functional of the end-of-frame states,
both with respect to the start-of-frame particle states and the Lame
parameters of every material.  FP64 path: 1e-7 relative (the forward states
of the two implementations agree to ~1e-13 and both adjoint solves run to
1e-12); mixed path (FP32 stored states and adjoint CG vectors, adjoint CG
to 1e-6): 1e-4, which the FP32 storage (relative 6e-8) and the adjoint
solves' tolerance times the small systems' condition numbers (tens) bound
with a wide margin (measured: at most 3.5e-6, on the Lame gradients)."""
import numpy as np
import pytest

import oracle
from helpers import rel_err

pytestmark = pytest.mark.gpu

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


def _weights(state_shapes, seed):
    rng = np.random.default_rng(seed)
    return {k: rng.standard_normal(s) for k, s in state_shapes.items()}


def _cmp(gpu_adj, or_adj, tol, what):
    for k in "xvBF":
        g = gpu_adj[k].cpu().numpy()
        assert rel_err(g, or_adj[k]) < tol, (what, k, rel_err(g, or_adj[k]))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_frame_adjoint_parity(ctx, precision):
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.inclusion_single(inv_dx=16, n_frames=3, delta=0.01)
    prec = b.OSMPM_FP64 if precision == "fp64" else b.OSMPM_MIXED
    tol = 1e-7 if precision == "fp64" else 1e-4
    so = b.solve_opts(newton_rtol=1e-12, newton_atol=1e-16, cg_rtol=1e-12 if precision == "fp64" else 1e-5)
    D = b.Domain(ctx, sc.B, precision=prec)
    O = oracle.Domain(sc.B)
    p, _ = sc.bc_params(0)
    D.set_bc_params(p)
    O.set_bc_params(p)
    W = _weights({k: v.shape for k, v in O.state().items()}, 3)
    print("single-domain frame adjoint,", precision, flush=True)
    ga, gmu, glam = b.single_frame_adjoint(D, sc.dT, so, W, adj_cg_rtol=1e-12 if precision == "fp64" else 1e-6)
    oa, omu, olam = oracle.single_frame_adjoint(O, sc.dT, oracle.solve_opts(**TIGHT_OR), W)
    _cmp(ga, oa, tol, "state")
    assert rel_err(gmu, omu) < tol and rel_err(glam, olam) < tol
    # the domain holds the end-of-frame state afterwards
    x = D.particles_input_order()[0]
    assert rel_err(x - sc.B.x, O.x - sc.B.x) < (1e-9 if precision == "fp64" else 1e-4)
    D.close()


def _schwarz_case(ctx, precision):
    """The small inclusion on both sides advanced two frames; the pair and
    the oracle hold the start of frame 3, K = the oracle's iteration count."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_tiny")
    prec = b.OSMPM_FP64 if precision == "fp64" else b.OSMPM_MIXED
    so = b.solve_opts(newton_rtol=1e-12, newton_atol=1e-16, cg_rtol=1e-12 if precision == "fp64" else 1e-5)
    go = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so)
    sor = oracle.solve_opts(**TIGHT_OR)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=sor, fine=sor)
    pair = b.SchwarzPair(ctx, sc, precision=prec)
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    for f in range(2):
        pB, pS = sc.bc_params(f)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        oracle.schwarz_frame(OB, OS, sc.dT, oo)
        pair.frame(go)
    pB, pS = sc.bc_params(2)
    OB.set_bc_params(pB)
    OS.set_bc_params(pS)
    pair.B.set_bc_params(pB)
    pair.S.set_bc_params(pS)
    sB0, sS0 = OB.state(), OS.state()
    K = oracle.schwarz_frame(OB, OS, sc.dT, oo).iters
    OB.set_state(sB0)
    OS.set_state(sS0)
    WB = _weights({k: v.shape for k, v in sB0.items()}, 5)
    WS = _weights({k: v.shape for k, v in sS0.items()}, 6)
    return sc, go, oo, pair, OB, OS, K, WB, WS


def _cmp_frame(g, o, tol):
    _cmp(g[0], o[0], tol, "B")
    _cmp(g[1], o[1], tol, "S")
    for a, b_ in zip(g[2:6], o[2:6]):
        assert rel_err(a, b_) < tol, (a, b_)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_schwarz_frame_adjoint_parity(ctx, precision):
    from paper_2605_09097_amd import binding as b

    sc, go, oo, pair, OB, OS, K, WB, WS = _schwarz_case(ctx, precision)
    tol = 1e-7 if precision == "fp64" else 1e-4
    print("Schwarz frame adjoint,", precision, "K =", K, flush=True)
    g = b.schwarz_frame_adjoint(pair.B, pair.S, sc.dT, go, K, WB, WS,
                                adj_cg_rtol=1e-12 if precision == "fp64" else 1e-6)
    o = oracle.schwarz_frame_adjoint(OB, OS, sc.dT, oo, K, WB, WS)
    _cmp_frame(g, o, tol)
    pair.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_schwarz_frame_adjoint_implicit_parity(ctx, precision):
    """The fixed-point adjoint with a fixed number of passes (30) against
    the oracle's, then (FP64) with the pass count left to the tolerance: the
    same count on both sides."""
    from paper_2605_09097_amd import binding as b

    sc, go, oo, pair, OB, OS, K, WB, WS = _schwarz_case(ctx, precision)
    tol = 1e-7 if precision == "fp64" else 1e-4
    rtol = 1e-12 if precision == "fp64" else 1e-6
    print("implicit Schwarz frame adjoint, 30 passes,", precision, "K =", K, flush=True)
    g = b.schwarz_frame_adjoint_implicit(pair.B, pair.S, sc.dT, go, K, WB, WS, fp_tol=0.0, fp_max=30,
                                         adj_cg_rtol=rtol)
    o = oracle.schwarz_frame_adjoint_implicit(OB, OS, sc.dT, oo, K, WB, WS, fp_tol=0.0, fp_max=30)
    assert g[6] == 30 and o[6] == 30
    _cmp_frame(g, o, tol)
    if precision == "fp64":
        # a fresh pair and oracle at the start of the same frame
        pair.close()
        sc, go, oo, pair, OB, OS, K2, WB, WS = _schwarz_case(ctx, precision)
        assert K2 == K
        print("implicit Schwarz frame adjoint to fp_tol 1e-9, fp64", flush=True)
        g = b.schwarz_frame_adjoint_implicit(pair.B, pair.S, sc.dT, go, K, WB, WS, fp_tol=1e-9, fp_max=200,
                                             adj_cg_rtol=rtol)
        o = oracle.schwarz_frame_adjoint_implicit(OB, OS, sc.dT, oo, K, WB, WS, fp_tol=1e-9, fp_max=200)
        assert g[6] == o[6] and g[6] > 30, (g[6], o[6])
        _cmp_frame(g, o, tol)
        # the pair holds the end-of-frame state afterwards, as after the forward call
        xg = pair.S.particles_input_order()[0]
        assert rel_err(xg - sc.S.x, OS.x - sc.S.x) < 1e-9
    pair.close()


def test_autograd_gradient_matches_oracle(ctx):
    """dL/dE through four frames of the small inclusion on the GPU
    (torch.autograd over OSMPMStep, checkpoints every two frames, so the
    reverse sweep restores and reruns segments) against the oracle's reverse
    sweep over the same frames (FP64, tight solves)."""
    import torch

    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import diff, scenes

    sc = scenes.workload("inclusion_tiny")
    n = 4
    so = b.solve_opts(newton_rtol=1e-12, newton_atol=1e-16, cg_rtol=1e-12)
    go = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so)
    idx, target = scenes.top_edge_target(sc, n, seed=3)
    tS = np.asarray(sc.S.x) + 1e-4 * np.random.default_rng(4).standard_normal(np.asarray(sc.S.x).shape)
    run = diff.SchwarzRun(ctx, sc, b.OSMPM_FP64, opts=go, checkpoint_every=2)
    E = torch.tensor(np.asarray(sc.S.E, dtype=np.float64), requires_grad=True)
    xB, xS = diff.osmpm_step().apply(E, run, n)
    tgt = torch.as_tensor(target, device=xB.device)
    tSd = torch.as_tensor(tS, device=xS.device)
    L = 0.5 * ((xB[torch.as_tensor(idx, device=xB.device)] - tgt) ** 2).sum() + 0.5 * ((xS - tSd) ** 2).sum()
    print("autograd through", n, "frames, iters", run.iters, flush=True)
    L.backward()
    run.close()

    sor = oracle.solve_opts(**TIGHT_OR)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=sor, fine=sor)
    E0 = np.asarray(sc.S.E, dtype=np.float64)
    Bd, Sd, starts, iters = oracle.schwarz_run(sc, E0, n, oo)
    assert iters == run.iters
    r = Bd.x[idx] - target
    q = Sd.x - tS
    Lo = 0.5 * float(np.sum(r * r)) + 0.5 * float(np.sum(q * q))
    xbar = np.zeros_like(Bd.x)
    xbar[idx] = r
    # (the reverse sweep leaves the oracle domains at an earlier state)
    dE, _, _ = oracle.schwarz_run_gradient(sc, E0, Bd, Sd, starts, iters, oo, {"x": xbar}, {"x": q})
    assert abs(float(L.detach()) - Lo) <= 1e-9 * abs(Lo)
    assert rel_err(E.grad.numpy(), dE) < 1e-6, (E.grad.numpy(), dE)
