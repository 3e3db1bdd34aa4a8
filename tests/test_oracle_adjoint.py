"""Pins of the oracle's reverse mode (CPU): the adjoint of a frame against
central finite differences of the forward oracle.

The loss is a random linear functional of the end-of-frame particle states,
L = sum_k <W_k, state_k>, so dL/d(start state) and dL/d(mu, lam) of every
material come from one adjoint run.  Forward solves run to tight tolerances
(Newton 1e-13 relative, CG 1e-14) and the Schwarz frame with its iteration
count held at the forward's value, so finite differences see the same
discrete decisions.  A dropped term of the adjoint (a transfer's position
dependence, the material or F^n terms of the solve, a Dirichlet coupling,
a projection or interpolation transpose) shows up as an O(1) relative error.
"""
import numpy as np
import pytest

import oracle

TIGHT = dict(newton_rtol=1e-13, newton_atol=1e-18, cg_rtol=1e-14, max_newton=60, max_cg=20000)
TOL = 1e-6


def _scenes():
    from paper_2605_09097_amd import scenes

    return scenes


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_single_frame_adjoint_matches_fd():
    sc = _scenes().inclusion_single(inv_dx=16, n_frames=3, delta=0.01)
    opts = oracle.solve_opts(**TIGHT)
    D = oracle.Domain(sc.B)
    p, _ = sc.bc_params(0)
    D.set_bc_params(p)
    rng = np.random.default_rng(0)
    s0 = D.state()
    W = {k: rng.standard_normal(v.shape) for k, v in s0.items()}
    mu0, lam0 = D.mu.copy(), D.lam.copy()

    def run(st, mu, lam):
        D.set_state(st)
        D.set_lame(mu, lam)
        D.single_frame(sc.dT, opts)
        out = D.state()
        return sum(float(np.sum(W[k] * out[k])) for k in W)

    D.set_state(s0)
    adj, mub, lab = oracle.single_frame_adjoint(D, sc.dT, opts, W)
    for m in range(len(mu0)):
        for which, base, bar in (("mu", mu0, mub), ("lam", lam0, lab)):
            h = 1e-5 * base[m]
            b1, b2 = base.copy(), base.copy()
            b1[m] += h
            b2[m] -= h
            if which == "mu":
                fd = (run(s0, b1, lam0) - run(s0, b2, lam0)) / (2 * h)
            else:
                fd = (run(s0, mu0, b1) - run(s0, mu0, b2)) / (2 * h)
            assert _rel(bar[m], fd) < TOL, (which, m, bar[m], fd)
    for k, step in (("x", 1e-4 / 16), ("v", 1e-4), ("B", 1e-4), ("F", 1e-5)):
        dirn = rng.standard_normal(s0[k].shape)
        s1 = {kk: vv.copy() for kk, vv in s0.items()}
        s2 = {kk: vv.copy() for kk, vv in s0.items()}
        s1[k] = s0[k] + step * dirn
        s2[k] = s0[k] - step * dirn
        fd = (run(s1, mu0, lam0) - run(s2, mu0, lam0)) / (2 * step)
        assert _rel(float(np.sum(adj[k] * dirn)), fd) < TOL, k


@pytest.fixture(scope="module")
def schwarz_case():
    """The small inclusion advanced three frames (so the fine domain moves),
    then the adjoint of frame 3 against its forward."""
    sc = _scenes().workload("inclusion_tiny")
    so = oracle.solve_opts(**TIGHT)
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so)
    for f in range(3):
        pB, pS = sc.bc_params(f)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        oracle.schwarz_frame(OB, OS, sc.dT, oo)
    pB, pS = sc.bc_params(3)
    OB.set_bc_params(pB)
    OS.set_bc_params(pS)
    sB0, sS0 = OB.state(), OS.state()
    K = oracle.schwarz_frame(OB, OS, sc.dT, oo).iters
    of = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so, force_iters=K)
    rng = np.random.default_rng(1)
    WB = {k: rng.standard_normal(v.shape) for k, v in sB0.items()}
    WS = {k: rng.standard_normal(v.shape) for k, v in sS0.items()}
    lame = (OB.mu.copy(), OB.lam.copy(), OS.mu.copy(), OS.lam.copy())

    def run(sB, sS, muB, lamB, muS, lamS):
        OB.set_state(sB)
        OS.set_state(sS)
        OB.set_lame(muB, lamB)
        OS.set_lame(muS, lamS)
        oracle.schwarz_frame(OB, OS, sc.dT, of)
        oB, oS = OB.state(), OS.state()
        return sum(float(np.sum(WB[k] * oB[k])) for k in WB) + sum(float(np.sum(WS[k] * oS[k])) for k in WS)

    OB.set_state(sB0)
    OS.set_state(sS0)
    adj = oracle.schwarz_frame_adjoint(OB, OS, sc.dT, of, K, WB, WS)
    return dict(run=run, adj=adj, sB0=sB0, sS0=sS0, lame=lame, K=K, rng=rng)


def test_schwarz_frame_adjoint_materials_match_fd(schwarz_case):
    c = schwarz_case
    aB, aS, mubB, labB, mubS, labS = c["adj"]
    muB0, lamB0, muS0, lamS0 = c["lame"]
    assert c["K"] >= 2
    # material 0 (the matrix) lives in both domains, material 1 (the inclusion) in the fine one
    for m in range(len(muS0)):
        for which in ("mu", "lam"):
            base = (muS0 if which == "mu" else lamS0)[m]
            h = 1e-5 * base

            def perturb(sgn):
                mB, lB, mS, lS = muB0.copy(), lamB0.copy(), muS0.copy(), lamS0.copy()
                tgt = (mB, mS) if which == "mu" else (lB, lS)
                for arr in tgt:
                    if m < len(arr):
                        arr[m] += sgn * h
                return c["run"](c["sB0"], c["sS0"], mB, lB, mS, lS)

            fd = (perturb(1) - perturb(-1)) / (2 * h)
            bB = (mubB if which == "mu" else labB)
            bS = (mubS if which == "mu" else labS)
            ad = (bB[m] if m < len(bB) else 0.0) + bS[m]
            assert _rel(ad, fd) < TOL, (which, m, ad, fd)


@pytest.mark.parametrize("dom", ["B", "S"])
def test_schwarz_frame_adjoint_states_match_fd(schwarz_case, dom):
    c = schwarz_case
    aB, aS = c["adj"][0], c["adj"][1]
    lame = c["lame"]
    for k, step in (("x", 1e-4 / 50), ("v", 1e-4), ("B", 1e-5), ("F", 1e-5)):
        s0 = c["sB0"] if dom == "B" else c["sS0"]
        dirn = c["rng"].standard_normal(s0[k].shape)
        s1 = {kk: vv.copy() for kk, vv in s0.items()}
        s2 = {kk: vv.copy() for kk, vv in s0.items()}
        s1[k] = s0[k] + step * dirn
        s2[k] = s0[k] - step * dirn
        if dom == "B":
            fd = (c["run"](s1, c["sS0"], *lame) - c["run"](s2, c["sS0"], *lame)) / (2 * step)
            ad = float(np.sum(aB[k] * dirn))
        else:
            fd = (c["run"](c["sB0"], s1, *lame) - c["run"](c["sB0"], s2, *lame)) / (2 * step)
            ad = float(np.sum(aS[k] * dirn))
        assert _rel(ad, fd) < TOL, (dom, k, ad, fd)


def test_multi_frame_gradient_matches_fd():
    """dL/dE through four Schwarz frames of the small inclusion (oracle
    reverse sweep) against central differences of the forward with every
    frame's Schwarz iteration count held.  L = seeded top-edge mismatch of the
    coarse domain + a seeded mismatch of the fine particle positions (the
    inclusion modulus reaches the top edge only weakly within four frames)."""
    scenes = _scenes()
    sc = scenes.workload("inclusion_tiny")
    n = 4
    so = oracle.solve_opts(**TIGHT)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so)
    E0 = np.asarray(sc.S.E, dtype=np.float64)
    idx, target = scenes.top_edge_target(sc, n, seed=3)
    tS = np.asarray(sc.S.x) + 1e-4 * np.random.default_rng(4).standard_normal(np.asarray(sc.S.x).shape)

    def loss(Bd, Sd):
        r = Bd.x[idx] - target
        q = Sd.x - tS
        return 0.5 * float(np.sum(r * r)) + 0.5 * float(np.sum(q * q)), r, q

    Bd, Sd, starts, iters = oracle.schwarz_run(sc, E0, n, oo)
    L0, r, q = loss(Bd, Sd)
    xbar = np.zeros_like(Bd.x)
    xbar[idx] = r
    dE, _, _ = oracle.schwarz_run_gradient(sc, E0, Bd, Sd, starts, iters, oo, {"x": xbar}, {"x": q})

    def loss_at(E):
        Bf, Sf = oracle.Domain(sc.B), oracle.Domain(sc.S)
        mu, lam = oracle.lame(E, np.asarray(sc.S.nu))
        Bf.set_lame(mu[:1], lam[:1])
        Sf.set_lame(mu, lam)
        for f in range(n):
            pB, pS = sc.bc_params(f)
            Bf.set_bc_params(pB)
            Sf.set_bc_params(pS)
            of = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so, force_iters=iters[f])
            oracle.schwarz_frame(Bf, Sf, sc.dT, of)
        return loss(Bf, Sf)[0]

    for m in range(len(E0)):
        h = 1e-4 * E0[m]
        Ep, Em = E0.copy(), E0.copy()
        Ep[m] += h
        Em[m] -= h
        fd = (loss_at(Ep) - loss_at(Em)) / (2 * h)
        assert _rel(dE[m], fd) < 1e-5, (m, dE[m], fd)
