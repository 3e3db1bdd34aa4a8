"""Pins of the oracle's implicit (fixed-point) adjoint of the Schwarz frame.

The Schwarz iteration of Alg. 1 contracts (Sec. 2.3), so its fixed point
z* = Phi(z*) is a smooth function of the start-of-frame states and the
materials.  Its derivative is fixed without the adjoint: central differences
of the forward frame run to the fixed point within rounding (60 forced
iterations; the small inclusion contracts by ~0.6 per iteration, so the
interface residual is below 1e-12 and no discrete decision moves with the
perturbation).  The implicit adjoint must match those differences

* when computed from the same converged forward (to 1e-6, the bar of the
  unrolled adjoint's pins), and
* when computed from the forward at the paper's tolerance eps_conv = 1e-5
  (22 iterations), to 2e-5: it is linearised at an iterate within the
  forward tolerance of z*.

A wrong linearisation point (an earlier iterate's intermediates), a Neumann
term whose material or start-state contribution is dropped, or a missing
Step-1 / Step-2 transpose shows up as an error of the order of the first
Schwarz residual (~4%) or larger.
"""
import numpy as np
import pytest

import oracle

TIGHT = dict(newton_rtol=1e-13, newton_atol=1e-18, cg_rtol=1e-14, max_newton=60, max_cg=20000)
K_CONV = 60


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.fixture(scope="module")
def case():
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_tiny")
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
    K_paper = oracle.schwarz_frame(OB, OS, sc.dT, oo).iters
    oc = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so, force_iters=K_CONV)
    OB.set_state(sB0)
    OS.set_state(sS0)
    st = oracle.schwarz_frame(OB, OS, sc.dT, oc)
    assert st.r_B < 1e-12 and st.r_S < 1e-12
    rng = np.random.default_rng(7)
    WB = {k: rng.standard_normal(v.shape) for k, v in sB0.items()}
    WS = {k: rng.standard_normal(v.shape) for k, v in sS0.items()}
    lame = (OB.mu.copy(), OB.lam.copy(), OS.mu.copy(), OS.lam.copy())

    def run(sB, sS, muB, lamB, muS, lamS):
        OB.set_state(sB)
        OS.set_state(sS)
        OB.set_lame(muB, lamB)
        OS.set_lame(muS, lamS)
        oracle.schwarz_frame(OB, OS, sc.dT, oc)
        oB, oS = OB.state(), OS.state()
        return sum(float(np.sum(WB[k] * oB[k])) for k in WB) + sum(float(np.sum(WS[k] * oS[k])) for k in WS)

    adj = {}
    for name, K in (("conv", K_CONV), ("paper", K_paper)):
        of = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=so, fine=so, force_iters=K)
        OB.set_state(sB0)
        OS.set_state(sS0)
        adj[name] = oracle.schwarz_frame_adjoint_implicit(OB, OS, sc.dT, of, K, WB, WS, fp_tol=1e-13, fp_max=400)
    return dict(run=run, adj=adj, sB0=sB0, sS0=sS0, lame=lame, K_paper=K_paper, rng=rng, sc=sc, so=so,
                OB=OB, OS=OS, WB=WB, WS=WS)


def _material_fd(c, m, which):
    muB0, lamB0, muS0, lamS0 = c["lame"]
    base = (muS0 if which == "mu" else lamS0)[m]
    h = 1e-5 * base

    def perturb(sgn):
        mB, lB, mS, lS = muB0.copy(), lamB0.copy(), muS0.copy(), lamS0.copy()
        for arr in ((mB, mS) if which == "mu" else (lB, lS)):
            if m < len(arr):
                arr[m] += sgn * h
        return c["run"](c["sB0"], c["sS0"], mB, lB, mS, lS)

    return (perturb(1) - perturb(-1)) / (2 * h)


def _state_fds(c):
    out = []
    for dom in ("B", "S"):
        for k, step in (("x", 1e-4 / 50), ("v", 1e-4), ("F", 1e-5)):
            s0 = c["sB0"] if dom == "B" else c["sS0"]
            dirn = c["rng"].standard_normal(s0[k].shape)
            s1 = {kk: vv.copy() for kk, vv in s0.items()}
            s2 = {kk: vv.copy() for kk, vv in s0.items()}
            s1[k] = s0[k] + step * dirn
            s2[k] = s0[k] - step * dirn
            if dom == "B":
                fd = (c["run"](s1, c["sS0"], *c["lame"]) - c["run"](s2, c["sS0"], *c["lame"])) / (2 * step)
            else:
                fd = (c["run"](c["sB0"], s1, *c["lame"]) - c["run"](c["sB0"], s2, *c["lame"])) / (2 * step)
            out.append((dom, k, dirn, fd))
    return out


@pytest.fixture(scope="module")
def fds(case):
    mats = {(m, w): _material_fd(case, m, w) for m in range(len(case["lame"][2])) for w in ("mu", "lam")}
    return mats, _state_fds(case)


@pytest.mark.parametrize("name,tol", [("conv", 1e-6), ("paper", 2e-5)])
def test_implicit_adjoint_matches_fd_of_fixed_point(case, fds, name, tol):
    aB, aS, mubB, labB, mubS, labS, passes = case["adj"][name]
    assert passes > 20  # the series runs at the forward's contraction rate
    mats, states = fds
    for (m, which), fd in mats.items():
        bB = mubB if which == "mu" else labB
        bS = mubS if which == "mu" else labS
        ad = (bB[m] if m < len(bB) else 0.0) + bS[m]
        assert _rel(ad, fd) < tol, (name, which, m, ad, fd)
    for dom, k, dirn, fd in states:
        ad = float(np.sum((aB if dom == "B" else aS)[k] * dirn))
        assert _rel(ad, fd) < tol, (name, dom, k, ad, fd)


def test_implicit_adjoint_reports_non_convergence(case):
    c = case
    of = oracle.schwarz_opts(c["sc"].M, eps_tol=c["sc"].eps_tol, coarse=c["so"], fine=c["so"], force_iters=2)
    c["OB"].set_state(c["sB0"])
    c["OS"].set_state(c["sS0"])
    c["OB"].set_lame(*c["lame"][:2])
    c["OS"].set_lame(*c["lame"][2:])
    with pytest.raises(oracle.OracleError):
        oracle.schwarz_frame_adjoint_implicit(c["OB"], c["OS"], c["sc"].dT, of, 2, c["WB"], c["WS"], fp_tol=1e-30,
                                              fp_max=2)
