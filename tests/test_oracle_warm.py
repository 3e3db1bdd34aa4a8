"""Pins of the oracle's warm-started Schwarz iterations.

With warm_start, every implicit solve after a frame's first Schwarz
iteration starts from the same solve's solution in the previous iteration
and tests Newton convergence against the initial gradient norm of that
solve's first (cold) iteration.  Only the initial iterate changes, so the
frames must reach the cold-started frames' results to the solvers'
tolerances (Newton rtol 1e-8 of the initial gradient, CG rtol 1e-10), with
the same Schwarz iteration counts and fewer Newton iterations.  Checked on
the pair frame (small inclusion and small 3D fold) and on the frame with two
refined regions."""
import numpy as np
import pytest

import oracle
from paper_2605_09097_amd import scenes


def _run(sc, n_frames, warm):
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, warm_start=warm)
    stats = []
    for f in range(n_frames):
        pB, pS = sc.bc_params(f)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        stats.append(oracle.schwarz_frame(OB, OS, sc.dT, oo))
    return OB, OS, stats


@pytest.mark.parametrize("name,frames", [("inclusion_tiny", 4), ("fold_tiny", 1)])
def test_warm_started_frames_reach_the_cold_started_result(name, frames):
    sc = scenes.workload(name)
    Bc, Sc, sc_stats = _run(sc, frames, False)
    Bw, Sw, sw_stats = _run(sc, frames, True)
    assert [s.iters for s in sc_stats] == [s.iters for s in sw_stats]
    newton_cold = sum(s.newton_B + s.newton_S for s in sc_stats)
    newton_warm = sum(s.newton_B + s.newton_S for s in sw_stats)
    assert newton_warm < newton_cold
    for (Oc, Ow, spec) in ((Bc, Bw, sc.B), (Sc, Sw, sc.S)):
        disp = np.abs(Oc.x - spec.x).max()
        assert np.abs(Ow.x - Oc.x).max() < 1e-6 * disp
        assert np.abs(Ow.F - Oc.F).max() < 1e-6 * np.abs(Oc.F - np.eye(spec.dim)).max()


def test_warm_started_multi_domain_frame():
    sc = scenes.two_inclusion_scene(20, 50, delta=0.01, n_frames=10)
    res = {}
    for warm in (False, True):
        OB = oracle.Domain(sc.B)
        OS = [oracle.Domain(s) for s in sc.S]
        oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, warm_start=warm)
        st = []
        for f in range(2):
            pB, _ = sc.bc_params(f)
            OB.set_bc_params(pB)
            st.append(oracle.schwarz_frame_multi(OB, OS, sc.dT, oo))
        res[warm] = (OB, OS, st)
    (Bc, Sc, stc), (Bw, Sw, stw) = res[False], res[True]
    assert [s.iters for s in stc] == [s.iters for s in stw]
    assert sum(s.newton_B + s.newton_S for s in stw) < sum(s.newton_B + s.newton_S for s in stc)
    assert np.abs(Bw.x - Bc.x).max() < 1e-6 * np.abs(Bc.x - sc.B.x).max()
    for Ow, Oc, spec in zip(Sw, Sc, sc.S):
        assert np.abs(Ow.x - Oc.x).max() < 1e-6 * np.abs(Oc.x - spec.x).max()
