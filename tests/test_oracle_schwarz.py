"""Pins of the oracle's Schwarz frame (Alg. 1) against results fixed without it.

* A rigid translation of stress-free material through the coupled frame is
  reproduced exactly: every transfer in the loop (P2G, the spatial projection
  and interpolation, the temporal interpolation, the Dirichlet data of the
  solves, G2P and advection) maps a uniform velocity field to itself, so the
  first Schwarz iteration already meets the tolerance and no Newton step is
  taken.  The only departure is the projection's regulariser eps_tol.
* At identical resolution the two-domain run of the cantilever (Sec. 4.1)
  agrees with the single-domain run of the same beam: both discretise the
  same problem and the paper reports the two as nearly coincident.  The
  comparison runs over the early frames, particle by particle (the beams are
  sampled on the same unjittered lattice), against the beam's deflection:
  tightly at the tip and away from the overlap, loosely inside it.
"""
import dataclasses

import numpy as np

import oracle
from paper_2605_09097_amd import scenes


def _stress_free(spec, v0):
    """The domain with uniform velocity v0, no affine part, F = I, and no
    scene-BC groups (only the boundary-layer marker kept)."""
    n, d = spec.x.shape
    return dataclasses.replace(spec, bc_kind=[], bc_mask=[],
                               flags=(spec.flags & np.uint8(1)).astype(spec.flags.dtype),
                               v=np.tile(v0, (n, 1)), B=np.zeros((n, d, d)),
                               F=np.tile(np.eye(d), (n, 1, 1)))


def test_rigid_translation_through_schwarz_frames():
    sc = scenes.workload("inclusion_tiny")
    v0 = np.array([0.3, -0.2])
    B, S = _stress_free(sc.B, v0), _stress_free(sc.S, v0)
    OB, OS = oracle.Domain(B), oracle.Domain(S)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    step = sc.dT * np.linalg.norm(v0)
    for f in range(3):
        st = oracle.schwarz_frame(OB, OS, sc.dT, oo)
        assert st.converged and st.iters == 1
        assert st.newton_B == 0 and st.newton_S == 0
        assert st.n_recv_B > 0 and st.n_recv_S > 0
        for O, spec in ((OB, B), (OS, S)):
            drift = O.x - spec.x - (f + 1) * sc.dT * v0
            assert np.abs(drift).max() < 1e-8 * step
            assert np.abs(O.v - v0).max() < 1e-9 * np.linalg.norm(v0)
            assert np.abs(O.F - np.eye(2)).max() < 1e-10


def _by_position(x, digits=12):
    return {tuple(np.round(p, digits)): i for i, p in enumerate(x)}


def test_dual_domain_matches_single_domain_cantilever():
    """20 frames (t = 0.04 s) at dx = 1/100.  The tip deflection, the
    quantity the paper compares, agrees to 1e-5; over the whole beam the L2
    difference stays within 3%, and outside the band x in [0.30, 0.55]
    around the overlap [0.39, 0.45] every particle agrees to 0.5% of the
    deflection.  Inside the band the coupled run departs from the single one
    by up to ~4% of the deflection (the projection and interpolation smooth
    the velocity at the artificial boundaries); that local departure is an
    observed property of the method as read here, not a bound from the
    paper."""
    inv_dx, frames = 100, 20
    grav = (0.0, -9.81)
    so = oracle.solve_opts(gravity=grav)
    single = scenes.cantilever_scene(inv_dx=inv_dx, ppc1d=3, split=False)
    dual = scenes.cantilever_scene(inv_dx=inv_dx, ppc1d=3, split=True)
    O1 = oracle.Domain(single.B)
    O1.set_bc_params(single.bc_params(0)[0])
    OL, OR = oracle.Domain(dual.B), oracle.Domain(dual.S)
    pL, pR = dual.bc_params(0)
    OL.set_bc_params(pL)
    OR.set_bc_params(pR)
    oo = oracle.schwarz_opts(1, eps_tol=dual.eps_tol, coarse=so, fine=so)
    for _ in range(frames):
        O1.single_frame(single.dT, so)
        st = oracle.schwarz_frame(OL, OR, dual.dT, oo)
        assert st.converged
    u1 = O1.x - single.B.x
    deflection = np.abs(u1[:, 1]).max()
    assert deflection > 5e-3  # the beam has moved well beyond rounding
    tip1 = np.argmax(single.B.x[:, 0])
    tip2 = np.argmax(dual.S.x[:, 0])
    assert abs((OR.x[tip2] - dual.S.x[tip2])[1] - u1[tip1, 1]) < 1e-5 * abs(u1[tip1, 1])
    index = _by_position(single.B.x)
    num = den = far = 0.0
    for O, spec in ((OL, dual.B), (OR, dual.S)):
        u = O.x - spec.x
        for j, p in enumerate(spec.x):
            i = index[tuple(np.round(p, 12))]
            e = u[j] - u1[i]
            num += float(e @ e)
            den += float(u1[i] @ u1[i])
            if p[0] < 0.30 or p[0] > 0.55:
                far = max(far, np.abs(e).max())
    assert np.sqrt(num / den) < 3e-2
    assert far < 5e-3 * deflection
