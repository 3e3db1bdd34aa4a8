"""Physics pin of the oracle: Hertzian line contact (Sec. 4.2).

A compliant cylinder of radius R pressed onto a rigid plane by a force F per
unit length develops a semi-elliptic contact pressure
p(x) = p_max sqrt(1 - (x/b)^2) with half-width b = 2 sqrt(F R (1 - nu^2) /
(pi E)) and p_max = 2 F / (pi b) (the paper's closed form, quoted from
Johnson's Contact Mechanics).  The paper reports that its numerical profile
converges to this solution as the resolution near the contact increases, the
error falling roughly linearly with the cell size.  This test checks the
single-domain implicit MPM of the oracle (P2G, the backward-Euler energy,
Newton-CG with line search, G2P) for the same trend.

Readings (the paper states the closed form and the material, not how its
contact is imposed or measured):

* Body: the lower cap y <= H of a disc of radius R = 0.5 touching the plane
  y = 0 at x = 0 (H = 0.2: the contact width stays well inside the body),
  E = 200 kPa, nu = 0.3, rho = 1000 (the paper's values), 2x2 particles per
  cell at unjittered sub-cell centres.
* The rigid frictionless plane is MPM's grid wall: every active node at
  y <= 0 is held in y and free in x; a node of the wall row whose reaction
  would pull the body down is released and the step solved again (the
  contact is one-sided).
* Load: the particle layer of the flat top face is driven down by 0.02 in
  four quasi-static backward-Euler increments of 1000 s each (inertia ~1e-9
  of the stiffness), x free (a frictionless plate).  F is the measured
  reaction of the plane, which must equal that of the plate (equilibrium).
* Measures of the computed reaction profile r_i (node spacing dx): b from
  the second moment, since sum x^2 p / sum p = b^2 / 4 for the semi-ellipse,
  and p_max from the quadratic mean, since the integral of p^2 is
  (4/3) b p_max^2.  Both are compared with the closed form at the measured F.

Measured: at dx = R/20, R/40, R/80 the relative errors of b are +22%, +11%,
+1.3% and those of p_max -22%, -13%, -3.5% (about halving with each
refinement).  The test asserts equilibrium, monotone decrease of both errors,
and less than 6% error at R/80.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2605_09097_amd import scenes

pytestmark = pytest.mark.slow

E, NU, RHO, R = 2e5, 0.3, 1000.0, 0.5
H = 0.2
PRESS, STEPS, DT = 0.02, 4, 1000.0


def _cap(inv_dx, ppc1d=2):
    dx = 1.0 / inv_dx
    sub = (np.arange(ppc1d) + 0.5) / ppc1d
    half = math.sqrt(2 * R * H - H * H)
    nx, ny = int(math.ceil(half * inv_dx)) + 1, int(math.ceil(H * inv_dx))
    g = np.meshgrid(((np.arange(-nx, nx)[:, None] + sub[None, :]).ravel()) * dx,
                    ((np.arange(0, ny)[:, None] + sub[None, :]).ravel()) * dx, indexing="ij")
    p = np.stack([g[0].ravel(), g[1].ravel()], axis=1)
    x = p[(np.hypot(p[:, 0], p[:, 1] - R) <= R) & (p[:, 1] <= H)]
    n = len(x)
    top = x[:, 1] > H - dx / ppc1d
    vol = np.full(n, dx * dx / ppc1d ** 2)
    pad = 4
    lo, hi = [-nx - pad, -pad], [nx + pad, ny + pad]
    # group 0: the driven top layer (TRANSLATE, y only); group 1: the wall
    # nodes, assigned below (FIX, y only)
    return scenes.DomainSpec(
        dim=2, h0=dx, origin_q=[lo[0], lo[1], 0], dx_q=1, n_nodes=[hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, 1], x=x,
        v=np.zeros((n, 2)), B=np.zeros((n, 2, 2)), F=np.tile(np.eye(2), (n, 1, 1)), mass=RHO * vol, vol=vol,
        mat=np.zeros(n, np.int32), flags=np.where(top, 2, 0).astype(np.uint8), E=np.array([E]), nu=np.array([NU]),
        bc_kind=[oracle.BC_TRANSLATE, oracle.BC_FIX], bc_mask=[0b10, 0b10], m_ref=float(RHO * vol[0]),
        tau=1e-3 * float(RHO * vol[0]), ppc1d=ppc1d)


def _press(inv_dx):
    """Returns (F_plane, F_plate, b, p_max) after the loading increments."""
    dx = 1.0 / inv_dx
    O = oracle.Domain(_cap(inv_dx))
    params = np.zeros((2, 8))
    params[0, 1] = -(PRESS / STEPS) / DT
    O.set_bc_params(params)
    so = oracle.solve_opts(newton_rtol=1e-10, max_newton=100)
    xn = O.node_positions()
    row0 = np.abs(xn[:, 1]) < 1e-12
    for _ in range(STEPS):
        O.p2g()
        wall = (xn[:, 1] < 1e-12) & (O.m > 0)
        released = np.zeros(len(xn), bool)
        for _ in range(10):
            O.bcg[wall & ~released, 1] = 1
            O.bcg[released, 1] = -1
            st = O.solve(DT, so)
            assert st.converged
            r = O.gradient(DT, O.u)[:, 1]  # reaction of a held DOF (stationarity of E - r u)
            pull = wall & ~released & row0 & (r < 0)
            if not pull.any():
                break
            released |= pull
        plate = O.bcg[:, 1] == 0
        O.g2p(DT)
    rw = np.where(wall & ~released, r, 0.0)
    F, F_plate = rw.sum(), -r[plate].sum()
    xc = (rw * xn[:, 0]).sum() / F
    b = 2.0 * math.sqrt((rw * (xn[:, 0] - xc) ** 2).sum() / F)
    p_max = math.sqrt(3.0 * ((rw / dx) ** 2 * dx).sum() / (4.0 * b))
    return F, F_plate, b, p_max


def test_contact_pressure_converges_to_hertz():
    errs = []
    for inv_dx in (40, 80, 160):
        F, F_plate, b, p_max = _press(inv_dx)
        assert F > 0 and abs(F - F_plate) <= 1e-6 * F
        b_h = 2.0 * math.sqrt(F * R * (1.0 - NU ** 2) / (math.pi * E))
        p_h = 2.0 * F / (math.pi * b_h)
        errs.append((abs(b / b_h - 1.0), abs(p_max / p_h - 1.0)))
        print("dx = R/%d: F %.1f, b %.4f (Hertz %.4f), p_max %.0f (Hertz %.0f)" % (inv_dx // 2, F, b, b_h, p_max,
                                                                                     p_h))
    (b1, p1), (b2, p2), (b3, p3) = errs
    assert b1 > b2 > b3 and p1 > p2 > p3
    assert b3 < 0.06 and p3 < 0.06
