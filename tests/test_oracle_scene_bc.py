"""Pins of the oracle's scene boundary conditions against closed forms.

The prescribed-displacement drives of the benchmark scenes (the translated
top edge of the inclusion, the rotated free end of the 3D fold) enter every
implicit solve as Dirichlet data on grid nodes.  When every active node of a
stress-free body carries the same drive, no degree of freedom is left free,
and G2P moves each particle by the interpolated node displacement.  Quadratic
B-splines reproduce affine fields exactly (partition of unity and linear
reproduction), and both drives are affine in the node position, so the body
must move rigidly:

* TRANSLATE with velocity c: after n frames x_p = x_p^0 + n dt c and F = I;
* ROTATE about the axis through c with unit direction k at rate omega: each
  frame applies the rotation R(k, omega dt) to x - c, so after n frames
  x_p = c + R(k, n omega dt)(x_p^0 - c) and F = R(k, n omega dt).

The expected rotation comes from scipy's rotation-vector map, an
implementation independent of the oracle's Rodrigues formula; a sign error
(rotating the other way), an axis error or a dropped term of the formula
fails these tests.  Particles sit at unjittered sub-cell centres, and the
selection threshold is zero, so every active node is driven.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2605_09097_amd import scenes


def _block(dim, inv_dx, lo, hi, pad, bc_kind, ppc1d=2, E=5e5, nu=0.35, rho=1000.0):
    """Stress-free block of cells lo..hi-1 (per axis), all particles in scene
    group 0, grid padded by `pad` cells; lattice pitch = dx."""
    dx = 1.0 / inv_dx
    sub = (np.arange(ppc1d) + 0.5) / ppc1d
    axes = [(np.arange(lo[a], hi[a])[:, None] + sub[None, :]).ravel() for a in range(dim)]
    g = np.meshgrid(*axes, indexing="ij")
    x = np.stack([c.ravel() for c in g], axis=1) * dx
    n = len(x)
    vol = np.full(n, dx ** dim / ppc1d ** dim)
    spec = scenes.DomainSpec(
        dim=dim, h0=dx, origin_q=[lo[a] - pad for a in range(dim)] + [0] * (3 - dim), dx_q=1,
        n_nodes=[hi[a] - lo[a] + 2 * pad + 1 for a in range(dim)] + [1] * (3 - dim), x=x, v=np.zeros((n, dim)),
        B=np.zeros((n, dim, dim)), F=np.tile(np.eye(dim), (n, 1, 1)), mass=rho * vol, vol=vol,
        mat=np.zeros(n, np.int32), flags=np.full(n, 2, np.uint8), E=np.array([E]), nu=np.array([nu]),
        bc_kind=[bc_kind], bc_mask=[(1 << dim) - 1], m_ref=float(rho * vol[0]), tau=0.0, ppc1d=ppc1d)
    return spec


def _run(spec, params, dt, frames):
    O = oracle.Domain(spec)
    O.set_bc_params(params)
    so = oracle.solve_opts()
    for _ in range(frames):
        st = O.single_frame(dt, so)
        # every active DOF is prescribed: nothing is left to solve for
        assert st.converged and st.newton_iters == 0 and st.cg_iters == 0
        dr, _ = O.dirichlet(dt)
        active = O.m > 0
        assert dr[active].all()
    return O


@pytest.mark.parametrize("dim", [2, 3])
def test_translate_drive_moves_the_body_rigidly(dim):
    spec = _block(dim, 20, [4] * dim, [10, 8, 7][:dim], 4, oracle.BC_TRANSLATE)
    c = np.array([0.7, -0.4, 0.25][:dim])
    params = np.zeros((1, 8))
    params[0, :dim] = c
    dt, frames = 2e-2, 5
    O = _run(spec, params, dt, frames)
    L = 1.0  # displacement scale: frames * dt * |c| ~ 0.08
    assert np.abs(O.x - (spec.x + frames * dt * c)).max() < 1e-13 * L
    assert np.abs(O.F - np.eye(dim)).max() < 1e-13
    assert np.abs(O.v - c).max() < 1e-12 * np.linalg.norm(c)


@pytest.mark.parametrize("axis", [(0.0, -1.0, 0.0), (1.0, 2.0, -2.0)])
def test_rotate_drive_turns_the_body_rigidly(axis):
    spec = _block(3, 20, [8, 8, 8], [14, 12, 10], 8, oracle.BC_ROTATE)
    k = np.asarray(axis) / np.linalg.norm(axis)
    centre = np.array([0.45, 0.5, 0.42])
    omega, dt, frames = 2.5, 2e-2, 6  # 0.05 rad per frame, 0.3 rad in all
    params = np.zeros((1, 8))
    params[0, :7] = list(centre) + list(k) + [omega]
    O = _run(spec, params, dt, frames)
    R = Rotation.from_rotvec(k * omega * dt * frames).as_matrix()
    x_exact = centre + (spec.x - centre) @ R.T
    span = np.abs(spec.x - centre).max()
    assert np.abs(O.x - x_exact).max() < 1e-12 * span
    assert np.abs(O.F - R).max() < 1e-12
    # the last frame's particle velocity is the chord of one step's rotation
    R1 = Rotation.from_rotvec(k * omega * dt).as_matrix()
    x_prev = centre + (spec.x - centre) @ Rotation.from_rotvec(k * omega * dt * (frames - 1)).as_matrix().T
    v_exact = ((x_prev - centre) @ (R1 - np.eye(3)).T) / dt
    assert np.abs(O.v - v_exact).max() < 1e-10 * omega * span


def test_rotate_drive_turns_counterclockwise_about_its_axis():
    """Right-hand rule: a positive rate about +z carries a point on the +x
    side of the axis towards +y; about -y (the fold's hinge) it lifts a point
    on the +x side towards +z."""
    for axis, lift in (((0.0, 0.0, 1.0), 1), ((0.0, -1.0, 0.0), 2)):
        spec = _block(3, 20, [12, 8, 8], [14, 10, 10], 8, oracle.BC_ROTATE)
        centre = np.array([0.4, 0.45, 0.45])
        params = np.zeros((1, 8))
        params[0, :7] = list(centre) + list(axis) + [1.0]
        O = _run(spec, params, 0.05, 1)
        right = spec.x[:, 0] > centre[0]
        assert right.all()
        assert (O.x[:, lift] - spec.x[:, lift] > 0).all()
        # and by the angle of the rotation, 0.05 rad, at the particles' radius
        r = spec.x[:, 0] - centre[0]
        assert np.allclose(O.x[:, lift] - spec.x[:, lift],
                           r * math.sin(0.05) + (spec.x[:, lift] - centre[lift]) * (math.cos(0.05) - 1.0),
                           rtol=0, atol=1e-13)
