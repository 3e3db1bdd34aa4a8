"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: textbook
identities of the quadratic B-spline, conservation laws of the APIC transfers
(including the angular-momentum statement of the remark on interface
transfer consistency, Sec. 3.4), finite differences of the incremental
potential (Eq. discrete_energy), a library eigen-solver, a library optimiser,
brute-force searches and closed-form special cases.
"""
import numpy as np
import pytest

import oracle
from helpers import rel_err, tiny_domain

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- B-spline
@pytest.mark.parametrize("dim", [2, 3])
def test_bspline_identities(dim):
    """Partition of unity, zero gradient sum, linear reproduction, the
    gradient identity sum x_i grad N_i^T = I and the APIC inertia tensor
    sum N (x_i - x_p)(x_i - x_p)^T = dx^2/4 I of the quadratic B-spline."""
    spec = tiny_domain(dim=dim, n_particles=20, seed=1)
    D = oracle.Domain(spec)
    X = D.node_positions()
    dx = spec.dx
    for p in range(spec.n_particles):
        flat, N, gN = D.weights(spec.x[p])
        xi = X[flat]
        assert abs(N.sum() - 1.0) < 1e-14
        assert np.abs(gN.sum(axis=0)).max() < 1e-12 / dx
        assert np.abs((N[:, None] * xi).sum(axis=0) - spec.x[p]).max() < 1e-14
        assert np.abs(xi.T @ gN - np.eye(dim)).max() < 1e-12
        r = xi - spec.x[p]
        Dp = (N[:, None, None] * r[:, :, None] * r[:, None, :]).sum(axis=0)
        assert np.abs(Dp - dx * dx / 4 * np.eye(dim)).max() < 1e-14


def test_bspline_values_at_cell_centre():
    """At f = 1 (particle on a node) the 1D weights are (1/8, 3/4, 1/8)."""
    spec = tiny_domain(dim=2, n_particles=1, seed=2)
    D = oracle.Domain(spec)
    X = D.node_positions()
    node = 4 + 9 * 4
    flat, N, gN = D.weights(X[node])
    w = np.array([0.125, 0.75, 0.125])
    assert np.allclose(N.reshape(3, 3), np.outer(w, w), atol=1e-15)
    assert flat[4] == node


# ---------------------------------------------------------------- sort
def _brute_cell(x, origin, dx, n):
    """The base node by search: the integer b with b + 1/2 <= xi < b + 3/2."""
    xi = (x - origin) / dx
    for b in range(n - 2):
        if b + 0.5 <= xi < b + 1.5:
            return b
    raise AssertionError("outside")


@pytest.mark.parametrize("tile", [(1, 1), (4, 4), (3, 5), (8, 8)])
def test_sort_matches_stable_brute_force(tile):
    spec = tiny_domain(dim=2, n_cells=12, n_particles=300, seed=3, margin=1)
    # stress ties: duplicate a few particles so keys repeat with order to keep
    spec.x[100:120] = spec.x[0:20]
    D = oracle.Domain(spec)
    perm, cs = D.sort(tile)
    n = spec.n_nodes[0]
    ntx = -(-(n - 2) // tile[0])
    keys = []
    for p in range(spec.n_particles):
        bx = _brute_cell(spec.x[p, 0], 0.0, spec.dx, n)
        by = _brute_cell(spec.x[p, 1], 0.0, spec.dx, n)
        t = (by // tile[1]) * ntx + (bx // tile[0])
        keys.append(t * tile[0] * tile[1] + (by % tile[1]) * tile[0] + (bx % tile[0]))
    expect = sorted(range(spec.n_particles), key=lambda p: keys[p])  # stable
    assert list(perm) == expect
    counts = np.bincount(keys, minlength=len(cs) - 1)
    assert np.array_equal(np.diff(cs), counts)
    assert cs[0] == 0 and cs[-1] == spec.n_particles


# ---------------------------------------------------------------- P2G / G2P
@pytest.mark.parametrize("dim", [2, 3])
def test_p2g_conservation(dim):
    spec = tiny_domain(dim=dim, n_particles=60, seed=4)
    D = oracle.Domain(spec)
    D.p2g()
    m = D.m
    mv = D.vn * m[:, None]
    assert abs(m.sum() - spec.mass.sum()) <= 1e-13 * spec.mass.sum()
    P = (spec.mass[:, None] * spec.v).sum(axis=0)
    assert np.abs(mv.sum(axis=0) - P).max() <= 1e-13 * np.abs(spec.mass[:, None] * spec.v).sum()
    if dim == 2:
        X = D.node_positions()
        Lg = (X[:, 0] * mv[:, 1] - X[:, 1] * mv[:, 0]).sum()
        Lp = (spec.mass * (spec.x[:, 0] * spec.v[:, 1] - spec.x[:, 1] * spec.v[:, 0]
                           + spec.B[:, 1, 0] - spec.B[:, 0, 1])).sum()
        assert abs(Lg - Lp) <= 1e-12 * (abs(Lp) + np.abs(spec.mass[:, None] * spec.v).sum())


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_field_round_trip(dim):
    """Particles carrying v = a + C x and B = C dx^2/4: P2G gives the nodal
    field a + C x_i exactly, G2P returns v_p = a + C x_p, B_p = C dx^2/4 and
    F <- (I + dt C) F, and x advances by dt v_p."""
    rng = np.random.default_rng(5)
    spec = tiny_domain(dim=dim, n_particles=50, seed=5)
    a = rng.normal(size=dim)
    Cm = rng.normal(size=(dim, dim))
    dx = spec.dx
    spec.v = a + spec.x @ Cm.T
    spec.B = np.broadcast_to(Cm * dx * dx / 4, (spec.n_particles, dim, dim)).copy()
    D = oracle.Domain(spec)
    D.p2g()
    X = D.node_positions()
    act = D.m > 0
    assert np.abs(D.vn[act] - (a + X[act] @ Cm.T)).max() < 1e-12
    dt = 1e-3
    D.u[:] = dt * D.vn
    F0 = D.F.copy()
    x0 = D.x.copy()
    D.g2p(dt)
    vp = a + x0 @ Cm.T
    assert np.abs(D.v - vp).max() < 1e-12
    assert np.abs(D.B - Cm * dx * dx / 4).max() < 1e-12
    assert np.abs(D.F - np.einsum("ij,pjk->pik", np.eye(dim) + dt * Cm, F0)).max() < 1e-12
    assert np.abs(D.x - (x0 + dt * vp)).max() < 1e-15


# ---------------------------------------------------------------- Neo-Hookean
def _nh_psi_fd(F, mu, lam, h=1e-6):
    d = F.shape[0]
    P = np.zeros((d, d))
    for a in range(d):
        for b in range(d):
            E = np.zeros((d, d))
            E[a, b] = h
            P[a, b] = (oracle.nh_eval(F + E, mu, lam)[0] - oracle.nh_eval(F - E, mu, lam)[0]) / (2 * h)
    return P


@pytest.mark.parametrize("dim", [2, 3])
def test_neo_hookean_rest_state(dim):
    mu, lam = 3.0, 7.0
    psi, P, A, rc = oracle.nh_eval(np.eye(dim), mu, lam)
    assert rc == 0 and abs(psi) < 1e-15 and np.abs(P).max() < 1e-15
    lin = np.zeros((dim, dim, dim, dim))
    I = np.eye(dim)
    for i in range(dim):
        for j in range(dim):
            for k in range(dim):
                for l in range(dim):
                    lin[i, j, k, l] = mu * (I[i, k] * I[j, l] + I[i, l] * I[j, k]) + lam * I[i, j] * I[k, l]
    assert np.abs(A - lin.reshape(dim * dim, dim * dim)).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_neo_hookean_derivatives_fd(dim):
    rng = np.random.default_rng(6)
    mu, lam = 2.5e3, 6.0e3
    for _ in range(10):
        F = np.eye(dim) + rng.uniform(-0.25, 0.25, size=(dim, dim))
        J = np.linalg.det(F)
        assert 0.5 < J < 1.6
        psi, P, A, rc = oracle.nh_eval(F, mu, lam)
        Pfd = _nh_psi_fd(F, mu, lam)
        assert rel_err(P, Pfd) < 1e-7
        h = 1e-6
        Afd = np.zeros((dim * dim, dim * dim))
        for q in range(dim * dim):
            E = np.zeros(dim * dim)
            E[q] = h
            Pp = oracle.nh_eval(F + E.reshape(dim, dim), mu, lam)[1]
            Pm = oracle.nh_eval(F - E.reshape(dim, dim), mu, lam)[1]
            Afd[:, q] = ((Pp - Pm) / (2 * h)).ravel()
        assert rel_err(A, Afd) < 1e-7
        assert np.abs(A - A.T).max() < 1e-9 * np.abs(A).max()


def test_neo_hookean_inverted():
    psi, P, A, rc = oracle.nh_eval(np.diag([1.0, -0.5]), 1.0, 1.0)
    assert np.isinf(psi) and rc == 5


def test_psd_projection_matches_library_eigensolver():
    rng = np.random.default_rng(7)
    for n in (4, 9):
        for _ in range(5):
            X = rng.normal(size=(n, n))
            A = X + X.T
            w, V = np.linalg.eigh(A)
            expect = (V * np.maximum(w, 0)) @ V.T
            got = oracle.psd_project(A)
            assert np.abs(got - expect).max() < 1e-11 * np.abs(A).max()
    # a PSD matrix is returned untouched
    X = rng.normal(size=(4, 4))
    A = X @ X.T + 0.1 * np.eye(4)
    assert np.array_equal(oracle.psd_project(A), A)


# ---------------------------------------------------------------- energy
def _tiny_solve_domain(dim=2, seed=8, n_particles=30):
    spec = tiny_domain(dim=dim, n_particles=n_particles, seed=seed, F_spread=0.1)
    D = oracle.Domain(spec)
    D.p2g()
    return spec, D


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_is_energy_derivative(dim):
    spec, D = _tiny_solve_domain(dim=dim, n_particles=20 if dim == 3 else 30)
    rng = np.random.default_rng(9)
    dt = 1e-3
    act = D.m > 0
    u = np.where(act[:, None], rng.normal(size=(D.nn, dim)) * 1e-4, 0.0)
    grav = (0.3, -9.8, 0.1)[:dim]
    g = D.gradient(dt, u, grav)
    h = 1e-8
    idx = np.argwhere(act)[:, 0]
    for i in idx[:: max(1, len(idx) // 12)]:
        for a in range(dim):
            e = np.zeros_like(u)
            e[i, a] = h
            fd = (D.energy(dt, u + e, grav) - D.energy(dt, u - e, grav)) / (2 * h)
            assert abs(fd - g[i, a]) <= 1e-6 * (abs(g[i, a]) + 1e-3 * np.abs(g).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_hvp_is_gradient_derivative_and_symmetric(dim):
    spec, D = _tiny_solve_domain(dim=dim, n_particles=20 if dim == 3 else 30)
    rng = np.random.default_rng(10)
    dt = 1e-3
    act = D.m > 0
    u = np.where(act[:, None], rng.normal(size=(D.nn, dim)) * 1e-4, 0.0)
    w = np.where(act[:, None], rng.normal(size=(D.nn, dim)), 0.0)
    z = np.where(act[:, None], rng.normal(size=(D.nn, dim)), 0.0)
    Hw, diag = D.hvp(dt, u, w, project=False)
    h = 1e-7
    fd = (D.gradient(dt, u + h * w) - D.gradient(dt, u - h * w)) / (2 * h)
    assert rel_err(Hw, fd) < 1e-6
    Hz, _ = D.hvp(dt, u, z, project=False)
    assert abs((Hw * z).sum() - (Hz * w).sum()) <= 1e-12 * np.abs(Hw).sum() * np.abs(z).max()
    # the Jacobi diagonal is the diagonal of the assembled operator
    idx = np.argwhere(act)[:, 0][:6]
    for i in idx:
        for a in range(dim):
            e = np.zeros_like(u)
            e[i, a] = 1.0
            He, _ = D.hvp(dt, u, e, project=False)
            assert abs(He[i, a] - diag[i, a]) <= 1e-12 * abs(diag[i, a])


def test_projected_hvp_is_psd_and_equal_when_convex():
    spec, D = _tiny_solve_domain(dim=2, n_particles=30)
    rng = np.random.default_rng(11)
    dt = 1e-3
    act = D.m > 0
    u = np.where(act[:, None], rng.normal(size=(D.nn, 2)) * 1e-4, 0.0)
    for _ in range(5):
        w = np.where(act[:, None], rng.normal(size=(D.nn, 2)), 0.0)
        Hw, _ = D.hvp(dt, u, w, project=True)
        assert (Hw * w).sum() > 0
    # at F = I every particle block is the PSD linear-elastic tensor
    spec2 = tiny_domain(dim=2, n_particles=30, seed=12, F_spread=0.0)
    D2 = oracle.Domain(spec2)
    D2.p2g()
    w = np.where((D2.m > 0)[:, None], rng.normal(size=(D2.nn, 2)), 0.0)
    zero = np.zeros((D2.nn, 2))
    a, _ = D2.hvp(dt, zero, w, project=True)
    b, _ = D2.hvp(dt, zero, w, project=False)
    assert rel_err(a, b) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_delta_energy_equals_energy_difference(dim):
    spec, D = _tiny_solve_domain(dim=dim, n_particles=20 if dim == 3 else 30)
    rng = np.random.default_rng(13)
    dt = 1e-3
    act = D.m > 0
    u = np.where(act[:, None], rng.normal(size=(D.nn, dim)) * 1e-4, 0.0)
    du = np.where(act[:, None], rng.normal(size=(D.nn, dim)) * 1e-4, 0.0)
    grav = (0.0, -9.8, 0.0)[:dim]
    for alpha in (1.0, 0.5, 0.125):
        direct = D.energy(dt, u + alpha * du, grav) - D.energy(dt, u, grav)
        got = D.delta_energy(dt, u, du, alpha, grav)
        assert abs(got - direct) <= 1e-9 * abs(direct)
    # a step that inverts a particle is +inf
    big = np.where(act[:, None], rng.normal(size=(D.nn, dim)) * 10.0, 0.0)
    assert np.isinf(D.delta_energy(dt, u, big, 1.0, grav))


# ---------------------------------------------------------------- Newton
def test_newton_zero_stiffness_closed_form():
    """With mu = lam = 0 the minimiser is u = dt v^n + dt^2 g on every node."""
    spec = tiny_domain(dim=2, n_particles=40, seed=14, E=(0.0,), nu=(0.3,))
    D = oracle.Domain(spec)
    D.p2g()
    dt = 1e-2
    st = D.solve(dt, oracle.solve_opts(gravity=(0.0, -9.8)))
    act = D.m > 0
    expect = dt * D.vn + dt * dt * np.array([0.0, -9.8])
    assert st.converged
    assert np.abs(D.u[act] - expect[act]).max() < 1e-14


def test_newton_matches_library_minimiser():
    """The Newton-PCG-line-search minimiser of E over the free DOFs agrees with
    scipy's trust-region Newton-CG given the same energy and gradient."""
    from scipy.optimize import minimize

    spec = tiny_domain(dim=2, n_particles=40, seed=15, F_spread=0.05, v_scale=0.5,
                       flags=None, bc_kind=[0], bc_mask=[0b11])
    spec.flags[:5] = 2  # first five particles form a clamped group
    D = oracle.Domain(spec)
    D.p2g()
    dt = 2e-3
    grav = (0.0, -9.8)
    st = D.solve(dt, oracle.solve_opts(newton_rtol=1e-10, cg_rtol=1e-12, gravity=grav))
    assert st.converged
    u_newton = D.u.copy()
    dr, ud = D.dirichlet(dt)
    free = ((D.m > 0)[:, None] & (dr == 0))
    base = np.where(dr == 1, ud, 0.0)

    def f(z):
        u = base.copy()
        u[free] = z
        return D.energy(dt, u, grav)

    def g(z):
        u = base.copy()
        u[free] = z
        return D.gradient(dt, u, grav)[free]

    def hp(z, p):
        u = base.copy()
        u[free] = z
        w = np.zeros_like(u)
        w[free] = p
        return D.hvp(dt, u, w, project=False)[0][free]

    z0 = (dt * D.vn)[free]
    res = minimize(f, z0, jac=g, hessp=hp, method="trust-ncg", options={"gtol": 1e-12})
    assert rel_err(u_newton[free], res.x) < 1e-7


# ---------------------------------------------------------------- interface
def test_boundary_set_and_arbitration_toy():
    """Hand-worked toy.  Coarse grid dx = 4 h0, fine grid dx = 2 h0 starting at
    lattice point 8; every coarse node at an even lattice point inside the fine
    grid coincides with a fine node.  One coarse boundary particle and one fine
    boundary particle are placed so that exactly one coincident node is in both
    boundary sets; its donor is decided by the node masses."""
    h0 = 0.01
    Bs = tiny_domain(dim=2, n_cells=10, n_particles=1, seed=16, dx_q=4, h0=h0, m_ref=1.0)
    Ss = tiny_domain(dim=2, n_cells=12, n_particles=1, seed=17, dx_q=2, h0=h0, origin_q=[8, 8],
                     m_ref=1.0)
    # coarse particle exactly on coarse node (4, 4) = lattice (16, 16): stencil nodes 3..5
    Bs.x[0] = [0.16, 0.16]
    Bs.mass[0] = 1.0
    Bs.flags[0] = 1
    # fine particle on fine node (4, 4) = lattice (16, 16): stencil fine nodes 3..5 = lattice 14..18
    Ss.x[0] = [0.16, 0.16]
    Ss.flags[0] = 1
    for heavy_fine in (False, True):
        Ss.mass[0] = 2.0 if heavy_fine else 0.5
        Bs.tau = Ss.tau = 0.001
        Bd, Sd = oracle.Domain(Bs), oracle.Domain(Ss)
        Bd.p2g()
        Sd.p2g()
        n_amb = oracle.interface(Bd, Sd)
        # boundary sets: the 3x3 stencils (smallest N m = 0.5/64 > tau)
        assert Bd.gamma.sum() == 9 and Sd.gamma.sum() == 9
        # coincident lattice points of both sets: coarse lattice {12,16,20} vs fine {14,16,18}
        # -> only lattice (16,16)
        assert n_amb == 1
        I = 4 + 11 * 4
        j = 4 + 13 * 4
        assert Bd.gamma[I] and Sd.gamma[j]
        # node masses: coarse 1.0 * 9/16, fine m * 9/16
        if heavy_fine:
            assert Bd.recv[I] == 1 and Sd.recv[j] == 0
        else:
            assert Bd.recv[I] == 0 and Sd.recv[j] == 1
        assert Bd.recv.sum() == 9 - (0 if heavy_fine else 1)
        assert Sd.recv.sum() == 9 - (1 if heavy_fine else 0)
    # tie -> coarse side donates
    Ss.mass[0] = 1.0
    Bd, Sd = oracle.Domain(Bs), oracle.Domain(Ss)
    Bd.p2g()
    Sd.p2g()
    oracle.interface(Bd, Sd)
    assert Bd.recv[4 + 11 * 4] == 0 and Sd.recv[4 + 13 * 4] == 1


def test_boundary_set_brute_force():
    rng = np.random.default_rng(18)
    spec = tiny_domain(dim=2, n_cells=10, n_particles=80, seed=18)
    spec.flags[:] = (rng.random(80) < 0.4).astype(np.uint8)
    spec.tau = 0.05 * spec.mass.mean()
    D = oracle.Domain(spec)
    D.p2g()
    Bd2 = oracle.Domain(spec)  # a second domain far away so nothing coincides
    oracle.interface(D, Bd2) if False else None
    S = oracle.Domain(tiny_domain(dim=2, n_cells=10, n_particles=1, seed=19, origin_q=[1000, 1000]))
    S.p2g()
    S._s.m_ref = D._s.m_ref
    oracle.interface(D, S)
    scale = 2.0 ** 32 / spec.m_ref
    q = np.zeros(D.nn, np.int64)
    for p in range(80):
        if spec.flags[p] & 1:
            flat, N, _ = D.weights(spec.x[p])
            q[flat] += np.rint(N * (spec.mass[p] * scale)).astype(np.int64)
    expect = (q > np.rint(spec.tau * scale)) & (D.m > 0)
    assert np.array_equal(D.gamma.astype(bool), expect)


def test_projection_and_interpolation_identities():
    """Pi of a constant fine field is that constant on every coarse receiver
    with support (eps_tol = 0); I of an affine coarse field is exact; T_m
    returns its endpoints at m = 0 and m = M and is linear in between."""
    sc_B = tiny_domain(dim=2, n_cells=14, n_particles=150, seed=20, dx_q=4, h0=0.01, m_ref=1.0,
                       margin=2)
    sc_S = tiny_domain(dim=2, n_cells=16, n_particles=200, seed=21, dx_q=2, h0=0.01,
                       origin_q=[8, 8], m_ref=1.0, margin=2)
    sc_B.flags[:] = 1
    sc_S.flags[:] = 1
    sc_B.tau = sc_S.tau = 0.0
    Bd, Sd = oracle.Domain(sc_B), oracle.Domain(sc_S)
    Bd.p2g()
    Sd.p2g()
    oracle.interface(Bd, Sd)
    c = np.array([0.7, -0.3])
    vS = np.broadcast_to(c, (Sd.nn, 2)).copy()
    out = oracle.project(Sd, Bd, 0.0, vS)
    # receivers whose coarse support holds fine mass get exactly c
    num_support = oracle.project(Sd, Bd, 0.0, np.ones((Sd.nn, 2)))
    has = (Bd.recv == 1) & (np.abs(num_support[:, 0] - 1.0) < 1e-12)
    assert has.sum() > 0
    assert np.abs(out[has] - c).max() < 1e-14
    # I of an affine coarse field
    a = np.array([0.1, 0.2])
    Cm = np.array([[0.3, -0.4], [0.5, 0.7]])
    XB = Bd.node_positions()
    vB = np.where((Bd.m > 0)[:, None], a + XB @ Cm.T, 0.0)
    got = oracle.interp(Bd, vB, Sd)
    XS = Sd.node_positions()
    # fine receivers whose whole coarse stencil is active
    ok = []
    for j in np.argwhere(Sd.recv == 1)[:, 0]:
        flat, N, _ = Bd.weights(XS[j])
        if np.all(Bd.m[flat] > 0):
            ok.append(j)
    assert len(ok) > 0
    assert np.abs(got[ok] - (a + XS[ok] @ Cm.T)).max() < 1e-13
    vn, vn1 = np.random.default_rng(0).normal(size=(2, 50))
    assert np.array_equal(oracle.temporal(0, 4, vn, vn1), vn)
    assert np.allclose(oracle.temporal(4, 4, vn, vn1), vn1, atol=0, rtol=0)
    assert np.allclose(oracle.temporal(1, 4, vn, vn1), 0.75 * vn + 0.25 * vn1, rtol=1e-15)
