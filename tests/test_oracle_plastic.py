"""Pins of the oracle's elastoplastic extension (von Mises in Hencky strain,
applied after G2P's deformation-gradient update; the paper names
elastoplastic hinges as future work, Sec. 4.4 and Sec. 5).

The projection is checked against what defines it, not against its own
formula: below the yield surface nothing changes; above it the result lies
on the surface, keeps det F, the polar rotation and the principal
directions, is idempotent, and equals the closest point of the von Mises
set in logarithmic principal strain found by a general constrained
minimiser (scipy SLSQP) from the singular values of F (numpy SVD).  In a
frame, the plastic run equals the elastic run followed by the projection of
every particle's F (the solve sees only the start-of-frame F), and the
reverse mode refuses plastic domains."""
import numpy as np
import pytest

import oracle

MU = 4.0e4


def _rand_F(rng, d, amp):
    F = np.eye(d) + amp * rng.standard_normal((d, d))
    if np.linalg.det(F) <= 0.1:
        F = np.eye(d) + 0.3 * amp * rng.standard_normal((d, d))
    return F


def _hencky(F):
    s = np.linalg.svd(F, compute_uv=False)
    return np.sort(np.log(s))


def _dev_norm(eps):
    return np.linalg.norm(eps - eps.mean())


@pytest.mark.parametrize("d", [2, 3])
def test_below_yield_is_untouched(d):
    rng = np.random.default_rng(1 + d)
    for _ in range(50):
        F = _rand_F(rng, d, 0.02)
        k = _dev_norm(_hencky(F))
        tau = 2.0 * MU * k * 1.05
        Fn, changed = oracle.vm_return(F, MU, tau)
        assert not changed and np.array_equal(Fn, F)
    F = _rand_F(rng, d, 0.3)
    for tau in (0.0, -1.0, np.inf):
        Fn, changed = oracle.vm_return(F, MU, tau)
        assert not changed and np.array_equal(Fn, F)


@pytest.mark.parametrize("d", [2, 3])
def test_projection_invariants(d):
    rng = np.random.default_rng(10 + d)
    n_changed = 0
    for _ in range(200):
        F = _rand_F(rng, d, 0.25)
        ky = 0.5 * _dev_norm(_hencky(F)) * rng.uniform(0.1, 0.9)
        tau = 2.0 * MU * ky
        Fn, changed = oracle.vm_return(F, MU, tau)
        assert changed
        n_changed += 1
        eps_n = _hencky(Fn)
        # on the yield surface, volume kept
        assert abs(_dev_norm(eps_n) - ky) <= 1e-10 * max(ky, 1e-12)
        assert abs(np.linalg.det(Fn) - np.linalg.det(F)) <= 1e-12 * abs(np.linalg.det(F))
        # same polar rotation, same principal directions of C = F^T F
        U, _, Vt = np.linalg.svd(F)
        Un, _, Vtn = np.linalg.svd(Fn)
        R, Rn = U @ Vt, Un @ Vtn
        assert np.abs(R - Rn).max() <= 1e-10
        C, Cn = F.T @ F, Fn.T @ Fn
        assert np.abs(C @ Cn - Cn @ C).max() <= 1e-10 * np.abs(C).max() ** 2
        # idempotent
        Fnn, changed2 = oracle.vm_return(Fn, MU, tau * (1.0 + 1e-9))
        assert not changed2 and np.array_equal(Fnn, Fn)
    assert n_changed == 200


@pytest.mark.parametrize("d", [2, 3])
def test_closest_point_against_a_general_minimiser(d):
    """The projected log-stretches are the point of the set {|dev e| <= k,
    tr e = tr eps} closest to eps, found independently by SLSQP."""
    opt = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(20 + d)
    for _ in range(20):
        F = _rand_F(rng, d, 0.3)
        eps = _hencky(F)
        ky = _dev_norm(eps) * rng.uniform(0.2, 0.8)
        Fn, _ = oracle.vm_return(F, MU, 2.0 * MU * ky)
        cons = [{"type": "eq", "fun": lambda e: np.sum(e) - np.sum(eps)},
                {"type": "ineq", "fun": lambda e: ky ** 2 - np.sum((e - e.mean()) ** 2)}]
        obj = lambda e: np.sum((e - eps) ** 2)
        r = opt.minimize(obj, eps.mean() + 0.0 * eps, constraints=cons, method="SLSQP",
                         options={"ftol": 1e-13, "maxiter": 500})
        e_or = _hencky(Fn)
        # the oracle's point is feasible, no worse than the minimiser's, and
        # the same point
        assert abs(np.sum(e_or) - np.sum(eps)) <= 1e-12 and _dev_norm(e_or) <= ky * (1 + 1e-10)
        assert obj(e_or) <= obj(r.x) * (1 + 1e-8) + 1e-12  # the minimiser stops just outside the set
        assert np.abs(np.sort(r.x) - e_or).max() <= 1e-5 * max(1.0, np.abs(eps).max())


def _plastic_scene():
    from paper_2605_09097_amd import scenes

    # the inclusion's misfit strains the matrix near the interface past a
    # low yield stress
    return scenes.inclusion_single(inv_dx=20, n_frames=3, delta=0.05, loaded=False)


def test_frame_equals_elastic_frame_then_projection():
    sc = _plastic_scene()
    so = oracle.solve_opts(newton_rtol=1e-12, newton_atol=1e-16, cg_rtol=1e-13, max_newton=60, max_cg=20000)
    De, Dp = oracle.Domain(sc.B), oracle.Domain(sc.B)
    p, _ = sc.bc_params(0)
    De.set_bc_params(p)
    Dp.set_bc_params(p)
    mu = De.mu
    tau = np.full(len(mu), 0.0)
    tau[0] = 2.0 * mu[0] * 2e-4  # the matrix near the inclusion yields, the inclusion stays elastic
    Dp.set_yield(tau)
    De.single_frame(sc.dT, so)
    Dp.single_frame(sc.dT, so)
    for k in ("x", "v", "B"):
        assert np.array_equal(getattr(De, k), getattr(Dp, k)), k
    n_yield = 0
    for q in range(len(De.F)):
        Fq, changed = oracle.vm_return(De.F[q], mu[De.mat[q]], tau[De.mat[q]])
        n_yield += changed
        assert np.array_equal(Fq, Dp.F[q])
        if De.mat[q] == 0:
            assert _dev_norm(_hencky(Dp.F[q])) <= 0.004 * (1 + 1e-10)
    assert 0 < n_yield < len(De.F)


def test_reverse_mode_refuses_plastic_domains():
    sc = _plastic_scene()
    D = oracle.Domain(sc.B)
    D.set_yield(np.full(len(D.mu), 2.0 * D.mu[0] * 0.004))
    so = oracle.solve_opts()
    W = {k: np.zeros_like(v) for k, v in D.state().items()}
    with pytest.raises(Exception):
        oracle.single_frame_adjoint(D, sc.dT, so, W)
    D.set_yield(None)
    oracle.single_frame_adjoint(D, sc.dT, so, W)
