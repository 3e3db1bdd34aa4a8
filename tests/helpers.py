"""Small seeded inputs shared by the oracle pins and the GPU parity tests."""
import numpy as np

from paper_2605_09097_amd.scenes import DomainSpec


def tiny_domain(dim=2, n_cells=8, n_particles=40, seed=0, dx_q=4, h0=0.025 / 4, origin_q=None,
                E=(1e4, 3e4), nu=(0.3, 0.35), rho=1000.0, F_spread=0.15, v_scale=0.2,
                B_scale=0.5, margin=2, flags=None, bc_kind=(), bc_mask=(), tau_rel=1e-3,
                m_ref=None):
    """A grid of n_cells per axis and random particles kept `margin` cells away
    from the grid edge, random velocities, affine matrices and deformation
    gradients with det F in roughly [0.7, 1.3]."""
    rng = np.random.default_rng(seed)
    n_nodes = [n_cells + 1] * dim
    origin_q = list(origin_q) if origin_q is not None else [0] * dim
    dx = dx_q * h0
    lo = np.array([origin_q[a] * h0 for a in range(dim)]) + margin * dx
    hi = lo + (n_cells - 2 * margin) * dx
    x = lo + rng.random((n_particles, dim)) * (hi - lo)
    v = rng.normal(size=(n_particles, dim)) * v_scale
    B = rng.normal(size=(n_particles, dim, dim)) * B_scale * dx
    F = np.eye(dim) + rng.uniform(-F_spread, F_spread, size=(n_particles, dim, dim))
    vol = np.full(n_particles, dx ** dim / 4)
    mass = rho * vol * (1.0 + 0.2 * rng.random(n_particles))
    mat = rng.integers(0, len(E), n_particles).astype(np.int32)
    if flags is None:
        flags = np.zeros(n_particles, np.uint8)
    m_ref = m_ref if m_ref is not None else rho * dx ** dim / 4
    return DomainSpec(dim=dim, h0=h0, origin_q=origin_q, dx_q=dx_q, n_nodes=n_nodes, x=x, v=v, B=B,
                      F=F, mass=mass, vol=vol, mat=mat, flags=np.asarray(flags, np.uint8),
                      E=np.asarray(E, float), nu=np.asarray(nu, float), bc_kind=list(bc_kind),
                      bc_mask=list(bc_mask), m_ref=m_ref, tau=tau_rel * float(mass.mean()))


def rel_err(a, b):
    """Relative error of a against the reference b: the larger of the 2-norm
    ratio |a - b|_2 / |b|_2 and the max-norm ratio |a - b|_inf / |b|_inf, so
    that an error confined to a few entries is not diluted over the rest."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    if a.size == 0 and b.size == 0:
        return 0.0
    e2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    einf = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    return float(max(e2, einf))
