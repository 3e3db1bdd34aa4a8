"""Edge cases of the HIP path against the FP64 oracle.

* An empty domain: P2G, the implicit solve and G2P succeed with an empty
  grid (the Newton test passes at iteration 0: the gradient and its scale
  are both zero), and the same domain then takes particles again.
* One particle, and 600 particles sharing one stencil base node (a single
  non-empty bin and tile, so the per-tile particle loops run many passes).
* A coupled frame whose domains carry no Schwarz-boundary particles: the
  boundary and receiver sets are empty, the residuals are 0, the iteration
  stops after its first pass and each domain runs on its own.
* A fine grid not covered by the coarse grid's stencils: out-of-grid on
  both sides.
* A grid of more than 1024 blocks of 256 nodes with scattered particle
  clusters: the active-node list is then built from a scan of the per-block
  counts instead of per-block sums (the solve runs over that list).  On
  small tiles the same grid makes the split-mode CG reduction run on
  several workgroups.
* Argument limits: capacity above 2^28 particles, more particles than the
  capacity, a grid of more than 2^28 nodes, a grid whose whole tiles hold
  more than 2^28 bins (each refused before anything is allocated).

Bars as in the other parity tests: bit-exact for integers, 1e-10 (FP64) and
1e-5 (mixed) relative for real outputs.
"""
import warnings

import numpy as np
import pytest

import oracle
from helpers import rel_err, tiny_domain

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09097_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


def _b():
    from paper_2605_09097_amd import binding

    return binding


def _prec(b, name):
    return b.OSMPM_FP64 if name == "fp64" else b.OSMPM_MIXED


def _solve_opts(b, name, grav):
    return b.solve_opts(gravity=grav, cg_rtol=1e-10 if name == "fp64" else 1e-5)


def _step_parity(ctx, D, spec, name, dt=2e-3):
    """P2G, implicit solve and G2P on D against the oracle from spec."""
    b = _b()
    dim = spec.dim
    grav = (0.0, -9.8, 0.0)[:dim]
    D.p2g()
    st = D.implicit_solve(dt, _solve_opts(b, name, grav))
    m, vn, u = D.grid_state()
    _, _, q = D.sets()
    ctx.sync()
    O = oracle.Domain(spec)
    O.p2g()
    ost = O.solve(dt, oracle.solve_opts(gravity=grav))
    assert np.array_equal(q.cpu().numpy(), O.q_all)
    assert st.converged == ost.converged == 1
    if name == "fp64":
        assert st.newton_iters == ost.newton_iters
    assert rel_err(u.cpu().numpy(), O.u) < TOL[name]
    D.g2p(dt)
    O.g2p(dt)
    x, v, Bm, F = D.particles_input_order()
    assert rel_err(x - spec.x, O.x - spec.x) < TOL[name]
    assert rel_err(v, O.v) < TOL[name]
    assert rel_err(F - np.eye(dim), O.F - np.eye(dim)) < TOL[name]


@pytest.mark.parametrize("name", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_empty_domain_then_refilled(ctx, dim, name):
    b = _b()
    cells = 8 if dim == 2 else 6
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)  # the mean mass of no particles
        empty = tiny_domain(dim=dim, n_cells=cells, n_particles=0, seed=40)
    empty.tau = 0.0
    empty.m_ref = 1.0
    D = b.Domain(ctx, empty, _prec(b, name), capacity=300)
    D.p2g()
    st = D.implicit_solve(1e-3, _solve_opts(b, name, (0.0, -9.8, 0.0)[:dim]))
    D.g2p(1e-3)
    m, vn, u = D.grid_state()
    ctx.sync()
    assert st.converged == 1 and st.newton_iters == 0
    assert not m.cpu().numpy().any() and not u.cpu().numpy().any()
    full = tiny_domain(dim=dim, n_cells=cells, n_particles=250, seed=41, F_spread=0.08)
    full.m_ref = 1.0
    D.set_particles(full)
    _step_parity(ctx, D, full, name)
    D.close()


@pytest.mark.parametrize("name", ["fp64", "mixed"])
def test_single_particle(ctx, name):
    b = _b()
    spec = tiny_domain(dim=2, n_cells=8, n_particles=1, seed=42, F_spread=0.08)
    D = b.Domain(ctx, spec, _prec(b, name))
    _step_parity(ctx, D, spec, name)
    D.close()


@pytest.mark.parametrize("name", ["fp64", "mixed"])
def test_all_particles_on_one_base_node(ctx, name):
    b = _b()
    spec = tiny_domain(dim=2, n_cells=12, n_particles=600, seed=43, F_spread=0.05, v_scale=0.05)
    rng = np.random.default_rng(43)
    # base node floor(x / dx - 1/2) = 5 on both axes
    spec.x[:] = (5.5 + 0.999 * rng.random(spec.x.shape)) * spec.dx
    D = b.Domain(ctx, spec, _prec(b, name), tile=(4, 4))
    D.p2g()
    perm, cs = D.sort_result()
    ctx.sync()
    operm, ocs = oracle.Domain(spec).sort((4, 4))
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    assert np.count_nonzero(np.diff(ocs)) == 1  # one non-empty bin
    _step_parity(ctx, D, spec, name)
    D.close()


def _sparse_clusters(dim, cells, seed=49):
    """twelve clusters of 40 particles spread over a grid of `cells` cells
    per axis, so that the active nodes lie in a few scattered blocks"""
    spec = tiny_domain(dim=dim, n_cells=cells, n_particles=480, seed=seed, F_spread=0.08, v_scale=0.1)
    rng = np.random.default_rng(seed)
    centres = (3.0 + (cells - 6) * rng.random((12, dim))) * spec.dx
    spec.x[:] = np.repeat(centres, 40, axis=0) + rng.uniform(-1.5, 1.5, (480, dim)) * spec.dx
    return spec


@pytest.mark.parametrize("name", ["fp64", "mixed"])
@pytest.mark.parametrize("dim,cells", [(2, 600), (3, 70)])
def test_large_sparse_grid(ctx, dim, cells, name):
    """361,201 (2D) or 357,911 (3D) nodes, more than 1024 node blocks, with
    scattered particle clusters."""
    b = _b()
    spec = _sparse_clusters(dim, cells)
    assert ((cells + 1) ** dim + 255) // 256 > 1024
    D = b.Domain(ctx, spec, _prec(b, name))
    _step_parity(ctx, D, spec, name)
    D.close()


@pytest.mark.parametrize("name", ["fp64", "mixed"])
def test_cg_scalars_from_several_workgroups(ctx, name):
    """CG scalars formed in their own launch (split mode) by several
    workgroups per domain: on 4 x 4 tiles the 600 x 600-cell grid has 22,500
    tile slots, so the reduction launch takes five workgroups, each adding a
    share of the partial sums, the last to finish adding theirs.  Against the
    oracle, and against the fused form (same Newton and CG counts, solution
    equal to rounding)."""
    b = _b()
    spec = _sparse_clusters(2, 600, seed=50)
    out = {}
    try:
        for mode in (1, 0):
            ctx.cg_split(mode)
            D = b.Domain(ctx, spec, _prec(b, name), tile=(4, 4))
            if mode == 1:
                _step_parity(ctx, D, spec, name)
                D.close()
                D = b.Domain(ctx, spec, _prec(b, name), tile=(4, 4))
            D.p2g()
            st = D.implicit_solve(2e-3, _solve_opts(b, name, (0.0, -9.8)))
            out[mode] = ((st.newton_iters, st.cg_iters), D.grid_state()[2].cpu().numpy().copy())
            D.close()
    finally:
        ctx.cg_split(-1)
    assert out[1][0] == out[0][0]
    assert rel_err(out[1][1], out[0][1]) < 1e-12


def test_large_sparse_grid_cycle_graphs(ctx):
    """Solves on a grid above the size at which a solve sizes its tangent and
    CG launches to the working workgroups (4913 tiles of 4^3 cells), as cycle
    graphs keyed by those sizes: two steps with graphs (the second replays
    the cached cycles) give the eager steps' counts and solutions (FP64; the
    grid's atomic sums vary in order either way)."""
    b = _b()
    spec = _sparse_clusters(3, 70, seed=51)
    res = {}
    try:
        for graphs in (1, 0):
            ctx.graphs(graphs)
            D = b.Domain(ctx, spec, b.OSMPM_FP64)
            out = []
            for _ in range(2):
                D.p2g()
                st = D.implicit_solve(2e-3, _solve_opts(b, "fp64", (0.0, -9.8, 0.0)))
                D.g2p(2e-3)
                out.append(((st.newton_iters, st.cg_iters), D.grid_state()[2].cpu().numpy().copy()))
            D.close()
            res[graphs] = out
    finally:
        ctx.graphs(0)
    for g, e in zip(res[1], res[0]):
        assert g[0] == e[0]
        assert rel_err(g[1], e[1]) < 1e-12


def _uncoupled_pair(cover):
    """Coarse dx = 0.025 and fine dx = 0.0125 domains with no Schwarz-boundary
    particles.  cover=True: the coarse grid [0, 0.3]^2 holds the 3^2 stencil
    of every node of the fine grid [0.05, 0.25]^2; cover=False: both grids
    span [0, 0.2]^2, so fine nodes near the edge have coarse stencils that
    leave the coarse grid."""
    h0 = 0.025 / 4
    Bs = tiny_domain(dim=2, n_cells=12 if cover else 8, dx_q=4, h0=h0, n_particles=200, seed=44,
                     F_spread=0.05)
    Ss = tiny_domain(dim=2, n_cells=16, dx_q=2, h0=h0, origin_q=[8, 8] if cover else [0, 0],
                     n_particles=300, seed=45, F_spread=0.05)
    Ss.m_ref = Bs.m_ref
    return Bs, Ss


@pytest.mark.parametrize("name", ["fp64", "mixed"])
def test_schwarz_frame_without_receivers(ctx, name):
    b = _b()
    from paper_2605_09097_amd import scenes

    Bs, Ss = _uncoupled_pair(cover=True)
    zero = np.zeros((1, 8))
    sc = scenes.Scene(name="no_receivers", B=Bs, S=Ss, dT=2e-3, M=2, n_frames=2,
                      bc_params=lambda f: (zero, zero))
    pair = b.SchwarzPair(ctx, sc, precision=_prec(b, name))
    solve = b.solve_opts(cg_rtol=1e-10 if name == "fp64" else 1e-5)
    go = b.schwarz_opts(sc.M, coarse=solve, fine=solve)
    OB, OS = oracle.Domain(Bs), oracle.Domain(Ss)
    oo = oracle.schwarz_opts(sc.M)
    for _ in range(2):
        st = pair.frame(go)
        ost = oracle.schwarz_frame(OB, OS, sc.dT, oo)
        assert (st.iters, st.converged) == (ost.iters, ost.converged) == (1, 1)
        assert (st.n_recv_B, st.n_recv_S, st.n_amb) == (ost.n_recv_B, ost.n_recv_S, ost.n_amb) == (0, 0, 0)
        assert st.r_B == 0.0 and st.r_S == 0.0
    for Dg, Do, spec in ((pair.B, OB, Bs), (pair.S, OS, Ss)):
        m, vn, u = Dg.grid_state()
        x, v, Bm, F = Dg.particles_input_order()
        assert rel_err(u.cpu().numpy(), Do.u) < TOL[name]
        assert rel_err(x - spec.x, Do.x - spec.x) < TOL[name]
        assert rel_err(F - np.eye(2), Do.F - np.eye(2)) < TOL[name]
    pair.close()


def test_schwarz_frame_fine_grid_outside_coarse_grid(ctx):
    """A fine grid whose edge nodes have no coarse stencil: the oracle and the
    library both report out-of-grid (status 4).  Device-detected errors are
    sticky per context, so the test uses a context of its own (the shared
    one only gates the test on a GPU being present)."""
    b = _b()
    Bs, Ss = _uncoupled_pair(cover=False)
    with pytest.raises(RuntimeError, match="status 4"):
        oracle.schwarz_frame(oracle.Domain(Bs), oracle.Domain(Ss), 2e-3, oracle.schwarz_opts(2))
    own = b.Context(0)
    B, S = b.Domain(own, Bs), b.Domain(own, Ss)
    with pytest.raises(b.OsmpmError) as e:
        b.schwarz_frame(B, S, 2e-3, b.schwarz_opts(2))
        own.sync()
    assert e.value.status == b.OSMPM_E_OUT_OF_GRID
    B.close()
    S.close()
    own.close()


def test_argument_limits(ctx):
    b = _b()
    spec = tiny_domain(dim=2, n_cells=8, n_particles=10, seed=46)
    with pytest.raises(b.OsmpmError) as e:
        b.Domain(ctx, spec, capacity=(1 << 28) + 1)
    assert e.value.status == b.OSMPM_E_INVALID_ARG
    with pytest.raises(b.OsmpmError) as e:
        b.Domain(ctx, spec, capacity=5)  # 10 particles
    assert e.value.status == b.OSMPM_E_INVALID_ARG
    huge = tiny_domain(dim=3, n_cells=8, n_particles=10, seed=47)
    huge.n_nodes = [1 << 10, 1 << 10, 1 << 9]  # 2^29 nodes
    with pytest.raises(b.OsmpmError) as e:
        b.Domain(ctx, huge)
    assert e.value.status == b.OSMPM_E_INVALID_ARG
    padded = tiny_domain(dim=2, n_cells=8, n_particles=10, seed=47)
    padded.n_nodes = [3, 1 << 26, 1]  # 3 * 2^26 nodes, 64 * (2^26 - 2) bins in 64 x 1 tiles
    with pytest.raises(b.OsmpmError) as e:
        b.Domain(ctx, padded, tile=(64, 1))
    assert e.value.status == b.OSMPM_E_INVALID_ARG


def test_g2p_requires_a_solve_of_the_current_grid(ctx):
    """G2P reads the displacement of the implicit solve of the current grid:
    after a P2G with no solve it is refused (status 7), and accepted again
    once the grid has been solved."""
    b = _b()
    spec = tiny_domain(dim=2, n_cells=8, n_particles=40, seed=48, F_spread=0.05)
    D = b.Domain(ctx, spec)
    D.p2g()
    with pytest.raises(b.OsmpmError) as e:
        D.g2p(1e-3)
    assert e.value.status == b.OSMPM_E_STATE
    D.implicit_solve(1e-3, b.solve_opts())
    D.g2p(1e-3)
    D.p2g()
    with pytest.raises(b.OsmpmError) as e:
        D.g2p(1e-3)
    assert e.value.status == b.OSMPM_E_STATE
    ctx.sync()
    D.close()
