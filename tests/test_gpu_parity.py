"""GPU (gfx950) parity of the HIP path against the FP64 CPU oracle.

Every test calls the library through its C ABI (paper_2605_09097_amd.binding)
and the oracle on the same seeded inputs.  Bars: bit-exact for the sort
permutation, bin offsets, fixed-point node masses, boundary and receiver
sets; 1e-10 relative (2-norm) for FP64 grid displacements and particle
state (the FP64 parity target of the method's hot path).
"""
import numpy as np
import pytest

import oracle
from helpers import rel_err, tiny_domain

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09097_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


def _binding():
    from paper_2605_09097_amd import binding

    return binding


def _scenes():
    from paper_2605_09097_amd import scenes

    return scenes


# ---------------------------------------------------------------- sort
@pytest.mark.parametrize("tile", [(8, 8), (4, 4), (3, 5)])
def test_sort_bit_exact(ctx, tile):
    b = _binding()
    spec = tiny_domain(dim=2, n_cells=24, n_particles=3000, seed=31, margin=1)
    spec.x[1000:1200] = spec.x[0:200]  # repeated keys: stability matters
    D = b.Domain(ctx, spec, tile=tile)
    D.p2g()
    perm, cs = D.sort_result()
    ctx.sync()
    O = oracle.Domain(spec)
    operm, ocs = O.sort(tile)
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    D.close()


def test_sort_bit_exact_3d(ctx):
    b = _binding()
    spec = tiny_domain(dim=3, n_cells=12, n_particles=4000, seed=32, margin=1)
    spec.x[100:300] = spec.x[0:200]
    D = b.Domain(ctx, spec, tile=(4, 4, 4))
    D.p2g()
    perm, cs = D.sort_result()
    ctx.sync()
    operm, ocs = oracle.Domain(spec).sort((4, 4, 4))
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    D.close()


@pytest.mark.parametrize("name", ["inclusion_tiny", "inclusion_refined"])
def test_sort_scene_domains(ctx, name):
    """Both domains of the small and the refined inclusion (the refined fine
    grid has 25,600 bins, so the bin scan runs several passes with a ragged
    tail)."""
    b = _binding()
    sc = _scenes().workload(name)
    for spec in (sc.B, sc.S):
        D = b.Domain(ctx, spec)
        D.p2g()
        perm, cs = D.sort_result()
        ctx.sync()
        operm, ocs = oracle.Domain(spec).sort((8, 8))
        assert np.array_equal(perm.cpu().numpy(), operm)
        assert np.array_equal(cs.cpu().numpy(), ocs)
        D.close()


# ---------------------------------------------------------------- P2G
@pytest.mark.parametrize("dim", [2, 3])
def test_p2g_parity(ctx, dim):
    b = _binding()
    spec = tiny_domain(dim=dim, n_cells=16 if dim == 2 else 10, n_particles=2500, seed=33,
                       bc_kind=[0, 1], bc_mask=[3 if dim == 2 else 7, 2])
    spec.flags[:] = np.where(spec.x[:, 1] < spec.x[:, 1].min() + 2 * spec.dx, 2, 0) | \
        np.where(spec.x[:, 1] > spec.x[:, 1].max() - 2 * spec.dx, 4, 0)
    D = b.Domain(ctx, spec)
    D.p2g()
    m, vn, u = D.grid_state()
    g, r, q = D.sets()
    ctx.sync()
    O = oracle.Domain(spec)
    O.p2g()
    assert rel_err(m.cpu().numpy(), O.m) < 1e-13
    assert rel_err(vn.cpu().numpy(), O.vn) < 1e-12
    assert np.array_equal(q.cpu().numpy(), O.q_all)
    assert np.array_equal(m.cpu().numpy() > 0, O.m > 0)
    D.close()


# ---------------------------------------------------------------- implicit solve + G2P
@pytest.mark.parametrize("dim", [2, 3])
def test_implicit_solve_and_g2p_parity(ctx, dim):
    b = _binding()
    spec = tiny_domain(dim=dim, n_cells=16 if dim == 2 else 8, n_particles=1500 if dim == 2 else 800,
                       seed=34, F_spread=0.08, v_scale=0.3, bc_kind=[0], bc_mask=[3 if dim == 2 else 7])
    spec.flags[:] = np.where(spec.x[:, 1] < spec.x[:, 1].min() + 1.5 * spec.dx, 2, 0)
    dt = 2e-3
    grav = (0.0, -9.8, 0.0)[:dim]
    D = b.Domain(ctx, spec)
    D.p2g()
    st = D.implicit_solve(dt, b.solve_opts(gravity=grav))
    m, vn, u = D.grid_state()
    ctx.sync()
    O = oracle.Domain(spec)
    O.p2g()
    ost = O.solve(dt, oracle.solve_opts(gravity=grav))
    assert st.newton_iters == ost.newton_iters
    assert abs(st.cg_iters - ost.cg_iters) <= 1
    assert st.converged == ost.converged
    assert rel_err(u.cpu().numpy(), O.u) < FP64_TOL
    D.g2p(dt)
    O.g2p(dt)
    x, v, B, F = D.particles_input_order()
    assert rel_err(x - spec.x, O.x - spec.x) < FP64_TOL
    assert rel_err(v, O.v) < FP64_TOL
    assert rel_err(B, O.B) < FP64_TOL
    assert rel_err(F - np.eye(dim), O.F - np.eye(dim)) < FP64_TOL
    D.close()


# ---------------------------------------------------------------- interface operators
def test_interface_operators_parity(ctx):
    b = _binding()
    sc = _scenes().workload("inclusion_tiny")
    B = b.Domain(ctx, sc.B)
    S = b.Domain(ctx, sc.S)
    B.p2g()
    S.p2g()
    n_amb = b.interface_build(B, S)
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    OB.p2g()
    OS.p2g()
    o_amb = oracle.interface(OB, OS)
    assert n_amb == o_amb
    for Dg, Do in ((B, OB), (S, OS)):
        g, r, q = Dg.sets()
        ctx.sync()
        assert np.array_equal(g.cpu().numpy(), Do.gamma)
        assert np.array_equal(r.cpu().numpy(), Do.recv)
        assert np.array_equal(q.cpu().numpy(), Do.q_all)
    torch = ctx.torch
    pi = b.project_S_to_B(S, B, sc.eps_tol)
    opi = oracle.project(OS, OB, sc.eps_tol)
    ctx.sync()
    assert rel_err(pi.cpu().numpy(), opi) < 1e-13
    rng = np.random.default_rng(35)
    vB = rng.normal(size=(B.nn, 2))
    vB_t = torch.as_tensor(vB).to(ctx.device)
    it = b.interp_B_to_S(B, S, vB_t)
    oit = oracle.interp(OB, vB, OS)
    ctx.sync()
    assert rel_err(it.cpu().numpy(), oit) < 1e-13
    vn1 = torch.as_tensor(rng.normal(size=(S.nn, 2))).to(ctx.device)
    out = torch.empty_like(vn1)
    ctx.temporal_interp(1, 2, it, vn1, out)
    ctx.sync()
    assert rel_err(out.cpu().numpy(), oracle.temporal(1, 2, oit, vn1.cpu().numpy())) < 1e-13
    B.close()
    S.close()


# ---------------------------------------------------------------- Schwarz frames
def _schwarz_run(ctx, sc, n_frames):
    b = _binding()
    pair = b.SchwarzPair(ctx, sc)
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    go = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    out = []
    for f in range(n_frames):
        pB, pS = sc.bc_params(f)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        ost = oracle.schwarz_frame(OB, OS, sc.dT, oo)
        gst = pair.frame(go)
        out.append((gst, ost))
    return pair, OB, OS, out


def test_schwarz_frames_inclusion_tiny(ctx):
    """Three frames of the 2D inclusion at dx = 1/20 | 1/50, M = 2, FP64."""
    sc = _scenes().workload("inclusion_tiny")
    pair, OB, OS, stats = _schwarz_run(ctx, sc, 3)
    for gst, ost in stats:
        assert gst.iters == ost.iters
        assert gst.converged == ost.converged
        assert (gst.n_recv_B, gst.n_recv_S, gst.n_amb) == (ost.n_recv_B, ost.n_recv_S, ost.n_amb)
        assert gst.newton_B == ost.newton_B and gst.newton_S == ost.newton_S
    for Dg, Do, spec in ((pair.B, OB, sc.B), (pair.S, OS, sc.S)):
        m, vn, u = Dg.grid_state()
        x, v, Bm, F = Dg.particles_input_order()
        assert rel_err(u.cpu().numpy(), Do.u) < FP64_TOL
        assert rel_err(x - spec.x, Do.x - spec.x) < FP64_TOL
        assert rel_err(F - np.eye(2), Do.F - np.eye(2)) < FP64_TOL
    pair.close()


def test_single_frame_parity(ctx):
    b = _binding()
    sc = _scenes().inclusion_single(inv_dx=40, n_frames=3, delta=0.01)
    D = b.Domain(ctx, sc.B)
    O = oracle.Domain(sc.B)
    for f in range(2):
        p, _ = sc.bc_params(f)
        D.set_bc_params(p)
        O.set_bc_params(p)
        st = D.single_frame(sc.dT, b.solve_opts())
        ost = O.single_frame(sc.dT, oracle.solve_opts())
        assert st.newton_iters == ost.newton_iters
    m, vn, u = D.grid_state()
    x, v, Bm, F = D.particles_input_order()
    assert rel_err(u.cpu().numpy(), O.u) < FP64_TOL
    assert rel_err(x - sc.B.x, O.x - sc.B.x) < FP64_TOL
    D.close()


# ---------------------------------------------------------------- error paths
def test_out_of_grid_reported(ctx):
    """A particle outside its grid is reported (errors are sticky per context,
    so the test uses a context of its own); kernels clamp the stencil so the
    run stays in bounds."""
    b = _binding()
    own = b.Context(0)
    spec = tiny_domain(dim=2, n_cells=8, n_particles=10, seed=36)
    spec.x[3] = [-1.0, 0.05]
    D = b.Domain(own, spec)
    D.p2g()
    with pytest.raises(b.OsmpmError) as e:
        own.sync()
    assert e.value.status == b.OSMPM_E_OUT_OF_GRID
    D.close()
    own.close()


def test_schwarz_frames_fold_3d(ctx):
    """Two frames of the small 3D folding slab (27-node stencils, rotation
    drive, ambiguous overlap nodes in the arbitration), FP64."""
    sc = _scenes().workload("fold_tiny")
    print("3D fold, 2 frames", flush=True)
    pair, OB, OS, stats = _schwarz_run(ctx, sc, 2)
    for gst, ost in stats:
        assert gst.iters == ost.iters
        assert (gst.n_recv_B, gst.n_recv_S, gst.n_amb) == (ost.n_recv_B, ost.n_recv_S, ost.n_amb)
        assert gst.newton_B == ost.newton_B and gst.newton_S == ost.newton_S
    for Dg, Do, spec in ((pair.B, OB, sc.B), (pair.S, OS, sc.S)):
        _, _, u = Dg.grid_state()
        x, _, _, F = Dg.particles_input_order()
        assert rel_err(u.cpu().numpy(), Do.u) < FP64_TOL
        assert rel_err(x - spec.x, Do.x - spec.x) < FP64_TOL
        assert rel_err(F - np.eye(3), Do.F - np.eye(3)) < FP64_TOL
    pair.close()
