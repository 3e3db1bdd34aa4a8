"""GPU parity at the full sizes of the measured workloads.

* The refined 2D inclusion (coarse dx 1/160, fine dx 1/400, 62,308 + 45,244
  particles), the throughput workload: its first two Schwarz frames on the
  GPU against the same frames of the FP64 oracle, on the mixed path with the
  tile shapes the throughput run uses and with the default tiles, and on the
  FP64 path.
* The Hertz contact (634,738 + 378,944 particles, 2D) and the 3D fold
  (26,880 + 409,600 particles): a full run of the oracle takes hours, so the
  outputs it computes quickly are compared: the binning sort (bit-exact),
  the fixed-point node masses (bit-exact) and the P2G grid state.

* The throughput run's configuration (mixed, warm-started iterations) on the
  refined inclusion, and the 64-scene batch as launched by the throughput
  run with three sampled scenes checked against the oracle run of that
  scene alone.

Bars: bit-exact for integers; 1e-10 relative (2-norm) for the FP64 path with
equal Schwarz and Newton counts; 1e-5 for the mixed path (FP32 bulk, CG
tolerance 1e-5, which bounds the error each solve leaves).
"""
import numpy as np
import pytest

import oracle
from helpers import rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5
FRAMES = 2


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09097_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def headline():
    """The refined inclusion and its first frames on the oracle (~5 s)."""
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_refined")
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    stats = []
    for f in range(FRAMES):
        pB, pS = sc.bc_params(f)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        stats.append(oracle.schwarz_frame(OB, OS, sc.dT, oo))
    return sc, OB, OS, stats


def _compare(pair, sc, OB, OS, tol):
    for Dg, Do, spec in ((pair.B, OB, sc.B), (pair.S, OS, sc.S)):
        m, vn, u = Dg.grid_state()
        x, v, Bm, F = Dg.particles_input_order()
        assert rel_err(u.cpu().numpy(), Do.u) < tol
        assert rel_err(x - spec.x, Do.x - spec.x) < tol
        assert rel_err(v, Do.v) < tol
        assert rel_err(F - np.eye(2), Do.F - np.eye(2)) < tol


@pytest.mark.parametrize("tiles", [((16, 8), (8, 8)), (None, None)], ids=["tuned", "default"])
def test_headline_frames_mixed(ctx, headline, tiles):
    from paper_2605_09097_amd import binding as b

    sc, OB, OS, ostats = headline
    pair = b.SchwarzPair(ctx, sc, precision=b.OSMPM_MIXED, tile_B=tiles[0], tile_S=tiles[1])
    solve = b.solve_opts(cg_rtol=1e-5)
    go = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=solve, fine=solve)
    for f in range(FRAMES):
        st = pair.frame(go)
        assert st.converged
        assert abs(st.iters - ostats[f].iters) <= 1
        assert (st.n_recv_B, st.n_recv_S, st.n_amb) == (ostats[f].n_recv_B, ostats[f].n_recv_S,
                                                         ostats[f].n_amb)
    _compare(pair, sc, OB, OS, MIXED_TOL)
    pair.close()


def test_headline_frames_fp64(ctx, headline):
    from paper_2605_09097_amd import binding as b

    sc, OB, OS, ostats = headline
    pair = b.SchwarzPair(ctx, sc)
    go = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    for f in range(FRAMES):
        st = pair.frame(go)
        ost = ostats[f]
        assert (st.iters, st.converged) == (ost.iters, ost.converged)
        assert (st.newton_B, st.newton_S) == (ost.newton_B, ost.newton_S)
        assert (st.n_recv_B, st.n_recv_S, st.n_amb) == (ost.n_recv_B, ost.n_recv_S, ost.n_amb)
    _compare(pair, sc, OB, OS, FP64_TOL)
    pair.close()


@pytest.mark.parametrize("name,side,tile", [("hertz", "B", (16, 8)), ("hertz", "S", (8, 8)),
                                            ("fold", "B", (4, 4, 4)), ("fold", "S", (4, 4, 4))])
def test_large_domain_sort_and_p2g(ctx, name, side, tile):
    """One domain of a large workload on the mixed path: sort permutation and
    bin offsets bit-exact against the oracle's sort with the same tiles,
    fixed-point node masses bit-exact, node mass and P2G velocity to 1e-5."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    spec = getattr(scenes.workload(name), side)
    D = b.Domain(ctx, spec, precision=b.OSMPM_MIXED, tile=tile)
    D.p2g()
    perm, cs = D.sort_result()
    m, vn, u = D.grid_state()
    _, _, q = D.sets()
    ctx.sync()
    O = oracle.Domain(spec)
    operm, ocs = O.sort(tile)
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    O.p2g()
    assert np.array_equal(q.cpu().numpy(), O.q_all)
    assert np.array_equal(m.cpu().numpy() > 0, O.m > 0)
    assert rel_err(m.cpu().numpy(), O.m) < MIXED_TOL
    assert rel_err(vn.cpu().numpy(), O.vn) < MIXED_TOL
    D.close()


@pytest.fixture(scope="module")
def headline_warm():
    """The refined inclusion's first frames on the oracle with warm-started
    Schwarz iterations (the throughput run's setting)."""
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_refined")
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, warm_start=True)
    stats = []
    for f in range(FRAMES):
        pB, pS = sc.bc_params(f)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        stats.append(oracle.schwarz_frame(OB, OS, sc.dT, oo))
    return sc, OB, OS, stats


def test_headline_frames_mixed_warm(ctx, headline_warm):
    """The throughput run's configuration (mixed path, warm-started Schwarz
    iterations, tuned tiles) against the warm-started FP64 oracle."""
    from paper_2605_09097_amd import binding as b

    sc, OB, OS, ostats = headline_warm
    pair = b.SchwarzPair(ctx, sc, precision=b.OSMPM_MIXED, tile_B=(8, 4), tile_S=(8, 8))
    solve = b.solve_opts(cg_rtol=1e-5)
    go = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol, coarse=solve, fine=solve, warm_start=True)
    print("refined inclusion, warm-started, mixed", flush=True)
    for f in range(FRAMES):
        st = pair.frame(go)
        assert st.converged
        assert abs(st.iters - ostats[f].iters) <= 1
    _compare(pair, sc, OB, OS, MIXED_TOL)
    pair.close()


def test_batch64_sampled_scenes_mixed(ctx):
    """The batched configuration as the throughput run launches it (64 scenes
    of uneven sizes in shared launches, mixed path, warm-started iterations,
    16 x 16 tiles), one frame; three sampled scenes (the first, a middle and
    the last) against the FP64 oracle run of that scene alone."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    scs = [scenes.batch_scene(s) for s in range(64)]
    solve = b.solve_opts(cg_rtol=1e-5)
    go = b.schwarz_opts(scs[0].M, eps_tol=scs[0].eps_tol, coarse=solve, fine=solve, warm_start=True)
    batch = b.SchwarzBatch(ctx, scs, precision=b.OSMPM_MIXED, tile=(16, 16))
    print("64-scene batch, one frame", flush=True)
    gst = batch.frame(go)
    for s in (0, 31, 63):
        sc = scs[s]
        OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
        pB, pS = sc.bc_params(0)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        ost = oracle.schwarz_frame(OB, OS, sc.dT, oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol, warm_start=True))
        assert gst[s].converged and abs(gst[s].iters - ost.iters) <= 1, (s, gst[s].iters, ost.iters)
        _compare(batch.pairs[s], sc, OB, OS, MIXED_TOL)
    batch.close()
