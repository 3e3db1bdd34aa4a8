"""GPU parity of batched execution: many scenes of uneven sizes in shared
launches, each checked against the FP64 CPU oracle run on that scene alone.

A batch gives every scene its own Newton / CG / line-search / Schwarz
decisions, so per-scene iteration counts must equal the oracle's and the
per-scene results must meet the same bars as single-scene runs (1e-10
relative for the FP64 path, 1e-5 for the mixed path).
"""
import numpy as np
import pytest

import oracle
from helpers import rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09097_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


def _batch_scenes():
    """Three inclusion scenes with different grids, radii, moduli and jitter
    seeds (particle counts from ~1.7k to ~4k per scene)."""
    from paper_2605_09097_amd import scenes

    d = scenes.INCLUSION_DELTA
    return [scenes.inclusion_scene(20, 50, r_inc=0.04, E_inc=3e4, seed=11, delta=d, name="b0"),
            scenes.inclusion_scene(30, 60, r_inc=0.07, E_inc=1.5e5, seed=12, delta=d, name="b1"),
            scenes.inclusion_scene(20, 40, r_inc=0.05, E_inc=8e4, seed=13, delta=d, name="b2")]


def _oracle_frames(sc, n_frames):
    OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
    oo = oracle.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    stats = []
    for f in range(n_frames):
        pB, pS = sc.bc_params(f)
        OB.set_bc_params(pB)
        OS.set_bc_params(pS)
        stats.append(oracle.schwarz_frame(OB, OS, sc.dT, oo))
    return OB, OS, stats


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_schwarz_matches_oracle(ctx, precision):
    from paper_2605_09097_amd import binding as b

    scs = _batch_scenes()
    n_frames = 2
    if precision == "fp64":
        prec, tol, so = b.OSMPM_FP64, FP64_TOL, b.solve_opts()
    else:
        prec, tol, so = b.OSMPM_MIXED, MIXED_TOL, b.solve_opts(cg_rtol=1e-5)
    opts = b.schwarz_opts(scs[0].M, eps_tol=scs[0].eps_tol, coarse=so, fine=so)
    # A batch shares one projection regulariser eps_tol; each scene's oracle
    # run uses the same value.
    print("batch of %d scenes, %s, %d frames" % (len(scs), precision, n_frames), flush=True)
    batch = b.SchwarzBatch(ctx, scs, precision=prec)
    gstats = [batch.frame(opts) for _ in range(n_frames)]
    for i, sc in enumerate(scs):
        OB, OS = oracle.Domain(sc.B), oracle.Domain(sc.S)
        oo = oracle.schwarz_opts(sc.M, eps_tol=scs[0].eps_tol)
        for f in range(n_frames):
            pB, pS = sc.bc_params(f)
            OB.set_bc_params(pB)
            OS.set_bc_params(pS)
            ost = oracle.schwarz_frame(OB, OS, sc.dT, oo)
            gst = gstats[f][i]
            assert gst.iters == ost.iters
            assert gst.converged == ost.converged
            assert (gst.n_recv_B, gst.n_recv_S, gst.n_amb) == (ost.n_recv_B, ost.n_recv_S, ost.n_amb)
            if precision == "fp64":
                assert gst.newton_B == ost.newton_B and gst.newton_S == ost.newton_S
        pair = batch.pairs[i]
        for Dg, Do, spec in ((pair.B, OB, sc.B), (pair.S, OS, sc.S)):
            _, _, u = Dg.grid_state()
            x, _, _, F = Dg.particles_input_order()
            assert rel_err(u.cpu().numpy(), Do.u) < tol, (i, spec.dim)
            assert rel_err(x - spec.x, Do.x - spec.x) < tol
            # Particles store H = F - I, so the strain keeps the path's
            # relative accuracy in both precisions.
            assert rel_err(F - np.eye(2), Do.F - np.eye(2)) < tol
    batch.close()


def test_batch_equals_single_pair_runs(ctx):
    """Each scene of a batch reproduces its own single-pair GPU run: same
    Schwarz, Newton and CG counts, displacements equal to rounding."""
    from paper_2605_09097_amd import binding as b

    scs = _batch_scenes()
    opts = b.schwarz_opts(scs[0].M, eps_tol=scs[0].eps_tol)
    batch = b.SchwarzBatch(ctx, scs)
    bst = [batch.frame(opts) for _ in range(2)]
    for i, sc in enumerate(scs):
        pair = b.SchwarzPair(ctx, sc)
        for f in range(2):
            st = pair.frame(opts)
            g = bst[f][i]
            assert (st.iters, st.newton_B, st.newton_S) == (g.iters, g.newton_B, g.newton_S)
            assert abs(st.cg_B - g.cg_B) <= 2 and abs(st.cg_S - g.cg_S) <= 2
        for Dp, Db in ((pair.B, batch.pairs[i].B), (pair.S, batch.pairs[i].S)):
            ua = Dp.grid_state()[2].cpu().numpy()
            ub = Db.grid_state()[2].cpu().numpy()
            assert rel_err(ub, ua) < 1e-12
        pair.close()
    batch.close()


def test_batch_single_frames(ctx):
    """A batch of single domains of different sizes (single_frame) against
    the oracle's single-domain step on each."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    scs = [scenes.inclusion_single(inv_dx=40, n_frames=3, delta=0.01),
           scenes.inclusion_single(inv_dx=24, n_frames=3, delta=0.01, seed=5)]
    doms = [b.Domain(ctx, sc.B) for sc in scs]
    orc = [oracle.Domain(sc.B) for sc in scs]
    batch = b.Batch(ctx, doms)
    for f in range(2):
        for sc, D, O in zip(scs, doms, orc):
            p, _ = sc.bc_params(f)
            D.set_bc_params(p)
            O.set_bc_params(p)
        st = batch.single_frame(scs[0].dT, b.solve_opts())
        for i, O in enumerate(orc):
            ost = O.single_frame(scs[i].dT, oracle.solve_opts())
            assert st[i].newton_iters == ost.newton_iters
            assert st[i].converged == ost.converged
    for sc, D, O in zip(scs, doms, orc):
        u = D.grid_state()[2].cpu().numpy()
        x = D.particles_input_order()[0]
        assert rel_err(u, O.u) < FP64_TOL
        assert rel_err(x - sc.B.x, O.x - sc.B.x) < FP64_TOL
    batch.close()
    for D in doms:
        D.close()


def test_batch_rejects_bad_members(ctx):
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_tiny")
    B = b.Domain(ctx, sc.B)
    S = b.Domain(ctx, sc.S)
    with pytest.raises(b.OsmpmError):
        b.Batch(ctx, [B, B], [S, S])
    Sm = b.Domain(ctx, sc.S, precision=b.OSMPM_MIXED)
    with pytest.raises(b.OsmpmError):
        b.Batch(ctx, [B], [Sm])
    for D in (B, S, Sm):
        D.close()


def _binding_scene_x(sc):
    return sc.S.x


def test_graph_replay_matches_eager(ctx):
    """Solve cycles replayed as HIP graphs (osmpm_ctx_set_graphs) give the results of
    the same launches enqueued one by one, frame after frame (every frame
    replays the cached graphs many times, with eager work and host
    synchronisations in between): equal iteration counts, and state equal to
    rounding (grid sums use floating-point atomics, whose order varies from
    run to run either way)."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_tiny")
    opts = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    runs = {}
    for graphs in (True, False):
        ctx.graphs(graphs)
        pair = b.SchwarzPair(ctx, sc)
        out = []
        for _ in range(3):
            st = pair.frame(opts)
            out.append(((st.iters, st.newton_B, st.newton_S, st.cg_B, st.cg_S),
                        pair.B.grid_state()[2].cpu().numpy().copy(), pair.S.grid_state()[2].cpu().numpy().copy(),
                        pair.S.particles_input_order()[0].copy()))
        pair.close()
        runs[graphs] = out
    ctx.graphs(False)
    for fg, fe in zip(runs[True], runs[False]):
        assert fg[0] == fe[0]
        for a, e in zip(fg[1:3], fe[1:3]):
            assert rel_err(a, e) < 1e-12
        x0 = _binding_scene_x(sc)
        assert rel_err(fg[3] - x0, fe[3] - x0) < 1e-12


@pytest.mark.parametrize("warm", [False, True])
def test_whole_iteration_graphs_match_eager(ctx, warm):
    """Whole Schwarz iterations replayed as HIP graphs (osmpm_ctx_set_graphs
    mode 2, fixed-schedule solves: one Newton step of exactly 12 CG
    iterations, no halving) against the same frames enqueued launch by
    launch, on a batch of three scenes whose pairs leave the launches at
    different iterations: every frame replays the three cached iteration
    graphs (first, odd, even) several times, with eager work and host reads
    between the replays; Schwarz, Newton, CG, halving and failure counts are
    equal per scene and frame, and the state equal to rounding."""
    from paper_2605_09097_amd import binding as b

    scs = _batch_scenes()
    fixed = b.solve_opts(cg_rtol=0.0, max_newton=1, max_ls=0, max_cg=12)
    opts = b.schwarz_opts(scs[0].M, k_max=9, eps_tol=scs[0].eps_tol, coarse=fixed, fine=fixed, warm_start=warm)
    runs = {}
    for mode in (2, 0):
        ctx.graphs(mode)
        batch = b.SchwarzBatch(ctx, scs)
        frames = []
        for _ in range(3):
            st = batch.frame(opts)
            frames.append([(q.iters, q.converged, q.newton_B, q.newton_S, q.cg_B, q.cg_S, q.ls_B, q.ls_S,
                            q.unconv_B, q.unconv_S, q.lsfail_B, q.lsfail_S) for q in st])
            frames.append([(pr.B.grid_state()[2].cpu().numpy().copy(), pr.S.grid_state()[2].cpu().numpy().copy(),
                            pr.S.particles_input_order()[0].copy(), pr.B.particles_input_order()[0].copy())
                           for pr in batch.pairs])
        batch.close()
        runs[mode] = frames
    ctx.graphs(0)
    g, e = runs[2], runs[0]
    for f in range(0, len(g), 2):
        assert g[f] == e[f], (f // 2, g[f], e[f])
        for i, sc in enumerate(scs):
            for a, r in zip(g[f + 1][i][:2], e[f + 1][i][:2]):
                assert rel_err(a, r) < 1e-12
            assert rel_err(g[f + 1][i][2] - sc.S.x, e[f + 1][i][2] - sc.S.x) < 1e-12
            assert rel_err(g[f + 1][i][3] - sc.B.x, e[f + 1][i][3] - sc.B.x) < 1e-12
    # the schedule is what was asked for: at most one Newton attempt per
    # coarse solve (none where the start passes the Newton test), each of
    # exactly 12 CG iterations, taken or refused by the energy test
    for row in e[0]:
        iters, newton_B, cg_B, lsfail_B = row[0], row[2], row[4], row[10]
        assert newton_B + lsfail_B <= iters and cg_B == 12 * (newton_B + lsfail_B)


def test_whole_iteration_graphs_3d_pair(ctx):
    """The same comparison on the small 3D fold (27-node stencils, the
    rotation drive), one pair, warm-started iterations, three frames."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("fold_tiny")
    fixed = b.solve_opts(cg_rtol=0.0, max_newton=1, max_ls=0, max_cg=10)
    opts = b.schwarz_opts(sc.M, k_max=7, eps_tol=sc.eps_tol, coarse=fixed, fine=fixed, warm_start=True)
    runs = {}
    for mode in (2, 0):
        ctx.graphs(mode)
        pair = b.SchwarzPair(ctx, sc)
        out = []
        for _ in range(3):
            q = pair.frame(opts)
            out.append(((q.iters, q.newton_B, q.newton_S, q.cg_B, q.cg_S, q.lsfail_B, q.lsfail_S),
                        pair.B.grid_state()[2].cpu().numpy().copy(), pair.S.particles_input_order()[0].copy()))
        pair.close()
        runs[mode] = out
    ctx.graphs(0)
    # 27-node scatters sum with FP64 atomics in either order: rounding-level
    # differences grow over the frames' iterations, so the FP64 parity bar
    for g, e in zip(runs[2], runs[0]):
        assert g[0] == e[0]
        assert rel_err(g[1], e[1]) < 1e-10
        assert rel_err(g[2] - sc.S.x, e[2] - sc.S.x) < 1e-10


def test_graph_mode_rejects_unknown_values(ctx):
    from paper_2605_09097_amd import binding as b

    for bad in (-1, 3):
        with pytest.raises(b.OsmpmError):
            ctx.graphs(bad)
    ctx.graphs(0)


def test_autotune_picks_a_measured_candidate(ctx):
    from paper_2605_09097_amd import autotune
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_tiny")
    opts = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    cands = [(4, 4), (8, 8)]
    tB, tS, tim = autotune.tune_pair(ctx, sc, opts, candidates=cands, frames=1)
    assert tB in cands and tS in cands
    assert all(v > 0 for v in tim.values())
    t, tim2 = autotune.tune_batch(ctx, [sc, scenes.inclusion_scene(20, 40, seed=3, delta=0.01)], opts,
                                  candidates=cands)
    assert t in cands and set(tim2) == set(cands)


def test_cg_split_scalars_match_fused(ctx):
    """The CG scalars formed by a launch of their own (split mode, used for
    launches of many workgroups) give the results of the fused form: same
    Schwarz, Newton and CG counts, state equal to rounding."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_tiny")
    opts = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    runs = {}
    for mode in (1, 0):
        ctx.cg_split(mode)
        pair = b.SchwarzPair(ctx, sc)
        out = []
        for _ in range(2):
            st = pair.frame(opts)
            out.append(((st.iters, st.newton_B, st.newton_S, st.cg_B, st.cg_S),
                        pair.B.grid_state()[2].cpu().numpy().copy(), pair.S.grid_state()[2].cpu().numpy().copy()))
        pair.close()
        runs[mode] = out
    ctx.cg_split(-1)
    for fs, ff in zip(runs[1], runs[0]):
        assert fs[0] == ff[0]
        for a, e in zip(fs[1:], ff[1:]):
            assert rel_err(a, e) < 1e-12
