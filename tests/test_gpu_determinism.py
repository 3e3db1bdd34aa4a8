"""Determinism of the HIP path across repeated runs and launch shapes.

Integer outputs do not depend on the order of the atomics that form them:
the binning (a stable counting sort), the fixed-point node masses, the
active set, the boundary and receiver sets and the arbitration counts must
be bitwise identical whether a run is repeated or tiled differently.  Floating
point sums change only their rounding order, so FP64 grid displacements
agree to a few ulps of accumulated rounding (1e-12 relative) across tiles.
"""
import numpy as np
import pytest

from helpers import rel_err

pytestmark = pytest.mark.gpu

TILES = [(4, 4), (8, 8), (16, 8), (16, 16)]


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09097_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


def _p2g_outputs(ctx, spec, tile, precision):
    from paper_2605_09097_amd import binding as b

    D = b.Domain(ctx, spec, precision=precision, tile=tile)
    D.p2g()
    perm, _ = D.sort_result()
    m, vn, u = D.grid_state()
    _, _, q = D.sets()
    ctx.sync()
    out = (perm.cpu().numpy(), q.cpu().numpy(), (m.cpu().numpy() > 0))
    D.close()
    return out


@pytest.mark.parametrize("side", ["B", "S"])
def test_repeated_p2g_is_bitwise_identical(ctx, side):
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    spec = getattr(scenes.workload("inclusion_refined"), side)
    first = _p2g_outputs(ctx, spec, (8, 8), b.OSMPM_MIXED)
    for _ in range(2):
        again = _p2g_outputs(ctx, spec, (8, 8), b.OSMPM_MIXED)
        for a, c in zip(first, again):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("side", ["B", "S"])
def test_fixed_point_masses_do_not_depend_on_tiles(ctx, side):
    """The permutation depends on the tile shape (bins are tile-major); the
    fixed-point masses and the active set do not."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    spec = getattr(scenes.workload("inclusion_refined"), side)
    ref = _p2g_outputs(ctx, spec, TILES[0], b.OSMPM_MIXED)
    for tile in TILES[1:]:
        out = _p2g_outputs(ctx, spec, tile, b.OSMPM_MIXED)
        assert np.array_equal(out[1], ref[1])
        assert np.array_equal(out[2], ref[2])
        assert np.array_equal(np.sort(out[0]), np.arange(spec.n_particles))


def test_schwarz_frames_across_tiles(ctx):
    """Three FP64 frames of the small inclusion with four tile shapes: the
    same Schwarz, Newton and receiver counts, and displacements within
    rounding of each other."""
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.workload("inclusion_tiny")
    go = b.schwarz_opts(sc.M, eps_tol=sc.eps_tol)
    runs = []
    for tile in TILES:
        pair = b.SchwarzPair(ctx, sc, tile_B=tile, tile_S=tile)
        stats = []
        for _ in range(3):
            st = pair.frame(go)
            stats.append((st.iters, st.converged, st.newton_B, st.newton_S, st.n_recv_B, st.n_recv_S, st.n_amb))
        u = [D.grid_state()[2].cpu().numpy() for D in (pair.B, pair.S)]
        x = [D.particles_input_order()[0] for D in (pair.B, pair.S)]
        runs.append((stats, u, x))
        pair.close()
    for stats, u, x in runs[1:]:
        assert stats == runs[0][0]
        for a, c in zip(u, runs[0][1]):
            assert rel_err(a, c) < 1e-12
        for a, c, spec in zip(x, runs[0][2], (sc.B, sc.S)):
            assert rel_err(a - spec.x, c - spec.x) < 1e-12
