"""The single-frame adjoint entry point that allocates nothing
(osmpm_single_frame_adjoint_noalloc) against the allocating one
(osmpm_single_frame_adjoint), through the C ABI.

Both run the same kernels on the same inputs; only the origin of the work
arrays differs (a fixed per-device region instead of hipMalloc).  The
comparison uses the parity bar of the adjoint (FP64 1e-10 relative on every
adjoint array and the material derivatives, mixed 1e-6) and the end-of-frame
state.  Two calls in a row, the second on a smaller domain, show that the
region's leftover contents from the first call do not leak into the second.
A domain whose work arrays exceed the region is refused before any work."""
import numpy as np
import pytest

from helpers import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09097_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


def _case(ctx, inv_dx, prec, seed):
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.inclusion_single(inv_dx=inv_dx, n_frames=3, delta=0.01, seed=seed)
    rng = np.random.default_rng(seed + 11)
    W = {"x": rng.standard_normal(sc.B.x.shape), "v": rng.standard_normal(sc.B.v.shape),
         "B": rng.standard_normal(sc.B.B.shape), "F": rng.standard_normal(sc.B.F.shape)}
    doms = []
    for _ in range(2):
        D = b.Domain(ctx, sc.B, precision=prec)
        p, _ = sc.bc_params(0)
        D.set_bc_params(p)
        doms.append(D)
    return sc, W, doms


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_adjoint_matches_allocating_adjoint(ctx, precision):
    from paper_2605_09097_amd import binding as b

    prec = b.OSMPM_FP64 if precision == "fp64" else b.OSMPM_MIXED
    tol = 1e-10 if precision == "fp64" else 1e-6
    so = b.solve_opts(newton_rtol=1e-12, newton_atol=1e-16, cg_rtol=1e-12 if precision == "fp64" else 1e-5)
    adj_rtol = 1e-12 if precision == "fp64" else 1e-6
    for inv_dx, seed in ((32, 1), (16, 2)):  # the second call on a smaller domain
        sc, W, (Da, Dn) = _case(ctx, inv_dx, prec, seed)
        print("no-alloc adjoint,", precision, "inv_dx", inv_dx, "particles", sc.B.n_particles, flush=True)
        ga, gmu, glam = b.single_frame_adjoint(Da, sc.dT, so, W, adj_cg_rtol=adj_rtol)
        na, nmu, nlam = b.single_frame_adjoint(Dn, sc.dT, so, W, adj_cg_rtol=adj_rtol, noalloc=True)
        for k in "xvBF":
            g, n = ga[k].cpu().numpy(), na[k].cpu().numpy()
            assert np.isfinite(n).all()
            assert rel_err(n, g) <= tol, (k, rel_err(n, g))
            assert np.abs(n - g).max() <= tol * max(np.abs(g).max(), 1e-300), k
        assert rel_err(nmu, gmu) <= tol and rel_err(nlam, glam) <= tol
        # both domains hold the same end-of-frame state
        xa, xn = Da.particles_input_order()[0], Dn.particles_input_order()[0]
        assert rel_err(xn - sc.B.x, xa - sc.B.x) <= tol
        Da.close()
        Dn.close()


def test_noalloc_adjoint_refuses_a_domain_past_the_region(ctx):
    from paper_2605_09097_amd import binding as b
    from paper_2605_09097_amd import scenes

    sc = scenes.inclusion_single(inv_dx=16, n_frames=3, delta=0.01)
    # two stored points of 10^6 particles of capacity take ~240 MB > 64 MiB
    D = b.Domain(ctx, sc.B, precision=b.OSMPM_FP64, capacity=1_000_000)
    W = {k: np.zeros(getattr(sc.B, k).shape) for k in "xvBF"}
    with pytest.raises(b.OsmpmError) as e:
        b.single_frame_adjoint(D, sc.dT, b.solve_opts(), W, noalloc=True)
    assert e.value.status == b.OSMPM_E_INVALID_ARG
    assert "fixed region" in str(e.value)
    D.close()
