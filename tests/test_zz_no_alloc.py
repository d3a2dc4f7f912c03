"""The allocation-free slab Monte Carlo entry point (sdm_slab_mc_noalloc)
against the allocating one (sdm_slab_mc), through the C ABI: the same
kernels on the same inputs, with the FP64 per-tuple sums in the library's
static device scratch instead of a context buffer.  Two calls in a row (the
second smaller, so the scratch holds the first call's sums when it starts)
must each equal the allocating call to the rounding of the FP64 sums into
the float outputs (atomic additions may run in another order); sizes beyond
the scratch are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1912_05494_amd import sdm
    assert torch.cuda.is_available()
    ctx = sdm.Context(0)
    yield sdm, ctx, torch
    ctx.close()


def inputs(torch, rng, m):
    f = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float32)).cuda()
    return [f(rng.uniform(0.05, 1.0, m)), f(rng.uniform(380, 780, m)), f(rng.uniform(2, 5, m)),
            f(rng.uniform(0, 34, m)), f(rng.uniform(1.5, 1.58, m)), f(10 ** rng.uniform(-7, -5, m)),
            f(rng.uniform(0, 0.5, m))]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_allocating_entry_point(gpu, precision):
    sdm, ctx, torch = gpu
    rng = np.random.default_rng(17)
    for m, seed in ((5000, 3), (1234, 4)):   # the second call is smaller than the first
        inp = inputs(torch, rng, m)
        ref = sdm.slab_mc(ctx, *inp, n_photons=96, seed=seed, tuple0=11, precision=precision)
        got = sdm.slab_mc(ctx, *inp, n_photons=96, seed=seed, tuple0=11, precision=precision, noalloc=True)
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            g, r = g.cpu().numpy().astype(np.float64), r.cpu().numpy().astype(np.float64)
            assert np.all(np.abs(g - r) <= 2e-7 * np.abs(r) + 1e-12), (m, precision)
        assert float(ref[1].sum()) > 0.0


def test_noalloc_limits(gpu):
    sdm, ctx, torch = gpu
    rng = np.random.default_rng(5)
    big = inputs(torch, rng, 65537)
    with pytest.raises(sdm.SdmError, match="static scratch"):
        sdm.slab_mc(ctx, *big, n_photons=4, noalloc=True)
    # the largest size the scratch holds, then an empty call
    full = [x[:65536].contiguous() for x in big]
    R, T, A, W = sdm.slab_mc(ctx, *full, n_photons=4, noalloc=True)
    torch.cuda.synchronize()
    assert np.allclose((R + T + A).cpu().numpy(), 1.0, atol=1e-5)
    e = torch.empty(0, device="cuda")
    out = sdm.slab_mc(ctx, e, e, e, e, e, e, noalloc=True)
    assert all(x.numel() == 0 for x in out)
