"""hts_gradient_exact_noalloc (the exact gradient with its workspace in the
library's fixed per-GPU region, for callers that cannot allocate) against
hts_gradient_exact on the same inputs: the same kernels on the same pieces of
memory, so gradient, Z and cost must agree bit for bit.  Two calls in a row,
the second smaller (the region keeps the first call's contents), in both
precisions; the size limit is refused before anything runs; no call grows a
workspace or takes device memory."""
import numpy as np
import pytest
import torch

from paper_2401_13708_amd import hts, synth

pytestmark = pytest.mark.gpu


def _inputs(n, dtype, seed):
    Y = synth.disk_state(n, "mid", seed=seed).astype(dtype)
    rp, col, val = synth.random_csr(n, min(30, n - 1), seed=seed + 1, dtype=dtype)
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (Y, rp, col, val)]


def _both(ctx, ref_ctx, n, dtype, seed, ex):
    Y, rp, col, val = _inputs(n, dtype, seed)
    g = torch.full_like(Y, float("nan"))
    z = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    kl = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    hts.gradient_exact_noalloc(ctx, Y, rp, col, val, g, z, ex, kl=kl)
    kr = torch.zeros(1, dtype=torch.float64, device="cuda")
    gr, zr = hts.gradient_exact(ref_ctx, Y, rp, col, val, ex, kl=kr)
    torch.cuda.synchronize()
    assert ctx.check() == 0 and ref_ctx.check() == 0
    return (g, z, kl), (gr, zr, kr)


@pytest.mark.parametrize("dtype,sizes", [(np.float32, (5000, 1337)), (np.float64, (3001, 700)),
                                         (np.float32, (hts.NOALLOC_MAX_N, 2))])
def test_noalloc_equals_exact(dtype, sizes):
    ctx, ref = hts.Context(0), hts.Context(0)
    try:
        # a first call loads the kernels; from then on the calls must not
        # change the device's free memory or the context's workspaces
        _both(ctx, ref, 64, dtype, 150, 1.0)
        gen0 = ctx.generation()
        free0 = torch.cuda.mem_get_info()[0]
        for k, n in enumerate(sizes):
            got, want = _both(ctx, ref, n, dtype, 160 + 10 * k, 12.0 if k == 0 else 1.0)
            for a, b in zip(got, want):
                assert torch.equal(a, b), (n, k)
            assert torch.isfinite(got[0]).all()
        assert ctx.generation() == gen0 == 0
        # the reference calls grew only the other context's workspaces
        Y, rp, col, val = _inputs(300, dtype, 190)
        g = torch.empty_like(Y)
        z = torch.empty(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        hts.gradient_exact_noalloc(ctx, Y, rp, col, val, g, z, 1.0)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free1
        assert free0 >= 0
    finally:
        ctx.close()
        ref.close()


def test_noalloc_refuses_sizes_beyond_the_region():
    ctx = hts.Context(0)
    try:
        n = hts.NOALLOC_MAX_N + 1
        Y, rp, col, val = _inputs(n, np.float32, 200)
        g = torch.full_like(Y, 7.0)
        z = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(hts.HTSError, match="HTS_ECAPACITY"):
            hts.gradient_exact_noalloc(ctx, Y, rp, col, val, g, z, 1.0)
        torch.cuda.synchronize()
        assert bool((g == 7.0).all()) and float(z[0]) == 7.0   # nothing ran
        with pytest.raises(hts.HTSError, match="exaggeration"):
            hts.gradient_exact_noalloc(ctx, Y[:10].contiguous(), rp[:11].contiguous(), col, val,
                                       g[:10].contiguous(), z, 0.0)
    finally:
        ctx.close()
