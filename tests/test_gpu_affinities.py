"""GPU affinities against the oracle: k-NN indices and the CSR pattern of P
bit-exact, P values within rounding of the bisection (1e-12 double, 1e-6
single precision storage)."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_2401_13708_amd import hts, synth

pytestmark = pytest.mark.gpu


def _gpu(ctx, X, perp, k, p_dtype):
    knn, rp, col, val = hts.build_affinities(ctx, torch.from_numpy(X).cuda(), perp, k,
                                             p_dtype=p_dtype)
    torch.cuda.synchronize()
    assert ctx.check() == 0
    return knn.cpu().numpy(), rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()


def _check(ctx, X, perp, k, p_dtype, vtol):
    kg, rg, cg, vg = _gpu(ctx, X, perp, k, p_dtype)
    ko, ro, co, vo = oracle.build_affinities(X.astype(np.float64), perp, k)
    assert np.array_equal(kg, ko)
    assert np.array_equal(rg, ro)
    assert np.array_equal(cg, co)
    # single-precision storage: values below the normal range (tiny p of far
    # neighbours in tight clusters) carry an absolute error up to FLT_MIN
    atol = 1.2e-38 if vg.dtype == np.float32 else 0.0
    assert np.allclose(vg.astype(np.float64), vo, rtol=vtol, atol=atol)
    assert float(np.sum(vg.astype(np.float64))) == pytest.approx(1.0, abs=1e-5 if vtol > 1e-9 else 1e-12)


def test_cfg1_shape_f64(ctx):
    # N = 1000, D = 32 Gaussian mixture, perplexity 30, k = 90, double precision
    X = synth.gaussian_mixture(1000, 32, seed=1)
    _check(ctx, X, 30.0, 90, torch.float64, 1e-12)


def test_hierarchical_f32(ctx):
    X = synth.branching_walk(2500, 50, depth=6, seed=3)
    _check(ctx, X, 30.0, 90, torch.float32, 1e-6)


@pytest.mark.parametrize("n,d,k,perp", [(777, 17, 20, 5.0), (130, 1, 128, 40.0), (65, 3, 64, 10.0),
                                        (2, 5, 1, 0.5)])
def test_ragged_shapes(ctx, n, d, k, perp):
    X = synth.gaussian_mixture(n, d, seed=n + d)
    _check(ctx, X, perp, k, torch.float64, 1e-12)


def test_duplicate_points_tie_break(ctx):
    X = synth.gaussian_mixture(400, 8, seed=4)
    X[50:80] = X[3]          # 31 identical points: distances 0, ties by index
    X[200] = X[201]
    _check(ctx, X, 10.0, 40, torch.float64, 1e-12)


def test_capacity_error(ctx):
    X = torch.from_numpy(synth.gaussian_mixture(300, 8, seed=5)).cuda()
    rp = torch.empty(301, dtype=torch.int64, device="cuda")
    col = torch.empty(100, dtype=torch.int32, device="cuda")
    val = torch.empty(100, dtype=torch.float64, device="cuda")
    nnz = C.c_int64(0)
    rc = hts.lib().hts_build_affinities(ctx.h, hts._stream(None), hts._ptr(X), 300, 8, 1, 10.0, 30,
                                        None, hts._ptr(rp), hts._ptr(col), hts._ptr(val), 1, 100,
                                        C.byref(nnz))
    assert rc == -4
    assert 300 * 30 <= nnz.value <= 2 * 300 * 30
