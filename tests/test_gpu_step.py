"""GPU Riemannian step against the oracle (eqs. (16)-(18), Sec. 5 optimiser).

Near the rim the step is ill-conditioned (the Mobius addition divides by a
quantity that vanishes there, and the projection of eq. (18) fires or not by
one rounding), so each row's tolerance adds the row's own sensitivity,
measured by re-running the oracle on inputs perturbed at the rounding level
of the working precision."""
import numpy as np
import pytest
import torch

import oracle
from paper_2401_13708_amd import hts, synth
from gpu_inputs import STAGES, embedding

pytestmark = pytest.mark.gpu


def _sensitivity(Y, U, G, grad, eta, mu, mp, rel):
    base, _, _ = oracle.step(Y, U, G, grad, eta, mu, metric_power=mp)
    dev = np.zeros(Y.shape[0])
    for sy, su, sg in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        Yp, _, _ = oracle.step(Y * (1 + sy * rel), U * (1 + su * rel), G, grad * (1 + sg * rel), eta,
                               mu, metric_power=mp)
        dev = np.maximum(dev, np.abs(Yp - base).max(1))
    return base, dev


@pytest.mark.parametrize("stage", STAGES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("metric_power", [2, 1])
def test_step_matches_oracle(ctx, stage, dtype, metric_power):
    step_case(ctx, 3001, stage, dtype, metric_power)


def step_case(ctx, n, stage, dtype, metric_power):
    g = synth.rng(3)
    Y = embedding(n, stage, dtype)
    U = (g.normal(size=(n, 2)) * 1e-3).astype(dtype)
    G = g.uniform(0.2, 3.0, size=(n, 2)).astype(dtype)
    grad = (g.normal(size=(n, 2)) * 10).astype(dtype)
    grad[::7] *= 1e4                     # some large steps that reach the rim
    eta, mu = n / 12000.0, 0.8
    t = [torch.from_numpy(a.copy()).cuda() for a in (Y, U, G, grad)]
    hts.step(ctx, t[0], t[1], t[2], t[3], eta, mu, metric_power=metric_power)
    torch.cuda.synchronize()
    assert ctx.check() == 0
    Yg, Ug, Gg = (a.cpu().numpy() for a in t[:3])
    f = lambda a: a.astype(np.float64)
    Yo, Uo, Go = oracle.step(f(Y), f(U), f(G), f(grad), eta, mu, metric_power=metric_power)
    tol, rel = (2e-6, 1e-6) if dtype == np.float32 else (1e-12, 1e-14)
    assert np.allclose(Gg, Go, rtol=tol, atol=0)
    assert np.allclose(Ug, Uo, rtol=tol, atol=tol * np.abs(Uo).max())
    _, sens = _sensitivity(f(Y), f(U), f(G), f(grad), eta, mu, metric_power, rel)
    err = np.abs(f(Yg) - Yo).max(1)
    # a point the oracle leaves within the single-precision rounding of the
    # unit circle cannot be stored inside the disk: the projection of eq. (18)
    # applies to the stored value, giving (1 - eps) y / |y| instead
    rg, ro = np.hypot(*f(Yg).T), np.hypot(*Yo.T)
    cosang = np.sum(f(Yg) * Yo, 1) / (rg * ro)
    # (and in double precision the test of eq. (18) itself is decided by one
    # rounding for points that land within 1e-15 of the circle)
    at_eps = lambda r: np.abs(r - (1 - 1e-5)) < 2e-7
    projected = (((ro > 1 - 1e-6) & at_eps(rg)) | ((rg > 1 - 1e-6) & at_eps(ro))) & (cosang > 1 - 1e-9)
    ok = projected | (err <= tol + 10 * sens)
    assert np.all(ok), (np.nonzero(~ok)[0][:5], err[~ok][:5], sens[~ok][:5])
    assert np.all(np.sum(f(Yg) ** 2, 1) < 1.0)
    # most rows are well conditioned and must match to the working precision
    assert np.mean(err <= tol) > 0.8
