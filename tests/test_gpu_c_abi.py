"""One iteration through the C ABI alone: tests/c_abi/hts_iteration.cpp, a host
program linked to libhts.so that calls only the functions of include/hts.h
(tree, Barnes-Hut gradient, step), run as a child process on seeded inputs;
its gradient, Z and stepped points are checked against the FP64 oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2401_13708_amd import synth
from gpu_inputs import embedding, rel, rel_row

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "hts_iteration")


@pytest.mark.parametrize("n,stage", [(3000, "mid"), (517, "late")])
def test_c_caller_one_iteration(tmp_path, n, stage):
    if not os.path.exists(BIN):
        pytest.fail("the C-ABI caller is not built (__graft_entry__.build() builds it)")
    Y = embedding(n, stage, np.float32)
    rp, col, val = synth.random_csr(n, 30, seed=21, dtype=np.float32)
    theta, ex, eta, mu = 0.5, 12.0, n / 12000.0, 0.5
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.array([n, col.size], np.int64).tobytes())
        f.write(np.array([theta, ex, eta, mu], np.float64).tobytes())
        f.write(np.ascontiguousarray(Y, np.float32).tobytes())
        f.write(np.ascontiguousarray(rp, np.int64).tobytes())
        f.write(np.ascontiguousarray(col, np.int32).tobytes())
        f.write(np.ascontiguousarray(val, np.float32).tobytes())
    print("running", BIN, n, stage, flush=True)
    r = subprocess.run([BIN, str(src), str(dst)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(dst, "rb").read()
    g = np.frombuffer(raw[:8 * n], np.float32).reshape(n, 2)
    z = float(np.frombuffer(raw[8 * n:8 * n + 8], np.float64)[0])
    Y1 = np.frombuffer(raw[8 * n + 8:], np.float32).reshape(n, 2)
    Yo = Y.astype(np.float64)
    go, zo, _ = oracle.gradient_bh(Yo, rp, col, val.astype(np.float64), oracle.Tree(Yo), theta, ex)
    assert rel(g, go) < 1e-3
    assert rel_row(g, go) < 1e-3
    assert z == pytest.approx(zo, rel=1e-5)
    Yo1, _, _ = oracle.step(Yo, np.zeros_like(Yo), np.ones_like(Yo), go, eta, mu)
    # the step moves by eta * gains * metric * gradient: its error follows the
    # gradient's (1e-3) plus the rounding of single-precision positions
    move = np.abs(Yo1 - Yo).max()
    assert np.abs(Y1.astype(np.float64) - Yo1).max() <= 1e-3 * move + 1e-6
