"""The native driver paper_2401_13708_amd/native/hts_run (affinities and
iterations of the Sec. 5 schedule through include/hts.h, no Python in the
process) against the Python driver embed.Embedding on the same seeded input:
both make the same library calls in the same order on one stream, so the
embeddings after the same iterations are equal bit for bit."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_2401_13708_amd import hts, synth
from paper_2401_13708_amd.embed import Embedding

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "paper_2401_13708_amd", "native", "hts_run")


@pytest.mark.parametrize("n,d,it0,warmup,steps,item_list",
                         [(3000, 24, 0, 3, 5, -1), (1777, 10, 0, 248, 4, 2), (2100, 12, 247, 1, 4, -1)])
def test_native_driver_equals_python_driver(ctx, tmp_path, n, d, it0, warmup, steps, item_list):
    if not os.path.exists(BIN):
        pytest.fail("the native driver is not built (__graft_entry__.build() builds it)")
    src, dst = tmp_path / "in.bin", tmp_path / "y.bin"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--n", str(n), "--d", str(d),
                        "--write-native-input", str(src), "--native-start-iteration", str(it0)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(src, "rb").read()
    assert np.frombuffer(raw[8:16], np.int32).tolist() == [d, it0]
    X = np.frombuffer(raw[16:16 + 4 * n * d], np.float32).reshape(n, d)
    Y0 = synth.disk_uniform(n, 1e-4, seed=2 + 10 ** 6)
    cmd = [BIN, str(src), "--warmup", str(warmup), "--steps", str(steps), "--out", str(dst)]
    if item_list >= 0:
        cmd += ["--item-list", str(item_list)]
    print("running", cmd, flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n"] == n and line["steps"] == steps and line["iters_per_s"] > 0
    Yn = np.fromfile(dst, np.float32).reshape(n, 2)

    dev = torch.device("cuda", 0)
    _, rp, col, val = hts.build_affinities(ctx, torch.from_numpy(X.copy()).to(dev), 30.0, 90,
                                           p_dtype=torch.float32, want_knn=False)
    assert int(col.numel()) == line["nnz"]
    if item_list >= 0:
        ctx.set_item_list(item_list)
    try:
        # the file holds the state of the schedule at iteration it0, so the
        # native run continues the Python driver's run from the start
        emb = Embedding(ctx, rp, col, val, torch.from_numpy(Y0.copy()).to(dev), theta=0.5)
        emb.run(it0 + warmup + steps)
        torch.cuda.synchronize()
    finally:
        ctx.set_item_list(hts.DEFAULT_ITEM_LIST)
    assert ctx.check() == 0
    Yp = emb.Y.cpu().numpy()
    assert np.array_equal(Yn, Yp)
    # the iterations moved the points (the comparison is not of the start)
    assert not np.array_equal(Yp, Y0)


def test_native_reload_times_the_window_from_the_stored_state(ctx, tmp_path):
    # --reload: the warm-up (counting kernels) is undone by loading the
    # stored state again, so the timed steps are iterations it0 .. it0 + K - 1
    # of the schedule, as a window of bench.py
    n, d, it0, steps = 1500, 16, 7, 4
    src, dst = tmp_path / "in.bin", tmp_path / "y.bin"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--n", str(n), "--d", str(d),
                        "--write-native-input", str(src), "--native-start-iteration", str(it0)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(src, "rb").read()
    X = np.frombuffer(raw[16:16 + 4 * n * d], np.float32).reshape(n, d)
    cmd = [BIN, str(src), "--warmup", "3", "--reload", "--steps", str(steps), "--out", str(dst)]
    print("running", cmd, flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["start_iteration"] == it0 and line["steps"] == steps
    Yn = np.fromfile(dst, np.float32).reshape(n, 2)
    dev = torch.device("cuda", 0)
    _, rp, col, val = hts.build_affinities(ctx, torch.from_numpy(X.copy()).to(dev), 30.0, 90,
                                           p_dtype=torch.float32, want_knn=False)
    Y0 = synth.disk_uniform(n, 1e-4, seed=2 + 10 ** 6)
    emb = Embedding(ctx, rp, col, val, torch.from_numpy(Y0).to(dev), theta=0.5)
    emb.run(it0 + steps)
    torch.cuda.synchronize()
    assert ctx.check() == 0
    assert np.array_equal(Yn, emb.Y.cpu().numpy())
