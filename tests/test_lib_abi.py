"""The C-ABI library loads, exports every function include/hts.h declares,
and validates arguments on the host before touching the device."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2401_13708_amd import hts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    names = hts.header_functions()
    assert len(names) >= 14
    L = hts.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", hts.LIB_PATH], capture_output=True,
                         text=True).stdout
    for n in names:
        assert " T %s\n" % n in out, n
    assert set(hts._SIGS) == set(names)


def test_library_is_gfx950_code():
    # the fat binary carries a code object for the gfx950 target only
    blob = open(hts.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob
    assert b"amdgcn-amd-amdhsa--gfx942" not in blob


@pytest.mark.parametrize("call,msg", [
    (lambda L: L.hts_gradient_bh(None, None, None, 1, 0, None, None, None, 1.0, None, 0.5, None,
                                 None, None), "n = 1 < 2"),
    (lambda L: L.hts_gradient_exact(None, None, C.c_void_p(8), 10, 7, C.c_void_p(8),
                                    C.c_void_p(8), C.c_void_p(8), 1.0, C.c_void_p(8),
                                    C.c_void_p(8), None), "bad dtype"),
    (lambda L: L.hts_gradient_exact(None, None, C.c_void_p(8), 10, 0, C.c_void_p(8),
                                    C.c_void_p(8), C.c_void_p(8), 0.0, C.c_void_p(8),
                                    C.c_void_p(8), None), "exaggeration"),
    (lambda L: L.hts_gradient_bh(None, None, C.c_void_p(8), 10, 0, C.c_void_p(8), C.c_void_p(8),
                                 C.c_void_p(8), 1.0, C.c_void_p(8), -0.5, C.c_void_p(8),
                                 C.c_void_p(8), None), "ctx is NULL"),
    (lambda L: L.hts_step(None, None, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                          10, 0, -1.0, 0.5, 0.01, 1e-5, 2), "eta"),
    (lambda L: L.hts_step(None, None, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                          10, 0, 1.0, 0.5, 0.01, 1e-5, 3), "metric_power"),
    (lambda L: L.hts_build_affinities(None, None, C.c_void_p(8), 100, 5, 0, 40.0, 30, None,
                                      C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 0, 100,
                                      C.byref(C.c_int64())), "perplexity"),
    (lambda L: L.hts_build_affinities(None, None, C.c_void_p(8), 100, 5, 0, 10.0, 100, None,
                                      C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 0, 100,
                                      C.byref(C.c_int64())), "not in [1, n)"),
    (lambda L: L.hts_tree_create(None, 1, 20, C.byref(C.c_void_p())), "n_max < 2"),
    (lambda L: L.hts_tree_create(None, 100, 40, C.byref(C.c_void_p())), "max_depth"),
    (lambda L: L.hts_tree_create(None, 3_195_661, 20, C.byref(C.c_void_p())), "2^26"),
    (lambda L: L.hts_build_polar_tree(None, None, None, 10, 0, None), "NULL handle"),
    (lambda L: L.hts_workspace_generation(None, C.byref(C.c_uint64())), "NULL argument"),
])
def test_host_validation(call, msg):
    L = hts.lib()
    rc = call(L)
    assert rc == -1
    assert msg in hts.last_error()


def test_item_list_share_needs_a_context():
    # argument check on the host, before any device work (the negative share
    # is refused in tests/test_gpu_gradient.py, which has a context)
    L = hts.lib()
    assert L.hts_set_item_list(None, 5) != 0
    assert "ctx is NULL" in hts.last_error()
    assert L.hts_set_traversal_launch(None, 16384, 4) != 0
    assert "ctx is NULL" in hts.last_error()
    assert L.hts_set_attract_launch(None, 1) != 0
    assert "ctx is NULL" in hts.last_error()


def test_native_driver_input_file(tmp_path):
    # bench.py writes the native driver's input: header (n, d, start
    # iteration), the same seeded X and starting embedding the bench uses, and
    # the optimiser state
    import numpy as np
    from paper_2401_13708_amd import synth
    path = tmp_path / "in.bin"
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--n", "300", "--d", "5",
                        "--write-native-input", str(path)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    raw = path.read_bytes()
    assert np.frombuffer(raw[:8], np.int64)[0] == 300
    assert np.frombuffer(raw[8:16], np.int32).tolist() == [5, 0]
    assert len(raw) == 16 + 4 * 300 * 5 + 3 * 4 * 300 * 2
    X = np.frombuffer(raw[16:16 + 4 * 1500], np.float32).reshape(300, 5)
    Y, U, G = np.frombuffer(raw[16 + 4 * 1500:], np.float32).reshape(3, 300, 2)
    assert np.array_equal(X, synth.sigmoid_factor_mixture(300, 5, seed=2).astype(np.float32))
    assert np.array_equal(Y, synth.disk_uniform(300, 1e-4, seed=2 + 10 ** 6).astype(np.float32))
    assert not U.any() and (G == 1).all()   # the optimiser's start: update 0, gains 1


def test_native_driver_is_built_for_gfx950():
    exe = os.path.join(ROOT, "paper_2401_13708_amd", "native", "hts_run")
    assert os.path.exists(exe), "the native driver is not built (__graft_entry__.build() builds it)"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
    assert b"amdgcn-amd-amdhsa--gfx950" in open(exe, "rb").read()
