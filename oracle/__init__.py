"""ctypes binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The oracle (``hts_oracle.c``) is a
plain, slow, double-precision implementation of hyperbolic t-SNE written from
the paper; it shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hts_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
            "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.ora_dist.restype = C.c_double
        L.ora_dist.argtypes = [C.c_double] * 4
        L.ora_dist_grad.argtypes = [C.c_double] * 4 + [_D]
        L.ora_mobius_add.argtypes = [C.c_double] * 4 + [_D]
        L.ora_exp_map.argtypes = [C.c_double] * 4 + [_D]
        L.ora_einstein_midpoint.argtypes = [_D, C.c_int64, _D]
        L.ora_knn_rows.argtypes = [_D, C.c_int64, C.c_int32, C.c_int32, _I64, C.c_int64, _I32, _D]
        L.ora_cond_p.argtypes = [_D, C.c_int64, C.c_int32, C.c_double, _D, _D]
        L.ora_symmetrize.argtypes = [_I32, _D, C.c_int64, C.c_int32, _I64, _I32, _D, C.c_int64, _I64]
        L.ora_build_affinities.argtypes = [_D, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                                           _I32, _I64, _I32, _D, C.c_int64, _I64]
        L.ora_kl_cost.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double, _D]
        L.ora_cosne_cost.argtypes = [_D, C.c_int64, _I64, _I32, _D, _D, C.c_double, C.c_double, _D]
        L.ora_cosne_gradient.argtypes = [_D, C.c_int64, _D, C.c_double, C.c_double, _D, _D]
        L.ora_gradient_exact.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double, _D, _D]
        L.ora_gradient_exact_rows.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double,
                                              _I64, C.c_int64, C.c_double, _D]
        L.ora_z_exact.argtypes = [_D, C.c_int64, _D]
        L.ora_tree_build.argtypes = [_D, C.c_int64, C.c_int32, C.POINTER(C.c_void_p)]
        L.ora_tree_build_partition.argtypes = [_D, C.c_int64, C.c_int32, C.POINTER(C.c_void_p)]
        L.ora_tree_build_rule.argtypes = [_D, C.c_int64, C.c_int32, C.c_int32,
                                          C.POINTER(C.c_void_p)]
        L.ora_tree_build_partition_rule.argtypes = [_D, C.c_int64, C.c_int32, C.c_int32,
                                                    C.POINTER(C.c_void_p)]
        L.ora_radial_mid.restype = C.c_double
        L.ora_radial_mid.argtypes = [C.c_double, C.c_double, C.c_int32]
        L.ora_tree_free.argtypes = [C.c_void_p]
        L.ora_tree_num_nodes.restype = C.c_int64
        L.ora_tree_num_nodes.argtypes = [C.c_void_p]
        L.ora_tree_export.argtypes = [C.c_void_p, _I32, _I32, _I32, _I32, _D, _D, _D, _I64]
        L.ora_gradient_bh.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double, C.c_void_p,
                                      C.c_double, _D, _D, _I64]
        L.ora_gradient_bh_rows.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double,
                                           C.c_void_p, C.c_double, _I64, C.c_int64, C.c_double,
                                           _D, _I64]
        L.ora_euclid_cost.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double, _D]
        L.ora_gradient_euclid_exact.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double, _D,
                                                _D]
        L.ora_gradient_euclid_bh.argtypes = [_D, C.c_int64, _I64, _I32, _D, C.c_double,
                                             C.c_void_p, C.c_double, _D, _D, _I64]
        L.ora_tree_export_euclid.argtypes = [C.c_void_p, _D, _D]
        L.ora_step.argtypes = [_D, _D, _D, _D, C.c_int64, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_int32]
        L.ora_set_threads.argtypes = [C.c_int32]
        L.ora_get_threads.restype = C.c_int32
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed with code %d" % (what, rc))


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ora_get_threads())


# ---------------------------------------------------------------- geometry
def dist(a, b) -> float:
    return lib().ora_dist(float(a[0]), float(a[1]), float(b[0]), float(b[1]))


def dist_grad(a, b) -> np.ndarray:
    g = np.zeros(2)
    lib().ora_dist_grad(float(a[0]), float(a[1]), float(b[0]), float(b[1]), _p(g, _D))
    return g


def mobius_add(a, b) -> np.ndarray:
    o = np.zeros(2)
    lib().ora_mobius_add(float(a[0]), float(a[1]), float(b[0]), float(b[1]), _p(o, _D))
    return o


def exp_map(y, v) -> np.ndarray:
    o = np.zeros(2)
    lib().ora_exp_map(float(y[0]), float(y[1]), float(v[0]), float(v[1]), _p(o, _D))
    return o


def einstein_midpoint(Y) -> np.ndarray:
    Y = _f64(Y).reshape(-1, 2)
    o = np.zeros(2)
    lib().ora_einstein_midpoint(_p(Y, _D), Y.shape[0], _p(o, _D))
    return o


# ---------------------------------------------------------------- affinities
def knn_rows(X, k: int, rows=None):
    X = _f64(X)
    n, d = X.shape
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = n if rows_a is None else rows_a.size
    idx = np.zeros((nr, k), dtype=np.int32)
    d2 = np.zeros((nr, k))
    _check(lib().ora_knn_rows(_p(X, _D), n, d, k, _p(rows_a, _I64), nr, _p(idx, _I32),
                              _p(d2, _D)), "knn_rows")
    return idx, d2


def cond_p(d2, perplexity: float):
    d2 = _f64(d2)
    n, k = d2.shape
    p = np.zeros((n, k))
    beta = np.zeros(n)
    _check(lib().ora_cond_p(_p(d2, _D), n, k, float(perplexity), _p(p, _D), _p(beta, _D)), "cond_p")
    return p, beta


def symmetrize(knn, pc):
    knn = np.ascontiguousarray(knn, dtype=np.int32)
    pc = _f64(pc)
    n, k = knn.shape
    cap = 2 * n * k
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(cap, dtype=np.int32)
    val = np.zeros(cap)
    nnz = np.zeros(1, dtype=np.int64)
    _check(lib().ora_symmetrize(_p(knn, _I32), _p(pc, _D), n, k, _p(rp, _I64), _p(col, _I32),
                                _p(val, _D), cap, _p(nnz, _I64)), "symmetrize")
    m = int(nnz[0])
    return rp, col[:m].copy(), val[:m].copy()


def build_affinities(X, perplexity: float = 30.0, k: int = 90):
    X = _f64(X)
    n, d = X.shape
    cap = 2 * n * k
    knn = np.zeros((n, k), dtype=np.int32)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(cap, dtype=np.int32)
    val = np.zeros(cap)
    nnz = np.zeros(1, dtype=np.int64)
    _check(lib().ora_build_affinities(_p(X, _D), n, d, float(perplexity), k, _p(knn, _I32),
                                      _p(rp, _I64), _p(col, _I32), _p(val, _D), cap,
                                      _p(nnz, _I64)), "build_affinities")
    m = int(nnz[0])
    return knn, rp, col[:m].copy(), val[:m].copy()


# ---------------------------------------------------------------- cost / gradients
def _csr(rp, col, val):
    return (np.ascontiguousarray(rp, dtype=np.int64), np.ascontiguousarray(col, dtype=np.int32),
            _f64(val))


def cosne_cost(Y, rp, col, val, xnorm2, lambda1: float, lambda2: float) -> float:
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    xn = _f64(xnorm2)
    c = np.zeros(1)
    _check(lib().ora_cosne_cost(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32), _p(val, _D),
                                _p(xn, _D), float(lambda1), float(lambda2), _p(c, _D)), "cosne_cost")
    return float(c[0])


def cosne_gradient(Y, xnorm2, lambda1: float, lambda2: float, g_kl) -> np.ndarray:
    Y = _f64(Y).reshape(-1, 2)
    xn, gk = _f64(xnorm2), _f64(g_kl).reshape(-1, 2)
    g = np.zeros_like(Y)
    _check(lib().ora_cosne_gradient(_p(Y, _D), Y.shape[0], _p(xn, _D), float(lambda1),
                                    float(lambda2), _p(gk, _D), _p(g, _D)), "cosne_gradient")
    return g


def kl_cost(Y, rp, col, val, exaggeration: float = 1.0) -> float:
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    c = np.zeros(1)
    _check(lib().ora_kl_cost(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32), _p(val, _D),
                             float(exaggeration), _p(c, _D)), "kl_cost")
    return float(c[0])


def gradient_exact(Y, rp, col, val, exaggeration: float = 1.0):
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    g = np.zeros_like(Y)
    z = np.zeros(1)
    _check(lib().ora_gradient_exact(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32),
                                    _p(val, _D), float(exaggeration), _p(g, _D), _p(z, _D)),
           "gradient_exact")
    return g, float(z[0])


def z_exact(Y) -> float:
    Y = _f64(Y).reshape(-1, 2)
    z = np.zeros(1)
    _check(lib().ora_z_exact(_p(Y, _D), Y.shape[0], _p(z, _D)), "z_exact")
    return float(z[0])


def gradient_exact_rows(Y, rp, col, val, rows, z: float, exaggeration: float = 1.0):
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    g = np.zeros((rows.size, 2))
    _check(lib().ora_gradient_exact_rows(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32),
                                         _p(val, _D), float(exaggeration), _p(rows, _I64),
                                         rows.size, float(z), _p(g, _D)), "gradient_exact_rows")
    return g


def radial_mid(lo: float, hi: float, split_rule: int) -> float:
    """Radial split point of a cell (eq. (10) for rule 0, eq. (9) for rule 1)."""
    return float(lib().ora_radial_mid(float(lo), float(hi), int(split_rule)))


class Tree:
    """Polar quadtree built by insertion (or by recursive partition)."""

    def __init__(self, Y, max_depth: int = 20, method: str = "insert", split_rule: int = 0):
        self.Y = _f64(Y).reshape(-1, 2)
        h = C.c_void_p()
        fn = lib().ora_tree_build_rule if method == "insert" else lib().ora_tree_build_partition_rule
        _check(fn(_p(self.Y, _D), self.Y.shape[0], max_depth, int(split_rule), C.byref(h)),
               "tree_build")
        self.h = h
        self.n_nodes = int(lib().ora_tree_num_nodes(h))

    def export(self):
        m, n = self.n_nodes, self.Y.shape[0]
        out = dict(count=np.zeros(m, np.int32), depth=np.zeros(m, np.int32),
                   first=np.zeros(m, np.int32), next=np.zeros(m, np.int32),
                   mid=np.zeros((m, 2)), r_cell=np.zeros(m), bounds=np.zeros((m, 4)),
                   perm=np.zeros(n, np.int64))
        _check(lib().ora_tree_export(self.h, _p(out["count"], _I32), _p(out["depth"], _I32),
                                     _p(out["first"], _I32), _p(out["next"], _I32),
                                     _p(out["mid"], _D), _p(out["r_cell"], _D),
                                     _p(out["bounds"], _D), _p(out["perm"], _I64)), "tree_export")
        return out

    def export_euclid(self):
        """Per node (pre-order): Euclidean centre of mass and Euclidean diameter."""
        m = self.n_nodes
        cent, diam = np.zeros((m, 2)), np.zeros(m)
        _check(lib().ora_tree_export_euclid(self.h, _p(cent, _D), _p(diam, _D)), "export_euclid")
        return cent, diam

    def __del__(self):
        try:
            if self.h:
                lib().ora_tree_free(self.h)
                self.h = None
        except Exception:
            pass


def gradient_bh(Y, rp, col, val, tree: Tree, theta: float, exaggeration: float = 1.0):
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    g = np.zeros_like(Y)
    z = np.zeros(1)
    cnt = np.zeros(4, dtype=np.int64)
    _check(lib().ora_gradient_bh(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32), _p(val, _D),
                                 float(exaggeration), tree.h, float(theta), _p(g, _D), _p(z, _D),
                                 _p(cnt, _I64)), "gradient_bh")
    return g, float(z[0]), dict(tests=int(cnt[0]), accepts=int(cnt[1]), pairs=int(cnt[2]),
                                covered=int(cnt[3]))


def gradient_bh_rows(Y, rp, col, val, tree: Tree, theta: float, rows, z: float,
                     exaggeration: float = 1.0):
    """Barnes-Hut gradient rows of a subset of the queries, Z given."""
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    g = np.zeros((rows.size, 2))
    cnt = np.zeros(4, dtype=np.int64)
    _check(lib().ora_gradient_bh_rows(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32),
                                      _p(val, _D), float(exaggeration), tree.h, float(theta),
                                      _p(rows, _I64), rows.size, float(z), _p(g, _D),
                                      _p(cnt, _I64)), "gradient_bh_rows")
    return g, dict(tests=int(cnt[0]), accepts=int(cnt[1]), pairs=int(cnt[2]), covered=int(cnt[3]))


# ---- h-SNE (Sec. 4-C): Euclidean Student-t term of the disk coordinates ----

def euclid_cost(Y, rp, col, val, exaggeration: float = 1.0) -> float:
    """KL(P || Q^E) with q^E proportional to (1 + |y_i - y_j|^2)^-1."""
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    c = np.zeros(1)
    _check(lib().ora_euclid_cost(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32), _p(val, _D),
                                 float(exaggeration), _p(c, _D)), "euclid_cost")
    return float(c[0])


def gradient_euclid_exact(Y, rp, col, val, exaggeration: float = 1.0):
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    g = np.zeros_like(Y)
    z = np.zeros(1)
    _check(lib().ora_gradient_euclid_exact(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32),
                                           _p(val, _D), float(exaggeration), _p(g, _D), _p(z, _D)),
           "gradient_euclid_exact")
    return g, float(z[0])


def gradient_euclid_bh(Y, rp, col, val, tree: Tree, theta: float, exaggeration: float = 1.0):
    Y = _f64(Y).reshape(-1, 2)
    rp, col, val = _csr(rp, col, val)
    g = np.zeros_like(Y)
    z = np.zeros(1)
    cnt = np.zeros(4, dtype=np.int64)
    _check(lib().ora_gradient_euclid_bh(_p(Y, _D), Y.shape[0], _p(rp, _I64), _p(col, _I32),
                                        _p(val, _D), float(exaggeration), tree.h, float(theta),
                                        _p(g, _D), _p(z, _D), _p(cnt, _I64)), "gradient_euclid_bh")
    return g, float(z[0]), dict(tests=int(cnt[0]), accepts=int(cnt[1]), pairs=int(cnt[2]),
                                covered=int(cnt[3]))


def hsne_cost(Y, rp, col, val, lam: float, exaggeration: float = 1.0) -> float:
    """h-SNE cost as read: KL(P || Q^E) + lam KL(P || Q^H)."""
    return euclid_cost(Y, rp, col, val, exaggeration) + lam * kl_cost(Y, rp, col, val, exaggeration)


def hsne_gradient_bh(Y, rp, col, val, tree: Tree, theta: float, lam: float,
                     exaggeration: float = 1.0):
    """Euclidean plus lam times hyperbolic gradient; returns (g, Z^E, Z^H)."""
    ge, ze, _ = gradient_euclid_bh(Y, rp, col, val, tree, theta, exaggeration)
    gh, zh, _ = gradient_bh(Y, rp, col, val, tree, theta, exaggeration)
    return ge + lam * gh, ze, zh


def step(Y, update, gains, grad, eta: float, momentum: float, min_gain: float = 0.01,
         boundary_eps: float = 1e-5, metric_power: int = 2):
    """Returns new (Y, update, gains) arrays (inputs are not modified)."""
    Y = _f64(Y).reshape(-1, 2).copy()
    U = _f64(update).reshape(-1, 2).copy()
    G = _f64(gains).reshape(-1, 2).copy()
    g = _f64(grad).reshape(-1, 2)
    _check(lib().ora_step(_p(Y, _D), _p(U, _D), _p(G, _D), _p(g, _D), Y.shape[0], float(eta),
                          float(momentum), float(min_gain), float(boundary_eps), int(metric_power)),
           "step")
    return Y, U, G
