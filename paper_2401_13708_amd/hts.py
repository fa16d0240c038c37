"""Thin Python binding of libhts.so (the C ABI of include/hts.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.  The
binding raises if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhts.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hts.h")

HTS_F32, HTS_F64 = 0, 1
STATUS = {0: "HTS_OK", -1: "HTS_EINVAL", -2: "HTS_ENOMEM", -3: "HTS_EDEVICE",
          -4: "HTS_ECAPACITY", -5: "HTS_ENUMERIC"}
KCLASS = ["tree", "attract", "traverse", "exact", "finalize", "step", "knn", "items"]


class HTSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code


_lib = None
_P = C.c_void_p
_I32, _I64, _D = C.c_int32, C.c_int64, C.c_double

_SIGS = {
    "hts_last_error": (C.c_char_p, []),
    "hts_version": (C.c_char_p, []),
    "hts_create": (C.c_int, [_I32, C.POINTER(_P)]),
    "hts_destroy": (C.c_int, [_P]),
    "hts_check": (C.c_int, [_P, _P, C.POINTER(C.c_uint32)]),
    "hts_build_affinities": (C.c_int, [_P, _P, _P, _I64, _I32, _I32, _D, _I32, _P, _P, _P, _P,
                                       _I32, _I64, C.POINTER(_I64)]),
    "hts_tree_create": (C.c_int, [_P, _I64, _I32, C.POINTER(_P)]),
    "hts_tree_destroy": (C.c_int, [_P]),
    "hts_build_polar_tree": (C.c_int, [_P, _P, _P, _I64, _I32, _P]),
    "hts_tree_export": (C.c_int, [_P, _P, _P, C.POINTER(_I64), _I64, _P, _P, _P, _P, _P, _P, _P]),
    "hts_gradient_exact": (C.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P, _D, _P, _P, _P]),
    "hts_gradient_exact_noalloc": (C.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P, _D, _P, _P,
                                             _P]),
    "hts_gradient_bh": (C.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P, _D, _P, _D, _P, _P, _P]),
    "hts_gradient_hsne": (C.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P, _D, _D, _P, _D, _P, _P,
                                    _P]),
    "hts_step": (C.c_int, [_P, _P, _P, _P, _P, _P, _I64, _I32, _D, _D, _D, _D, _I32]),
    "hts_iteration_bh": (C.c_int, [_P, _P, _P, _P, _P, _I64, _I32, _P, _P, _P, _D, _P, _D, _P, _P,
                                   _D, _D, _D, _D, _I32]),
    "hts_tree_set_jobs": (C.c_int, [_P, _I32, C.POINTER(_I64)]),
    "hts_gradient_bh_jobs": (C.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P, _P, _P, _D, _P, _P,
                                       _P]),
    "hts_step_jobs": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _I64, _I32, _P, _P, _D, _D, _I32]),
    "hts_jobs_schedule": (C.c_int, [_P, _P, _I32, _P, _I32, _D, _D, _D, _P, _P]),
    "hts_set_item_points": (C.c_int, [_P, _I32]),
    "hts_set_item_list": (C.c_int, [_P, _I32]),
    "hts_set_traversal_launch": (C.c_int, [_P, _I32, _I32]),
    "hts_set_attract_launch": (C.c_int, [_P, _I32]),
    "hts_cosne_terms": (C.c_int, [_P, _P, _P, _I64, _I32, _P, _D, _D, _P]),
    "hts_tree_set_split": (C.c_int, [_P, _I32]),
    "hts_workspace_generation": (C.c_int, [_P, C.POINTER(C.c_uint64)]),
    "hts_timing_enable": (C.c_int, [_P, _I32]),
    "hts_timing_read": (C.c_int, [_P, C.POINTER(_D), C.POINTER(_I64)]),
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/hts.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hts_[a-z_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhts.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().hts_last_error().decode()


def _ck(code: int):
    if code != 0:
        raise HTSError(code, last_error())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dtype(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return HTS_F32
    if t.dtype == torch.float64:
        return HTS_F64
    raise TypeError("float32 or float64 expected, got %s" % t.dtype)


def _dev(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    return t


# traversal counters of one Barnes-Hut call (include/hts.h): six for the whole
# traversal (tests, accepted cells, leaf pairs, wave visits, visits with work,
# points covered), then the same six for its second kernel
STATS_BLOCK = 6
STATS_PER_CALL = 2 * STATS_BLOCK
DEFAULT_ITEM_POINTS = 288  # the library's default work-item size
DEFAULT_ITEM_LIST = 256    # the library's default item-list entries per phase-A wave
DEFAULT_ITEMS_GRID = 0     # the library's default phase-B workgroups (0: automatic) ...
DEFAULT_ITEMS_WAVES = 1    # ... of this many waves
DEFAULT_ATTRACT_LAUNCH = 0  # the attractive rows' launch: 0 automatic, 1 phase A, 2 phase B
ATTRACT_WITH_TOP_AT = 131072  # automatic: beside phase A from this many points in the largest job


def attract_in_items(where: int, largest_job: int) -> bool:
    """Whether the Barnes-Hut gradient computes the attractive rows in the
    traversal's second launch (the library's rule for hts_set_attract_launch)."""
    return where == 2 or (where == 0 and largest_job < ATTRACT_WITH_TOP_AT)


class Context:
    """hts_ctx on one device."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _ck(lib().hts_create(int(device), C.byref(h)))
        self.h = h
        self.device = device
        self.item_points = DEFAULT_ITEM_POINTS
        self.item_list = DEFAULT_ITEM_LIST
        self.traversal_launch = (DEFAULT_ITEMS_GRID, DEFAULT_ITEMS_WAVES)
        self.attract_launch = DEFAULT_ATTRACT_LAUNCH

    def close(self):
        if getattr(self, "h", None):
            lib().hts_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, stream=None) -> int:
        bits = C.c_uint32(0)
        code = lib().hts_check(self.h, _stream(stream), C.byref(bits))
        if code not in (0, -5):
            _ck(code)
        return int(bits.value)

    def set_item_list(self, items_per_wave: int):
        """Item-list entries per phase-A wave (device memory of the traversal)."""
        _ck(lib().hts_set_item_list(self.h, int(items_per_wave)))
        self.item_list = int(items_per_wave)

    def set_traversal_launch(self, workgroups: int = DEFAULT_ITEMS_GRID,
                             waves_per_workgroup: int = DEFAULT_ITEMS_WAVES):
        """Launch shape of the traversal's second kernel (a tuning parameter;
        the result does not depend on it)."""
        _ck(lib().hts_set_traversal_launch(self.h, int(workgroups), int(waves_per_workgroup)))
        self.traversal_launch = (int(workgroups), int(waves_per_workgroup))

    def set_attract_launch(self, where: int = DEFAULT_ATTRACT_LAUNCH):
        """Launch that computes the attractive term: 1 beside phase A, 2 at the
        end of phase B, 0 automatic (a tuning parameter; the result does not
        depend on it)."""
        _ck(lib().hts_set_attract_launch(self.h, int(where)))
        self.attract_launch = int(where)

    def set_item_points(self, s: int):
        """Barnes-Hut work-item size (a tuning parameter)."""
        _ck(lib().hts_set_item_points(self.h, int(s)))
        self.item_points = int(s)

    def generation(self) -> int:
        """Workspace generation: changes when device memory that earlier
        launches referenced is reallocated (captured graphs are then stale)."""
        g = C.c_uint64(0)
        _ck(lib().hts_workspace_generation(self.h, C.byref(g)))
        return int(g.value)

    # ------------------------------------------------------------ timing
    def timing(self, on: bool):
        _ck(lib().hts_timing_enable(self.h, 1 if on else 0))

    def timing_read(self) -> dict:
        ms = (C.c_double * len(KCLASS))()
        cnt = (C.c_int64 * len(KCLASS))()
        _ck(lib().hts_timing_read(self.h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KCLASS)}


class Tree:
    """hts_tree: polar quadtree storage for up to n_max points."""

    def __init__(self, ctx: Context, n_max: int, max_depth: int = 20):
        h = C.c_void_p()
        _ck(lib().hts_tree_create(ctx.h, int(n_max), int(max_depth), C.byref(h)))
        self.h = h
        self.ctx = ctx
        self.n_max = n_max
        self.max_depth = max_depth

    def set_split(self, rule: int):
        """Radial split: 0 equal lengths (eq. (10)), 1 equal areas (eq. (9))."""
        _ck(lib().hts_tree_set_split(self.h, int(rule)))
        self.split_rule = int(rule)

    def set_jobs(self, sizes):
        """Job layout: len(sizes) embeddings of these sizes, side by side."""
        arr = (C.c_int64 * len(sizes))(*[int(v) for v in sizes])
        _ck(lib().hts_tree_set_jobs(self.h, len(sizes), arr))
        self.jobs = [int(v) for v in sizes]

    def close(self):
        if getattr(self, "h", None):
            lib().hts_tree_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_affinities(ctx: Context, X: torch.Tensor, perplexity: float = 30.0, k: int = 90,
                     p_dtype=None, want_knn: bool = True, stream=None):
    """Returns (knn or None, row_ptr, col_idx, p_val) as device tensors."""
    _dev(X, "X")
    n, d = X.shape
    p_dtype = p_dtype or X.dtype
    dev = X.device
    cap = 2 * n * k
    knn = torch.empty((n, k), dtype=torch.int32, device=dev) if want_knn else None
    rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(cap, dtype=torch.int32, device=dev)
    val = torch.empty(cap, dtype=p_dtype, device=dev)
    nnz = C.c_int64(0)
    _ck(lib().hts_build_affinities(ctx.h, _stream(stream), _ptr(X), n, d, _dtype(X),
                                   float(perplexity), int(k), _ptr(knn), _ptr(rp), _ptr(col),
                                   _ptr(val), _dtype(val), cap, C.byref(nnz)))
    m = int(nnz.value)
    return knn, rp, col[:m], val[:m]


def build_polar_tree(ctx: Context, Y: torch.Tensor, tree: Tree, stream=None):
    _dev(Y, "Y")
    _ck(lib().hts_build_polar_tree(ctx.h, _stream(stream), _ptr(Y), Y.shape[0], _dtype(Y), tree.h))


def tree_export(ctx: Context, tree: Tree, n: int, stream=None) -> dict:
    m = C.c_int64(0)
    _ck(lib().hts_tree_export(ctx.h, _stream(stream), tree.h, C.byref(m), 0, None, None, None,
                              None, None, None, None))
    M = int(m.value)
    dev = torch.device("cuda", ctx.device)
    out = dict(count=torch.empty(M, dtype=torch.int32, device=dev),
               depth=torch.empty(M, dtype=torch.int32, device=dev),
               first=torch.empty(M, dtype=torch.int32, device=dev),
               next=torch.empty(M, dtype=torch.int32, device=dev),
               mid=torch.empty((M, 2), dtype=torch.float64, device=dev),
               r_cell=torch.empty(M, dtype=torch.float64, device=dev),
               perm=torch.empty(n, dtype=torch.int32, device=dev))
    _ck(lib().hts_tree_export(ctx.h, _stream(stream), tree.h, C.byref(m), M, _ptr(out["count"]),
                              _ptr(out["depth"]), _ptr(out["first"]), _ptr(out["next"]),
                              _ptr(out["mid"]), _ptr(out["r_cell"]), _ptr(out["perm"])))
    return {k: v.cpu().numpy() for k, v in out.items()}


def _csr_args(Y, row_ptr, col_idx, p_val):
    _dev(row_ptr, "row_ptr", torch.int64)
    _dev(col_idx, "col_idx", torch.int32)
    _dev(p_val, "p_val", Y.dtype)
    if row_ptr.numel() != Y.shape[0] + 1:
        raise ValueError("row_ptr must have n + 1 entries")


def gradient_exact(ctx: Context, Y, row_ptr, col_idx, p_val, exaggeration: float = 1.0,
                   grad=None, z=None, kl=None, stream=None):
    """Exact gradient into grad and Z into z; the cost of eq. (3) into kl (a
    device float64 tensor of one entry) when given."""
    _dev(Y, "Y")
    _csr_args(Y, row_ptr, col_idx, p_val)
    grad = torch.empty_like(Y) if grad is None else grad
    z = torch.empty(1, dtype=torch.float64, device=Y.device) if z is None else z
    if kl is not None:
        _dev(kl, "kl", torch.float64)
    _ck(lib().hts_gradient_exact(ctx.h, _stream(stream), _ptr(Y), Y.shape[0], _dtype(Y),
                                 _ptr(row_ptr), _ptr(col_idx), _ptr(p_val), float(exaggeration),
                                 _ptr(grad), _ptr(z), _ptr(kl)))
    return grad, z


NOALLOC_MAX_N = 65536  # HTS_NOALLOC_MAX_N of include/hts.h


def gradient_exact_noalloc(ctx: Context, Y, row_ptr, col_idx, p_val, grad, z,
                           exaggeration: float = 1.0, kl=None, stream=None):
    """gradient_exact without any device allocation in the library: the
    workspace is the library's fixed per-GPU region (n <= NOALLOC_MAX_N);
    grad, z (and kl) are caller-owned device tensors."""
    _dev(Y, "Y")
    _csr_args(Y, row_ptr, col_idx, p_val)
    _dev(grad, "grad", Y.dtype)
    _dev(z, "z", torch.float64)
    if kl is not None:
        _dev(kl, "kl", torch.float64)
    _ck(lib().hts_gradient_exact_noalloc(ctx.h, _stream(stream), _ptr(Y), Y.shape[0], _dtype(Y),
                                         _ptr(row_ptr), _ptr(col_idx), _ptr(p_val),
                                         float(exaggeration), _ptr(grad), _ptr(z), _ptr(kl)))
    return grad, z


def gradient_bh(ctx: Context, Y, row_ptr, col_idx, p_val, tree: Tree, theta: float = 0.5,
                exaggeration: float = 1.0, grad=None, z=None, stats=None, stream=None):
    _dev(Y, "Y")
    _csr_args(Y, row_ptr, col_idx, p_val)
    grad = torch.empty_like(Y) if grad is None else grad
    z = torch.empty(1, dtype=torch.float64, device=Y.device) if z is None else z
    if stats is not None:
        _dev(stats, "stats", torch.int64)
        if stats.numel() < STATS_PER_CALL:
            raise ValueError("stats needs %d int64 entries" % STATS_PER_CALL)
    _ck(lib().hts_gradient_bh(ctx.h, _stream(stream), _ptr(Y), Y.shape[0], _dtype(Y),
                              _ptr(row_ptr), _ptr(col_idx), _ptr(p_val), float(exaggeration),
                              tree.h, float(theta), _ptr(grad), _ptr(z), _ptr(stats)))
    return grad, z


def gradient_hsne(ctx: Context, Y, row_ptr, col_idx, p_val, tree: Tree, lam: float,
                  theta: float = 0.5, exaggeration: float = 1.0, grad=None, z=None, stats=None,
                  stream=None):
    """h-SNE gradient (Sec. 4-C): the Euclidean Student-t gradient of the disk
    coordinates plus lam times the hyperbolic one, both Barnes-Hut over the
    tree.  z (device float64[2]) receives Z^E and Z^H; stats, if given, holds
    24 int64 counters (Euclidean traversal, then hyperbolic)."""
    _dev(Y, "Y")
    _csr_args(Y, row_ptr, col_idx, p_val)
    grad = torch.empty_like(Y) if grad is None else grad
    z = torch.empty(2, dtype=torch.float64, device=Y.device) if z is None else z
    if stats is not None:
        _dev(stats, "stats", torch.int64)
        if stats.numel() < 2 * STATS_PER_CALL:
            raise ValueError("stats needs %d int64 entries" % (2 * STATS_PER_CALL))
    _ck(lib().hts_gradient_hsne(ctx.h, _stream(stream), _ptr(Y), Y.shape[0], _dtype(Y),
                                _ptr(row_ptr), _ptr(col_idx), _ptr(p_val), float(exaggeration),
                                float(lam), tree.h, float(theta), _ptr(grad), _ptr(z),
                                _ptr(stats)))
    return grad, z


def step(ctx: Context, Y, update, gains, grad, eta: float, momentum: float,
         min_gain: float = 0.01, boundary_eps: float = 1e-5, metric_power: int = 2, stream=None):
    for t, nm in ((Y, "Y"), (update, "update"), (gains, "gains"), (grad, "grad")):
        _dev(t, nm, Y.dtype)
    _ck(lib().hts_step(ctx.h, _stream(stream), _ptr(Y), _ptr(update), _ptr(gains), _ptr(grad),
                       Y.shape[0], _dtype(Y), float(eta), float(momentum), float(min_gain),
                       float(boundary_eps), int(metric_power)))


def iteration_bh(ctx: Context, Y, update, gains, row_ptr, col_idx, p_val, tree: Tree,
                 theta: float, exaggeration: float, eta: float, momentum: float, grad=None, z=None,
                 min_gain: float = 0.01, boundary_eps: float = 1e-5, metric_power: int = 2,
                 stream=None):
    """Tree, Barnes-Hut gradient and step in one call, bit for bit the three
    calls; returns grad, z."""
    for t, nm in ((Y, "Y"), (update, "update"), (gains, "gains")):
        _dev(t, nm, Y.dtype)
    _csr_args(Y, row_ptr, col_idx, p_val)
    grad = torch.empty_like(Y) if grad is None else grad
    z = torch.empty(1, dtype=torch.float64, device=Y.device) if z is None else z
    _ck(lib().hts_iteration_bh(ctx.h, _stream(stream), _ptr(Y), _ptr(update), _ptr(gains),
                               Y.shape[0], _dtype(Y), _ptr(row_ptr), _ptr(col_idx), _ptr(p_val),
                               float(exaggeration), tree.h, float(theta), _ptr(grad), _ptr(z),
                               float(eta), float(momentum), float(min_gain), float(boundary_eps),
                               int(metric_power)))
    return grad, z


def gradient_bh_jobs(ctx: Context, Y, row_ptr, col_idx, p_val, tree: Tree, exaggeration,
                     theta: float = 0.5, grad=None, z=None, stats=None, stream=None):
    """Barnes-Hut gradient of every job of the tree's layout; exaggeration
    and z are device float64 tensors with one entry per job."""
    _dev(Y, "Y")
    _csr_args(Y, row_ptr, col_idx, p_val)
    nj = len(tree.jobs)
    _dev(exaggeration, "exaggeration", torch.float64)
    if exaggeration.numel() != nj:
        raise ValueError("exaggeration needs one entry per job")
    grad = torch.empty_like(Y) if grad is None else grad
    z = torch.empty(nj, dtype=torch.float64, device=Y.device) if z is None else z
    if stats is not None:
        _dev(stats, "stats", torch.int64)
        if stats.numel() < STATS_PER_CALL:
            raise ValueError("stats needs %d int64 entries" % STATS_PER_CALL)
    _ck(lib().hts_gradient_bh_jobs(ctx.h, _stream(stream), _ptr(Y), Y.shape[0], _dtype(Y),
                                   _ptr(row_ptr), _ptr(col_idx), _ptr(p_val), _ptr(exaggeration),
                                   tree.h, float(theta), _ptr(grad), _ptr(z), _ptr(stats)))
    return grad, z


def step_jobs(ctx: Context, tree: Tree, Y, update, gains, grad, eta, momentum,
              min_gain: float = 0.01, boundary_eps: float = 1e-5, metric_power: int = 2,
              stream=None):
    """Riemannian step of every job; eta and momentum: device float64, one per job."""
    for t, nm in ((Y, "Y"), (update, "update"), (gains, "gains"), (grad, "grad")):
        _dev(t, nm, Y.dtype)
    for t, nm in ((eta, "eta"), (momentum, "momentum")):
        _dev(t, nm, torch.float64)
    _ck(lib().hts_step_jobs(ctx.h, _stream(stream), tree.h, _ptr(Y), _ptr(update), _ptr(gains),
                            _ptr(grad), Y.shape[0], _dtype(Y), _ptr(eta), _ptr(momentum),
                            float(min_gain), float(boundary_eps), int(metric_power)))


def jobs_schedule(ctx: Context, it, ee_iters: int, exaggeration: float, momentum_early: float,
                  momentum_late: float, ex_out, mu_out, stream=None):
    """Per-job optimiser schedule on the device; advances the int32 counters it."""
    _dev(it, "it", torch.int32)
    _dev(ex_out, "ex_out", torch.float64)
    _dev(mu_out, "mu_out", torch.float64)
    _ck(lib().hts_jobs_schedule(ctx.h, _stream(stream), it.numel(), _ptr(it), int(ee_iters),
                                float(exaggeration), float(momentum_early), float(momentum_late),
                                _ptr(ex_out), _ptr(mu_out)))


def cosne_terms(ctx: Context, Y, xnorm2, lambda1: float, lambda2: float, grad, stream=None):
    """CO-SNE gradient from the KL gradient in grad (in place)."""
    _dev(Y, "Y")
    _dev(grad, "grad", Y.dtype)
    _dev(xnorm2, "xnorm2", torch.float64)
    _ck(lib().hts_cosne_terms(ctx.h, _stream(stream), _ptr(Y), Y.shape[0], _dtype(Y),
                              _ptr(xnorm2), float(lambda1), float(lambda2), _ptr(grad)))
    return grad
