"""Python binding of the C ABI in include/gmm.h (libgmm.so, built in-tree).

Argument marshalling only: every function checks the torch tensors it is given
(device, dtype, shape, contiguity), passes their device pointers and the
current HIP stream to the C entry point of the same name, and raises
``GmmError`` on a non-zero return code.  All arithmetic runs in the HIP
kernels; there is no fallback: if the library is missing, importing the
binding's functions raises.

Shapes: X is a float32 (N, D) tensor whose rows are samples (the paper's
D x N column-major data matrix); a row stride >= D is allowed.  means and
diagonal covariances are (G, D) float32 (row g = column g of the paper's
matrices), full covariances (G, D, D), hefts (G,).
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmm.so")
HEADER = os.path.join(HERE, "..", "include", "gmm.h")

GMM_OK, GMM_EINVAL, GMM_EHIP = 0, -1, -2
GMM_DEV_OK, GMM_DEV_NONFINITE, GMM_DEV_NOTPD, GMM_DEV_BADDESC = 0, 1, 2, 4
SEED_SUBSET, SEED_SPREAD = 0, 1
COV_DIAG, COV_FULL = 0, 1
DIST_EUCL, DIST_MAHA = 0, 1
ASSIGN_EUCL, ASSIGN_PROB = 0, 1
PREC_FP32, PREC_BF16X3 = 0, 1
(PATH_ONEPASS_BF16X3, PATH_ONEPASS_FP32, PATH_WIDE_FP64, PATH_GENERIC, PATH_FULL_FP64,
 PATH_FULL_GENERIC, PATH_SLICED_BF16X3) = range(1, 8)


class GmmError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed with code {code} ({_status_string(code)})")
        self.code = code


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f32 = ctypes.c_float
_sz = ctypes.c_size_t

_SIGS = {
    "gmm_version": ([], _i32),
    "gmm_status_string": ([_i32], ctypes.c_char_p),
    "gmm_workspace_bytes": ([_i64, _i32, _i32, _i32, _i32], _sz),
    "gmm_global_stats": ([_vp, _i64, _i32, _i64, _vp, _vp, _vp, _sz, _vp], _i32),
    "gmm_kmeans_iter": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, _f32, _vp, _vp, _vp, _vp, _vp,
                         _vp, _i32, _vp, _vp, _vp, _sz, _vp], _i32),
    "gmm_em_iter": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _f32, _i32, _vp, _vp, _vp,
                     _vp, _sz, _vp], _i32),
    "gmm_loglik": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp,
                    _sz, _vp], _i32),
    "gmm_seed_means": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, _f32, _i64, _vp, _vp, _vp, _vp,
                        _sz, _vp], _i32),
    "gmm_log_p_gaussian": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                            _sz, _vp], _i32),
    "gmm_assign": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                    _vp], _i32),
    "gmm_em_iter_noalloc": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _f32, _i32, _vp,
                             _vp, _vp, _vp], _i32),
    "gmm_workspace_bytes_f64": ([_i64, _i32, _i32], _sz),
    "gmm_global_stats_f64": ([_vp, _i64, _i32, _i64, _vp, _vp, _vp, _sz, _vp], _i32),
    "gmm_kmeans_iter_f64": ([_vp, _i64, _i32, _i64, _i32, _i32, _vp, ctypes.c_double, _vp, _vp,
                             _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "gmm_em_iter_f64": ([_vp, _i64, _i32, _i64, _i32, _vp, _vp, _vp, ctypes.c_double, _vp, _vp,
                         _vp, _sz, _vp], _i32),
    "gmm_loglik_f64": ([_vp, _i64, _i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                        _vp], _i32),
    "gmm_em_path": ([_i32, _i32, _i32, _i32], _i32),
    "gmm_kmeans_path": ([_i32, _i32, _i32], _i32),
    "gmm_profile_enable": ([_i32], _i32),
    "gmm_profile_read": ([_i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)], _i32),
}

PROF_EM, PROF_KM_ASSIGN, PROF_KM_ACCUM, PROF_LOGLIK, PROF_STATS, PROF_BATCHED = range(6)

_lib = None


def library():
    """Load libgmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/gmm.h."""
    with open(HEADER) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gmm_[a-z0-9_]+)\s*\(", txt)))


def _status_string(code):
    try:
        return library().gmm_status_string(int(code)).decode()
    except Exception:
        return "?"


def _check(fn, rc):
    if rc != GMM_OK:
        raise GmmError(fn, rc)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor", optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _xptr(X):
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2:
        raise ValueError("X must be a float32 (N, D) device tensor")
    N, D = X.shape
    ldx = X.stride(0) if N > 1 else D
    if (D > 1 and X.stride(1) != 1) or ldx < D:
        raise ValueError("X rows must be contiguous samples with row stride >= D")
    return ctypes.c_void_p(X.data_ptr()), int(N), int(D), int(ldx)


def gmm_workspace_bytes(N, D, G, cov=COV_DIAG, prec=PREC_FP32):
    return int(library().gmm_workspace_bytes(int(N), int(D), int(G), int(cov), int(prec)))


def workspace(N, D, G, cov=COV_DIAG, prec=PREC_FP32, device="cuda"):
    """A device byte buffer large enough for every entry point at this shape."""
    n = gmm_workspace_bytes(N, D, G, cov, prec)
    if n == 0:
        raise GmmError("gmm_workspace_bytes", GMM_EINVAL)
    return torch.empty(n, dtype=torch.uint8, device=device)


def _ws(ws):
    if ws is None or ws.dtype != torch.uint8 or not ws.is_cuda:
        raise ValueError("ws must be a uint8 device tensor from workspace()")
    return ctypes.c_void_p(ws.data_ptr()), int(ws.numel())


def gmm_global_stats(X, mean_out, var_out, ws, stream=None):
    xp, N, D, ldx = _xptr(X)
    wp, wn = _ws(ws)
    rc = library().gmm_global_stats(xp, N, D, ldx, _ptr(mean_out, torch.float64, (D,), "mean_out"),
                                    _ptr(var_out, torch.float64, (D,), "var_out"), wp, wn,
                                    _stream(stream))
    _check("gmm_global_stats", rc)


def gmm_kmeans_iter(X, dist, gvar, var_floor, means, dcovs, hefts, counts, assign, inertia, prec,
                    n_recomputed, dev_status, ws, stream=None):
    xp, N, D, ldx = _xptr(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    rc = library().gmm_kmeans_iter(
        xp, N, D, ldx, G, int(dist), _ptr(gvar, torch.float64, (D,), "gvar", optional=True),
        float(var_floor), _ptr(means, torch.float32, (G, D), "means"),
        _ptr(dcovs, torch.float32, (G, D), "dcovs"), _ptr(hefts, torch.float32, (G,), "hefts"),
        _ptr(counts, torch.int64, (G,), "counts"),
        _ptr(assign, torch.int32, (N,), "assign", optional=True),
        _ptr(inertia, torch.float64, (1,), "inertia"), int(prec),
        _ptr(n_recomputed, torch.int64, (1,), "n_recomputed", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream))
    _check("gmm_kmeans_iter", rc)


def _covshape(cov, G, D):
    return (G, D, D) if cov == COV_FULL else (G, D)


def gmm_em_iter(X, cov, hefts, means, covs, var_floor, prec, mean_loglik, n_recomputed,
                dev_status, ws, stream=None):
    xp, N, D, ldx = _xptr(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    rc = library().gmm_em_iter(
        xp, N, D, ldx, G, int(cov), _ptr(hefts, torch.float32, (G,), "hefts"),
        _ptr(means, torch.float32, (G, D), "means"),
        _ptr(covs, torch.float32, _covshape(cov, G, D), "covs"), float(var_floor), int(prec),
        _ptr(mean_loglik, torch.float64, (1,), "mean_loglik"),
        _ptr(n_recomputed, torch.int64, (1,), "n_recomputed", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream))
    _check("gmm_em_iter", rc)


NOALLOC_SCRATCH_BYTES = 128 << 20


def gmm_em_iter_noalloc(X, cov, hefts, means, covs, var_floor, prec, mean_loglik, n_recomputed,
                        dev_status, stream=None):
    """gmm_em_iter without a workspace (the library's static per-GPU scratch)."""
    xp, N, D, ldx = _xptr(X)
    G = means.shape[0]
    rc = library().gmm_em_iter_noalloc(
        xp, N, D, ldx, G, int(cov), _ptr(hefts, torch.float32, (G,), "hefts"),
        _ptr(means, torch.float32, (G, D), "means"),
        _ptr(covs, torch.float32, _covshape(cov, G, D), "covs"), float(var_floor), int(prec),
        _ptr(mean_loglik, torch.float64, (1,), "mean_loglik"),
        _ptr(n_recomputed, torch.int64, (1,), "n_recomputed", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), _stream(stream))
    _check("gmm_em_iter_noalloc", rc)


def gmm_loglik(X, cov, hefts, means, covs, prec, mean_loglik, per_sample, dev_status, ws,
               stream=None):
    xp, N, D, ldx = _xptr(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    rc = library().gmm_loglik(
        xp, N, D, ldx, G, int(cov), _ptr(hefts, torch.float32, (G,), "hefts"),
        _ptr(means, torch.float32, (G, D), "means"),
        _ptr(covs, torch.float32, _covshape(cov, G, D), "covs"), int(prec),
        _ptr(mean_loglik, torch.float64, (1,), "mean_loglik"),
        _ptr(per_sample, torch.float32, (N,), "per_sample", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream))
    _check("gmm_loglik", rc)


def gmm_seed_means(X, mode, means, dev_status, ws, gvar=None, var_floor=0.0, first=0, idx=None,
                   stream=None):
    """Initial means into means (float32 (G, D)): SEED_SUBSET (idx: int64 (G,) device
    indices, or None for floor(g N / G)) or SEED_SPREAD (farthest-first from sample
    `first`; gvar: float64 (D,) global variances for the Mahalanobis weights)."""
    xp, N, D, ldx = _xptr(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    rc = library().gmm_seed_means(
        xp, N, D, ldx, G, int(mode), _ptr(gvar, torch.float64, (D,), "gvar", optional=True),
        float(var_floor), int(first), _ptr(idx, torch.int64, (G,), "idx", optional=True),
        _ptr(means, torch.float32, (G, D), "means"),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream))
    _check("gmm_seed_means", rc)


def gmm_log_p_gaussian(X, g, means, dcovs, mean_out, per_sample, dev_status, ws, stream=None):
    """Log-density under Gaussian g alone (no weight): mean_out (float64 [1]) and/or
    per_sample (float32 [N]); at least one of them."""
    xp, N, D, ldx = _xptr(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    rc = library().gmm_log_p_gaussian(
        xp, N, D, ldx, G, int(g), _ptr(means, torch.float32, (G, D), "means"),
        _ptr(dcovs, torch.float32, (G, D), "dcovs"),
        _ptr(mean_out, torch.float64, (1,), "mean_out", optional=True),
        _ptr(per_sample, torch.float32, (N,), "per_sample", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream))
    _check("gmm_log_p_gaussian", rc)


def gmm_assign(X, mode, hefts, means, dcovs, assign, hist, dev_status, ws, stream=None):
    xp, N, D, ldx = _xptr(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    rc = library().gmm_assign(
        xp, N, D, ldx, G, int(mode), _ptr(hefts, torch.float32, (G,), "hefts", optional=True),
        _ptr(means, torch.float32, (G, D), "means"),
        _ptr(dcovs, torch.float32, (G, D), "dcovs", optional=True),
        _ptr(assign, torch.int32, (N,), "assign"),
        _ptr(hist, torch.int64, (G,), "hist", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream))
    _check("gmm_assign", rc)


# ---- FP64 data (gmm_*_f64): X float64 (N, D), parameters float64 -----------

def _xptr64(X):
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float64 or X.dim() != 2:
        raise ValueError("X must be a float64 (N, D) device tensor")
    N, D = X.shape
    ldx = X.stride(0) if N > 1 else D
    if (D > 1 and X.stride(1) != 1) or ldx < D:
        raise ValueError("X rows must be contiguous samples with row stride >= D")
    return ctypes.c_void_p(X.data_ptr()), int(N), int(D), int(ldx)


def gmm_workspace_bytes_f64(N, D, G):
    return int(library().gmm_workspace_bytes_f64(int(N), int(D), int(G)))


def workspace_f64(N, D, G, device="cuda"):
    n = gmm_workspace_bytes_f64(N, D, G)
    if n == 0:
        raise GmmError("gmm_workspace_bytes_f64", GMM_EINVAL)
    return torch.empty(n, dtype=torch.uint8, device=device)


def gmm_global_stats_f64(X, mean_out, var_out, ws, stream=None):
    xp, N, D, ldx = _xptr64(X)
    wp, wn = _ws(ws)
    _check("gmm_global_stats_f64", library().gmm_global_stats_f64(
        xp, N, D, ldx, _ptr(mean_out, torch.float64, (D,), "mean_out"),
        _ptr(var_out, torch.float64, (D,), "var_out"), wp, wn, _stream(stream)))


def gmm_kmeans_iter_f64(X, dist, gvar, var_floor, means, dcovs, hefts, counts, assign, inertia,
                        n_recomputed, dev_status, ws, stream=None):
    xp, N, D, ldx = _xptr64(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    f = torch.float64
    _check("gmm_kmeans_iter_f64", library().gmm_kmeans_iter_f64(
        xp, N, D, ldx, G, int(dist), _ptr(gvar, f, (D,), "gvar", optional=True),
        float(var_floor), _ptr(means, f, (G, D), "means"), _ptr(dcovs, f, (G, D), "dcovs"),
        _ptr(hefts, f, (G,), "hefts"), _ptr(counts, torch.int64, (G,), "counts"),
        _ptr(assign, torch.int32, (N,), "assign", optional=True),
        _ptr(inertia, f, (1,), "inertia"),
        _ptr(n_recomputed, torch.int64, (1,), "n_recomputed", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream)))


def gmm_em_iter_f64(X, hefts, means, dcovs, var_floor, mean_loglik, dev_status, ws, stream=None):
    xp, N, D, ldx = _xptr64(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    f = torch.float64
    _check("gmm_em_iter_f64", library().gmm_em_iter_f64(
        xp, N, D, ldx, G, _ptr(hefts, f, (G,), "hefts"), _ptr(means, f, (G, D), "means"),
        _ptr(dcovs, f, (G, D), "dcovs"), float(var_floor), _ptr(mean_loglik, f, (1,), "mean_loglik"),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream)))


def gmm_loglik_f64(X, hefts, means, dcovs, mean_loglik, per_sample, dev_status, ws, stream=None):
    xp, N, D, ldx = _xptr64(X)
    G = means.shape[0]
    wp, wn = _ws(ws)
    f = torch.float64
    _check("gmm_loglik_f64", library().gmm_loglik_f64(
        xp, N, D, ldx, G, _ptr(hefts, f, (G,), "hefts"), _ptr(means, f, (G, D), "means"),
        _ptr(dcovs, f, (G, D), "dcovs"), _ptr(mean_loglik, f, (1,), "mean_loglik"),
        _ptr(per_sample, f, (N,), "per_sample", optional=True),
        _ptr(dev_status, torch.int32, (1,), "dev_status"), wp, wn, _stream(stream)))


def gmm_em_path(D, G, cov=COV_DIAG, prec=PREC_FP32):
    """Kernel family (PATH_*) that gmm_em_iter / gmm_loglik run for this shape."""
    rc = library().gmm_em_path(int(D), int(G), int(cov), int(prec))
    if rc < 0:
        raise GmmError("gmm_em_path", rc)
    return rc


def gmm_kmeans_path(D, G, prec=PREC_FP32):
    """Kernel family (PATH_*) that gmm_kmeans_iter runs for this shape."""
    rc = library().gmm_kmeans_path(int(D), int(G), int(prec))
    if rc < 0:
        raise GmmError("gmm_kmeans_path", rc)
    return rc


def gmm_profile_enable(on=True):
    _check("gmm_profile_enable", library().gmm_profile_enable(1 if on else 0))


def gmm_profile_read(kind):
    """(total milliseconds, launches) recorded for a kernel kind."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check("gmm_profile_read", library().gmm_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ---- many models (gmm_*_batched) ---------------------------------------------

class _Desc(ctypes.Structure):
    """Mirror of gmm_model_desc (96 bytes, 8-byte aligned)."""
    _fields_ = [("X", _vp), ("N", _i64), ("G", _i32), ("reserved", _i32), ("hefts", _vp),
                ("means", _vp), ("covs", _vp), ("counts", _vp), ("assign", _vp),
                ("loglik", _vp), ("inertia", _vp), ("gvar", _vp), ("dev_status", _vp)]


assert ctypes.sizeof(_Desc) == 96

_SIGS.update({
    "gmm_batched_workspace_bytes": ([_i32, _vp, _vp, _i32, _i32], _sz),
    "gmm_em_iter_batched": ([_vp, _i32, _vp, _vp, _i32, _f32, _i32, _i32, _vp, _sz, _vp], _i32),
    "gmm_loglik_batched": ([_vp, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _sz, _vp], _i32),
    "gmm_kmeans_iter_batched": ([_vp, _i32, _vp, _vp, _i32, _i32, _f32, _i32, _vp, _sz, _vp],
                                _i32),
    "gmm_global_stats_batched": ([_vp, _i32, _i32, _vp, _vp, _vp], _i32),
    "gmm_batched_autotune": ([_vp, _i32, _vp, _vp, _i32, _i32, _vp, _sz, _vp,
                              ctypes.POINTER(_i32)], _i32),
    "gmm_autotune_cache_size": ([], _i32),
    "gmm_autotune_cache_clear": ([], _i32),
})


class ModelBatch:
    """Many independent diagonal models sharing D, stored flat on the device.

    ``Xs`` is a list of contiguous float32 (N_m, D) device tensors (kept
    referenced: the descriptors point into them) and ``Gs`` the component
    counts.  Parameters of model m are views into flat arrays:
    ``hefts[m]`` (G_m,), ``means[m]`` / ``covs[m]`` (G_m, D), ``counts[m]``
    (G_m,) int64, ``assign[m]`` (N_m,) int32; per-model scalars are the rows
    of ``loglik``, ``inertia`` (float64) and ``dev_status`` (int32); ``gvar``
    is (n_models, D) float64.  The descriptor array is built once; the
    tensors never move, so batched calls on it can be captured into a graph.
    """

    def __init__(self, Xs, Gs, device="cuda"):
        if len(Xs) != len(Gs) or not Xs:
            raise ValueError("need one G per model and at least one model")
        D = int(Xs[0].shape[1])
        for X in Xs:
            if (X.dtype != torch.float32 or X.dim() != 2 or X.shape[1] != D
                    or not X.is_contiguous() or not X.is_cuda or X.shape[0] < 1):
                raise ValueError("every X must be a contiguous float32 (N>=1, D) device tensor")
        self.D = D
        self.n_models = len(Xs)
        self.Xs = list(Xs)
        self.Ns = [int(X.shape[0]) for X in Xs]
        self.Gs = [int(g) for g in Gs]
        self.Gmax = max(self.Gs)
        g_off = [0]
        for g in self.Gs:
            g_off.append(g_off[-1] + g)
        n_off = [0]
        for n in self.Ns:
            n_off.append(n_off[-1] + n)
        self.g_off, self.n_off = g_off, n_off
        kw = dict(device=device)
        self.hefts_flat = torch.zeros(g_off[-1], dtype=torch.float32, **kw)
        self.means_flat = torch.zeros(g_off[-1], D, dtype=torch.float32, **kw)
        self.covs_flat = torch.ones(g_off[-1], D, dtype=torch.float32, **kw)
        self.counts_flat = torch.zeros(g_off[-1], dtype=torch.int64, **kw)
        self.assign_flat = torch.zeros(n_off[-1], dtype=torch.int32, **kw)
        self.loglik = torch.zeros(self.n_models, dtype=torch.float64, **kw)
        self.inertia = torch.zeros(self.n_models, dtype=torch.float64, **kw)
        self.gvar = torch.ones(self.n_models, D, dtype=torch.float64, **kw)
        self.gmean = torch.zeros(self.n_models, D, dtype=torch.float64, **kw)
        self.dev_status = torch.zeros(self.n_models, dtype=torch.int32, **kw)
        sl = lambda t, m, off: t[off[m]:off[m + 1]]
        self.hefts = [sl(self.hefts_flat, m, g_off) for m in range(self.n_models)]
        self.means = [sl(self.means_flat, m, g_off) for m in range(self.n_models)]
        self.covs = [sl(self.covs_flat, m, g_off) for m in range(self.n_models)]
        self.counts = [sl(self.counts_flat, m, g_off) for m in range(self.n_models)]
        self.assign = [sl(self.assign_flat, m, n_off) for m in range(self.n_models)]
        arr = (_Desc * self.n_models)()
        e64, e32 = 8, 4
        for m in range(self.n_models):
            d = arr[m]
            d.X = self.Xs[m].data_ptr()
            d.N = self.Ns[m]
            d.G = self.Gs[m]
            d.reserved = 0
            d.hefts = self.hefts_flat.data_ptr() + e32 * g_off[m]
            d.means = self.means_flat.data_ptr() + e32 * D * g_off[m]
            d.covs = self.covs_flat.data_ptr() + e32 * D * g_off[m]
            d.counts = self.counts_flat.data_ptr() + e64 * g_off[m]
            d.assign = self.assign_flat.data_ptr() + e32 * n_off[m]
            d.loglik = self.loglik.data_ptr() + e64 * m
            d.inertia = self.inertia.data_ptr() + e64 * m
            d.gvar = self.gvar.data_ptr() + e64 * D * m
            d.dev_status = self.dev_status.data_ptr() + e32 * m
        host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
        self.desc = host.to(device)
        self._Ns = (_i64 * self.n_models)(*self.Ns)
        self._Gs = (_i32 * self.n_models)(*self.Gs)

    def _args(self):
        return ctypes.c_void_p(self.desc.data_ptr()), self.n_models, self._Ns, self._Gs, self.D

    def workspace(self, chunk=1024):
        n = library().gmm_batched_workspace_bytes(self.n_models, self._Ns, self._Gs, self.D,
                                                  int(chunk))
        if n == 0:
            raise GmmError("gmm_batched_workspace_bytes", GMM_EINVAL)
        return torch.empty(int(n), dtype=torch.uint8, device=self.desc.device)

    def set_params(self, m, hefts, means, covs):
        self.hefts[m].copy_(hefts)
        self.means[m].copy_(means)
        self.covs[m].copy_(covs)


def gmm_batched_workspace_bytes(batch, chunk):
    return int(library().gmm_batched_workspace_bytes(batch.n_models, batch._Ns, batch._Gs,
                                                     batch.D, int(chunk)))


def gmm_em_iter_batched(batch, var_floor, prec, chunk, ws, stream=None):
    wp, wn = _ws(ws)
    rc = library().gmm_em_iter_batched(*batch._args(), float(var_floor), int(prec), int(chunk),
                                       wp, wn, _stream(stream))
    _check("gmm_em_iter_batched", rc)


def gmm_loglik_batched(batch, prec, chunk, ws, stream=None):
    wp, wn = _ws(ws)
    rc = library().gmm_loglik_batched(*batch._args(), int(prec), int(chunk), wp, wn,
                                      _stream(stream))
    _check("gmm_loglik_batched", rc)


def gmm_kmeans_iter_batched(batch, dist, var_floor, chunk, ws, stream=None):
    wp, wn = _ws(ws)
    rc = library().gmm_kmeans_iter_batched(*batch._args(), int(dist), float(var_floor),
                                           int(chunk), wp, wn, _stream(stream))
    _check("gmm_kmeans_iter_batched", rc)


def gmm_global_stats_batched(batch, mean_out, var_out, stream=None):
    shape = (batch.n_models, batch.D)
    rc = library().gmm_global_stats_batched(
        ctypes.c_void_p(batch.desc.data_ptr()), batch.n_models, batch.D,
        _ptr(mean_out, torch.float64, shape, "mean_out"),
        _ptr(var_out, torch.float64, shape, "var_out"), _stream(stream))
    _check("gmm_global_stats_batched", rc)


def gmm_batched_autotune(batch, prec, ws, stream=None):
    wp, wn = _ws(ws)
    best = _i32(0)
    rc = library().gmm_batched_autotune(*batch._args(), int(prec), wp, wn, _stream(stream),
                                        ctypes.byref(best))
    _check("gmm_batched_autotune", rc)
    return int(best.value)


def gmm_autotune_cache_size():
    return int(library().gmm_autotune_cache_size())


def gmm_autotune_cache_clear():
    _check("gmm_autotune_cache_clear", library().gmm_autotune_cache_clear())
