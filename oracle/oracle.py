"""ctypes wrapper for the FP64 CPU oracle (``gmm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.

All functions take numpy arrays on the host.  Samples are D x N column-major,
i.e. a C-contiguous (N, D) array whose row i is sample i (one sample per
column of the paper's data matrix, Sec. 4 API): float64 arrays go to the
FP64-sample entry points (the paper's gmm_diag precision), anything else is
taken as float32.  Parameters
are promoted to float64: ``means`` and ``dcovs`` are (G, D) arrays (row g is
the paper's column g), full covariances are (G, D, D).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.c_int64
_i32 = ctypes.c_int


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
             "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_set_threads.argtypes = [_i32]
        L.oracle_get_threads.restype = _i32
        L.oracle_loglik.argtypes = [_fp, _i64, _i32, _i64, _i32, _i32, _dp, _dp, _dp, _dp, _dp]
        L.oracle_log_p_g.argtypes = [_fp, _i64, _i32, _i64, _i32, _dp, _dp, _i32, _dp]
        L.oracle_responsibilities.argtypes = [_fp, _i64, _i32, _i64, _i32, _i32, _dp, _dp, _dp, _dp]
        L.oracle_em_iter.argtypes = [_fp, _i64, _i32, _i64, _i32, _i32, _dp, _dp, _dp,
                                     ctypes.c_double, _dp, _dp, _dp, _dp, _dp]
        L.oracle_global_stats.argtypes = [_fp, _i64, _i32, _i64, _dp, _dp]
        L.oracle_kmeans_iter.argtypes = [_fp, _i64, _i32, _i64, _i32, _dp, _dp, ctypes.c_double,
                                         _dp, _dp, _dp, _i64p, _i32p, _dp, _dp]
        L.oracle_assign.argtypes = [_fp, _i64, _i32, _i64, _i32, _i32, _dp, _dp, _dp, _i32p]
        L.oracle_seed_spread.argtypes = [_fp, _i64, _i32, _i64, _i32, _dp, _i64, _i64p, _dp]
        L.oracle_kmeans_dists.argtypes = [_fp, _i64, _i32, _i64, _i32, _dp, _dp, _dp]
        for f in ("oracle_loglik", "oracle_log_p_g", "oracle_responsibilities", "oracle_em_iter",
                  "oracle_global_stats", "oracle_kmeans_iter", "oracle_assign",
                  "oracle_seed_spread", "oracle_kmeans_dists"):
            getattr(L, f).restype = _i32
            # FP64-sample twin: the same arguments with X as double*
            g64 = getattr(L, f + "_f64")
            g64.argtypes = [_dp] + list(getattr(L, f).argtypes[1:])
            g64.restype = _i32
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


class OracleError(RuntimeError):
    pass


def _X(X):
    """Samples as a C-contiguous (N, D) array: float64 input stays FP64 (the
    *_f64 entry points), anything else becomes float32."""
    X = np.asarray(X)
    X = np.ascontiguousarray(X, dtype=np.float64 if X.dtype == np.float64 else np.float32)
    if X.ndim != 2:
        raise ValueError("X must be (N, D)")
    return X, X.shape[0], X.shape[1]


def _call(name, X, *args):
    """Call the entry point for X's precision (name, or name_f64 for FP64)."""
    if X.dtype == np.float64:
        return getattr(lib(), name + "_f64")(X.ctypes.data_as(_dp), *args)
    return getattr(lib(), name)(X.ctypes.data_as(_fp), *args)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


NOT_PD = 2
NONFINITE = 1


def _check(rc, what):
    """Negative codes are argument/memory errors; NOT_PD (a covariance that is
    not positive definite) also raises; NONFINITE is returned as a status."""
    if rc < 0 or rc == NOT_PD:
        raise OracleError(f"{what}: error {rc}")
    return rc


def loglik(X, hefts, means, covs, full=False, per_sample=False):
    """Mean log-likelihood (Sec. 4 API avg_log_p) and optionally per-sample values."""
    X, N, D = _X(X)
    G = len(hefts)
    h, m, c = _d(hefts), _d(means), _d(covs)
    out = np.zeros(1)
    ps = np.zeros(N) if per_sample else None
    rc = _call("oracle_loglik", X, N, D, D, G, int(full), _p(h), _p(m), _p(c), _p(out),
                             _p(ps) if per_sample else None)
    _check(rc, "loglik")
    return (float(out[0]), ps) if per_sample else float(out[0])


def log_p_g(X, means, dcovs, g):
    X, N, D = _X(X)
    m, c = _d(means), _d(dcovs)
    out = np.zeros(N)
    _check(_call("oracle_log_p_g", X, N, D, D, m.shape[0], _p(m), _p(c), int(g), _p(out)),
           "log_p_g")
    return out


def responsibilities(X, hefts, means, covs, full=False):
    X, N, D = _X(X)
    G = len(hefts)
    h, m, c = _d(hefts), _d(means), _d(covs)
    out = np.zeros((N, G))
    _check(_call("oracle_responsibilities", X, N, D, D, G, int(full), _p(h), _p(m), _p(c),
                                         _p(out)), "responsibilities")
    return out


@dataclass
class EMResult:
    hefts: np.ndarray
    means: np.ndarray
    covs: np.ndarray
    mean_loglik: float  # of the INPUT parameters
    L: np.ndarray
    status: int


def em_iter(X, hefts, means, covs, var_floor, full=False) -> EMResult:
    X, N, D = _X(X)
    G = len(hefts)
    h, m, c = _d(hefts), _d(means), _d(covs)
    ho, mo, co = np.zeros_like(h), np.zeros_like(m), np.zeros_like(c)
    ll = np.zeros(1)
    L = np.zeros(G)
    rc = _call("oracle_em_iter", X, N, D, D, G, int(full), _p(h), _p(m), _p(c),
                              float(var_floor), _p(ho), _p(mo), _p(co), _p(ll), _p(L))
    _check(rc, "em_iter")
    return EMResult(ho, mo, co, float(ll[0]), L, rc)


def global_stats(X):
    X, N, D = _X(X)
    mean, var = np.zeros(D), np.zeros(D)
    _check(_call("oracle_global_stats", X, N, D, D, _p(mean), _p(var)), "global_stats")
    return mean, var


@dataclass
class KMResult:
    means: np.ndarray
    dcovs: np.ndarray
    hefts: np.ndarray
    counts: np.ndarray
    assign: np.ndarray
    inertia: float  # under the INPUT means
    gap: np.ndarray
    status: int


def kmeans_iter(X, means, lam, var_floor) -> KMResult:
    """One Lloyd iteration; ``lam`` is the per-dimension distance weight
    (ones for Euclidean, 1/global variance for Mahalanobis)."""
    X, N, D = _X(X)
    m = _d(means)
    G = m.shape[0]
    lam = _d(lam)
    mo, co, ho = np.zeros((G, D)), np.zeros((G, D)), np.zeros(G)
    counts = np.zeros(G, dtype=np.int64)
    assign = np.zeros(N, dtype=np.int32)
    inertia = np.zeros(1)
    gap = np.zeros(N)
    rc = _call("oracle_kmeans_iter", X, N, D, D, G, _p(lam), _p(m), float(var_floor),
                                  _p(mo), _p(co), _p(ho), _p(counts, _i64p), _p(assign, _i32p),
                                  _p(inertia), _p(gap))
    _check(rc, "kmeans_iter")
    return KMResult(mo, co, ho, counts, assign, float(inertia[0]), gap, rc)


def kmeans_dists(X, means, lam):
    """(N, G) matrix of k-means distances sum_d lam_d (x_d - mu_gd)^2 (Eq. 19's
    argument with Eq. 20's weights)."""
    X, N, D = _X(X)
    m = _d(means)
    G = m.shape[0]
    out = np.zeros((N, G))
    _check(_call("oracle_kmeans_dists", X, N, D, D, G, _p(_d(lam)), _p(m), _p(out)),
           "kmeans_dists")
    return out


def assign(X, hefts, means, dcovs, mode):
    """mode 0: Euclidean (eucl_dist); mode 1: probabilistic (prob_dist)."""
    X, N, D = _X(X)
    h, m, c = _d(hefts), _d(means), _d(dcovs)
    out = np.zeros(N, dtype=np.int32)
    _check(_call("oracle_assign", X, N, D, D, m.shape[0], int(mode), _p(h), _p(m), _p(c),
                               _p(out, _i32p)), "assign")
    return out


def seed_spread(X, G, first=0, lam=None):
    """Farthest-first seeding (Sec. 4 API static_spread / random_spread): the
    chosen sample indices (G,) and their coordinates (G, D)."""
    X, N, D = _X(X)
    idx = np.zeros(G, dtype=np.int64)
    means = np.zeros((G, D))
    lp = _p(_d(lam)) if lam is not None else None
    _check(_call("oracle_seed_spread", X, N, D, D, int(G), lp, int(first), _p(idx, _i64p),
                                    _p(means)), "seed_spread")
    return idx, means


def maha_lambda(var, var_floor):
    """Per-dimension weight of the global-diagonal Mahalanobis distance (Sec. 3.1,
    Eq. 20): reciprocal of the floored global variance."""
    v = np.maximum(np.asarray(var, dtype=np.float64), var_floor)
    return 1.0 / v
