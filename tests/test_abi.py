"""The C ABI library loads and exports every function include/gmm.h declares;
host-side argument validation rejects bad calls before any launch.  Runs on
the CPU: no call here reaches a kernel launch."""
import ctypes
import os

import pytest

from paper_1707_09094_amd import gmm

pytestmark = pytest.mark.skipif(not os.path.exists(gmm.LIB_PATH), reason="libgmm.so not built")


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(gmm.LIB_PATH)
    names = gmm.header_functions()
    assert "gmm_em_iter" in names and "gmm_kmeans_iter" in names and "gmm_loglik" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings():
    L = gmm.library()
    assert L.gmm_version() >= 1
    assert L.gmm_status_string(gmm.GMM_EINVAL).decode() == "invalid argument"


def test_workspace_bytes():
    assert gmm.gmm_workspace_bytes(1000, 4, 4) > 0
    big = gmm.gmm_workspace_bytes(1_000_000, 100, 100, gmm.COV_DIAG, gmm.PREC_BF16X3)
    assert big >= 1_000_000 * 4  # holds at least the k-means assignment scratch
    assert gmm.gmm_workspace_bytes(0, 4, 4) == 0
    assert gmm.gmm_workspace_bytes(10, 0, 4) == 0
    assert gmm.gmm_workspace_bytes(10, 4, 0) == 0
    assert gmm.gmm_workspace_bytes(10, 4, 4, cov=7) == 0
    assert gmm.gmm_workspace_bytes(10, 4, 4, prec=9) == 0
    assert gmm.gmm_workspace_bytes(10, 129, 4, cov=gmm.COV_FULL) == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def test_null_and_shape_arguments_rejected_on_host():
    L = gmm.library()
    ws = ctypes.c_void_p(0x100000)
    # null X
    assert L.gmm_global_stats(None, 10, 4, 4, FAKE, FAKE, ws, 1 << 30, None) == gmm.GMM_EINVAL
    # ldx < D
    assert L.gmm_global_stats(FAKE, 10, 4, 3, FAKE, FAKE, ws, 1 << 30, None) == gmm.GMM_EINVAL
    # N < 1
    assert L.gmm_em_iter(FAKE, 0, 4, 4, 2, 0, FAKE, FAKE, FAKE, 0.0, 0, FAKE, None, FAKE, ws,
                         1 << 30, None) == gmm.GMM_EINVAL
    # unknown covariance type / precision
    assert L.gmm_em_iter(FAKE, 10, 4, 4, 2, 5, FAKE, FAKE, FAKE, 0.0, 0, FAKE, None, FAKE, ws,
                         1 << 30, None) == gmm.GMM_EINVAL
    assert L.gmm_loglik(FAKE, 10, 4, 4, 2, 0, FAKE, FAKE, FAKE, 3, FAKE, None, FAKE, ws, 1 << 30,
                        None) == gmm.GMM_EINVAL
    # Mahalanobis k-means without global variances
    assert L.gmm_kmeans_iter(FAKE, 10, 4, 4, 2, gmm.DIST_MAHA, None, 0.0, FAKE, FAKE, FAKE, FAKE,
                             None, FAKE, 0, None, FAKE, ws, 1 << 30, None) == gmm.GMM_EINVAL
    # negative floor
    assert L.gmm_kmeans_iter(FAKE, 10, 4, 4, 2, gmm.DIST_EUCL, None, -1.0, FAKE, FAKE, FAKE, FAKE,
                             None, FAKE, 0, None, FAKE, ws, 1 << 30, None) == gmm.GMM_EINVAL
    # workspace too small / misaligned / missing
    assert L.gmm_em_iter(FAKE, 10, 4, 4, 2, 0, FAKE, FAKE, FAKE, 0.0, 0, FAKE, None, FAKE, ws, 16,
                         None) == gmm.GMM_EINVAL
    assert L.gmm_em_iter(FAKE, 10, 4, 4, 2, 0, FAKE, FAKE, FAKE, 0.0, 0, FAKE, None, FAKE,
                         ctypes.c_void_p(0x100010), 1 << 30, None) == gmm.GMM_EINVAL
    assert L.gmm_em_iter(FAKE, 10, 4, 4, 2, 0, FAKE, FAKE, FAKE, 0.0, 0, FAKE, None, FAKE, None,
                         1 << 30, None) == gmm.GMM_EINVAL
    # assign: unknown mode, prob mode without covariances
    assert L.gmm_assign(FAKE, 10, 4, 4, 2, 9, FAKE, FAKE, FAKE, FAKE, None, FAKE, ws, 1 << 30,
                        None) == gmm.GMM_EINVAL
    assert L.gmm_assign(FAKE, 10, 4, 4, 2, gmm.ASSIGN_PROB, FAKE, FAKE, None, FAKE, None, FAKE,
                        ws, 1 << 30, None) == gmm.GMM_EINVAL
    # seeding: unknown mode, spread start out of range, negative floor
    assert L.gmm_seed_means(FAKE, 10, 4, 4, 2, 7, None, 0.0, 0, None, FAKE, FAKE, ws, 1 << 30,
                            None) == gmm.GMM_EINVAL
    assert L.gmm_seed_means(FAKE, 10, 4, 4, 2, gmm.SEED_SPREAD, None, 0.0, 10, None, FAKE, FAKE,
                            ws, 1 << 30, None) == gmm.GMM_EINVAL
    assert L.gmm_seed_means(FAKE, 10, 4, 4, 2, gmm.SEED_SPREAD, None, -1.0, 0, None, FAKE, FAKE,
                            ws, 1 << 30, None) == gmm.GMM_EINVAL
    # log_p(X, g): g out of range, negative g, no output requested
    assert L.gmm_log_p_gaussian(FAKE, 10, 4, 4, 2, 2, FAKE, FAKE, FAKE, None, FAKE, ws, 1 << 30,
                                None) == gmm.GMM_EINVAL
    assert L.gmm_log_p_gaussian(FAKE, 10, 4, 4, 2, -1, FAKE, FAKE, FAKE, None, FAKE, ws, 1 << 30,
                                None) == gmm.GMM_EINVAL
    assert L.gmm_log_p_gaussian(FAKE, 10, 4, 4, 2, 0, FAKE, FAKE, None, None, FAKE, ws, 1 << 30,
                                None) == gmm.GMM_EINVAL
    # full covariance beyond the supported dimension
    assert L.gmm_em_iter(FAKE, 10, 200, 200, 2, gmm.COV_FULL, FAKE, FAKE, FAKE, 0.0, 0, FAKE,
                         None, FAKE, ws, 1 << 40, None) == gmm.GMM_EINVAL


def test_binding_refuses_host_tensors():
    import torch
    X = torch.zeros(10, 4)
    with pytest.raises(ValueError):
        gmm._xptr(X)


def test_kernel_path_selection():
    """Which kernel family each shape runs: the one-pass kernels for D, G <= 128
    (prec picks the arithmetic), the FP64 matrix-core kernels above 128
    components whatever prec says, the generic ones above 128 dimensions."""
    P = gmm
    assert P.gmm_em_path(100, 100, P.COV_DIAG, P.PREC_BF16X3) == P.PATH_ONEPASS_BF16X3
    assert P.gmm_em_path(100, 100, P.COV_DIAG, P.PREC_FP32) == P.PATH_ONEPASS_FP32
    for prec in (P.PREC_FP32, P.PREC_BF16X3):
        want = P.PATH_SLICED_BF16X3 if prec == P.PREC_BF16X3 else P.PATH_WIDE_FP64
        assert P.gmm_em_path(64, 512, P.COV_DIAG, prec) == want
        assert P.gmm_em_path(100, 300, P.COV_DIAG, prec) == want
        assert P.gmm_em_path(128, 129, P.COV_DIAG, prec) == want
        assert P.gmm_em_path(200, 5, P.COV_DIAG, prec) == P.PATH_GENERIC
        assert P.gmm_em_path(32, 64, P.COV_FULL, prec) == P.PATH_FULL_FP64
        assert P.gmm_em_path(80, 3, P.COV_FULL, prec) == P.PATH_FULL_GENERIC
        assert P.gmm_kmeans_path(64, 512, prec) == P.PATH_WIDE_FP64
        assert P.gmm_kmeans_path(300, 3, prec) == P.PATH_GENERIC
    assert P.gmm_kmeans_path(100, 100, P.PREC_BF16X3) == P.PATH_ONEPASS_BF16X3
    assert P.gmm_kmeans_path(100, 100, P.PREC_FP32) == P.PATH_ONEPASS_FP32
    L = P.library()
    assert L.gmm_em_path(0, 4, 0, 0) == P.GMM_EINVAL
    assert L.gmm_em_path(4, 4, 0, 5) == P.GMM_EINVAL
    assert L.gmm_em_path(200, 4, P.COV_FULL, 0) == P.GMM_EINVAL
    assert L.gmm_kmeans_path(4, 0, 0) == P.GMM_EINVAL
