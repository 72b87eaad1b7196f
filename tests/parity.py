"""Comparison helpers for GPU-vs-oracle parity: the relative errors of one EM or
k-means step.  Weights are compared relative to max(w, 1/N), means relative
to max(|mu|, sigma), variances relative to themselves, full covariance entries
relative to sqrt(S_dd S_ee); all within 1e-5, the mean log-likelihood within
1e-6."""
import numpy as np

PARAM_TOL = 1e-5    # weights, means, variances
LOGLIK_TOL = 1e-6   # mean log-likelihood


def rel_weights(w_gpu, w_ref, N):
    w_ref = np.asarray(w_ref, dtype=np.float64)
    return np.abs(np.asarray(w_gpu, np.float64) - w_ref) / np.maximum(w_ref, 1.0 / N)


def rel_means(mu_gpu, mu_ref, var_ref):
    mu_ref = np.asarray(mu_ref, np.float64)
    scale = np.maximum(np.abs(mu_ref), np.sqrt(np.asarray(var_ref, np.float64)))
    return np.abs(np.asarray(mu_gpu, np.float64) - mu_ref) / scale


def rel_vars(v_gpu, v_ref):
    v_ref = np.asarray(v_ref, np.float64)
    return np.abs(np.asarray(v_gpu, np.float64) - v_ref) / v_ref


def rel_full_cov(S_gpu, S_ref):
    S_ref = np.asarray(S_ref, np.float64)
    d = np.sqrt(np.einsum("gii->gi", S_ref))
    scale = d[:, :, None] * d[:, None, :]
    return np.abs(np.asarray(S_gpu, np.float64) - S_ref) / scale


def check_em(gpu, ref, N, live=None, tol=PARAM_TOL, ll_tol=LOGLIK_TOL, full=False):
    """gpu: dict hefts/means/covs/loglik; ref: oracle EMResult.  Components whose
    oracle L_g < 1 are exempt for means/covariances."""
    if live is None:
        live = ref.L >= 1.0
    ew = rel_weights(gpu["hefts"], ref.hefts, N).max()
    em = rel_means(gpu["means"][live], ref.means[live],
                   np.einsum("gii->gi", ref.covs[live]) if full else ref.covs[live]).max(initial=0)
    if full:
        ev = rel_full_cov(gpu["covs"][live], ref.covs[live]).max(initial=0)
    else:
        ev = rel_vars(gpu["covs"][live], ref.covs[live]).max(initial=0)
    el = abs(gpu["loglik"] - ref.mean_loglik) / abs(ref.mean_loglik)
    msg = f"weights {ew:.2e} means {em:.2e} covs {ev:.2e} loglik {el:.2e}"
    assert ew <= tol and em <= tol and ev <= tol and el <= ll_tol, msg
    return dict(weights=ew, means=em, covs=ev, loglik=el)


def check_kmeans(gk, rk, dists, N, tol=PARAM_TOL, rel_gap=1e-6):
    """One k-means step against the oracle's (rk) on the same input means;
    dists is the oracle's (N, G) distance matrix under those means.

    Assignments are bit-exact wherever the oracle's relative gap between the
    two nearest means is at least rel_gap; a sample below that gap
    ("ambiguous") may take any mean of its near set, the means whose distance
    lies within that relative gap of the nearest.  Clusters that no ambiguous
    sample can join must then match exactly: counts equal, means/dcovs within
    tol, weights within 1e-6 (relative to max(w, 1/N)); dead clusters'
    resurrected means are compared when no sample is ambiguous (the donor
    depends on the counts).  Inertia within 1e-9 relative, plus rel_gap of
    the ambiguous samples' own distances.  Returns the number of ambiguous
    samples."""
    dmin = dists.min(axis=1)
    near = (dists - dmin[:, None]) / np.maximum(dmin, 1e-300)[:, None] < rel_gap
    amb = rk.gap < rel_gap
    assert np.array_equal(gk["assign"][~amb], rk.assign[~amb])
    idx = np.nonzero(amb)[0]
    assert near[idx, gk["assign"][idx]].all(), "an ambiguous sample left its near set"
    touched = near[idx].any(axis=0) if len(idx) else np.zeros(len(rk.counts), bool)
    assert np.abs(gk["counts"] - rk.counts).sum() <= 2 * len(idx)
    free = ~touched
    np.testing.assert_array_equal(gk["counts"][free], rk.counts[free])
    live = free & (rk.counts > 0)
    if live.any():
        assert rel_means(gk["means"][live], rk.means[live], rk.dcovs[live]).max() <= tol
        assert rel_vars(gk["dcovs"][live], rk.dcovs[live]).max() <= tol
    assert rel_weights(gk["hefts"][free], rk.hefts[free], N).max(initial=0) <= 1e-6
    if not len(idx):
        dead = rk.counts == 0
        np.testing.assert_array_equal(gk["means"][dead], rk.means[dead].astype(np.float32))
    slack = rel_gap * float(dmin[idx].sum())
    assert abs(gk["inertia"] - rk.inertia) <= 1e-9 * abs(rk.inertia) + 1e-12 + slack, \
        (gk["inertia"], rk.inertia)
    return int(len(idx))
