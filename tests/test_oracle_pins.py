"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
library routines on special cases, 50-digit brute force in the linear domain,
the Appendix-A Q-function, invariants and a hand-derived worked example.
"""
import itertools
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.spatial.distance import cdist
from scipy.special import logsumexp
from scipy.stats import multivariate_normal

from paper_1707_09094_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LOG2PI = math.log(2 * math.pi)


def _rng(seed=0):
    return np.random.Generator(np.random.PCG64(seed))


def _spd(rng, D, ridge=0.3):
    A = rng.normal(size=(D, D)) * 0.5
    return A @ A.T + ridge * np.eye(D)


# --------------------------------------------------------------------------- P-1
@pytest.mark.parametrize("D,N", [(1, 50), (3, 200), (7, 1000)])
def test_single_component_closed_form_diag(oracle, D, N):
    """N_G = 1: l == 1, so Eqs. 5-7 give w = 1, the sample mean and the population
    variance; the log-likelihood of that fit has the closed form
    -1/2 [D (log 2 pi + 1) + sum_d log var_d]."""
    rng = _rng(D)
    X = (rng.normal(size=(N, D)) * rng.uniform(0.5, 3, size=D) + rng.normal(size=D) * 4).astype(np.float32)
    X64 = X.astype(np.float64)
    # arbitrary starting parameters: the answer must not depend on them
    res = oracle.em_iter(X, [1.0], rng.normal(size=(1, D)), rng.uniform(0.1, 5, size=(1, D)), 1e-10)
    mean = X64.mean(axis=0)
    var = X64.var(axis=0, ddof=0)
    np.testing.assert_allclose(res.hefts, [1.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.means[0], mean, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(res.covs[0], var, rtol=1e-11)
    ll = oracle.loglik(X, res.hefts, res.means, res.covs)
    closed = -0.5 * (D * (LOG2PI + 1.0) + np.log(var).sum())
    assert abs(ll - closed) <= 1e-11 * abs(closed)


@pytest.mark.parametrize("D,N", [(2, 300), (5, 2000)])
def test_single_component_closed_form_full(oracle, D, N):
    """Full covariance, N_G = 1: Sigma = np.cov(bias=True); loglik =
    -1/2 [D (log 2 pi + 1) + log|S|] (slogdet)."""
    rng = _rng(10 + D)
    C = _spd(rng, D)
    X = rng.multivariate_normal(rng.normal(size=D) * 3, C, size=N).astype(np.float32)
    X64 = X.astype(np.float64)
    res = oracle.em_iter(X, [1.0], np.zeros((1, D)), np.eye(D)[None] * 2.0, 1e-10, full=True)
    np.testing.assert_allclose(res.means[0], X64.mean(axis=0), rtol=1e-12, atol=1e-12)
    S = np.cov(X64, rowvar=False, bias=True)
    np.testing.assert_allclose(res.covs[0], S, rtol=1e-10, atol=1e-12)
    ll = oracle.loglik(X, res.hefts, res.means, res.covs, full=True)
    closed = -0.5 * (D * (LOG2PI + 1.0) + np.linalg.slogdet(S)[1])
    assert abs(ll - closed) <= 1e-11 * abs(closed)


def test_variance_floor_constant_dimension(oracle):
    """A constant dimension has variance 0; the floor (Sec. 2.2) makes it exactly
    var_floor, and values above the floor are untouched."""
    rng = _rng(3)
    X = rng.normal(size=(500, 3)).astype(np.float32)
    X[:, 1] = 2.5
    floor = 1e-3
    res = oracle.em_iter(X, [1.0], np.zeros((1, 3)), np.ones((1, 3)), floor)
    assert res.covs[0, 1] == floor
    v = X.astype(np.float64).var(axis=0)
    np.testing.assert_allclose(res.covs[0, [0, 2]], v[[0, 2]], rtol=1e-12)
    # full covariance: floor on the diagonal only
    resf = oracle.em_iter(X, [1.0], np.zeros((1, 3)), np.eye(3)[None], floor, full=True)
    assert resf.covs[0, 1, 1] == floor
    assert resf.covs[0, 0, 1] == resf.covs[0, 1, 0]


# --------------------------------------------------------------------------- P-13
@pytest.mark.parametrize("D,G", [(1, 3), (4, 5), (9, 2)])
def test_loglik_matches_scipy_diag(oracle, D, G):
    rng = _rng(20 + D)
    N = 300
    X = rng.normal(size=(N, D)).astype(np.float32) * 2
    w = rng.dirichlet(np.ones(G))
    mu = rng.normal(size=(G, D)) * 2
    var = rng.uniform(0.1, 4, size=(G, D))
    mean_ll, ps = oracle.loglik(X, w, mu, var, per_sample=True)
    X64 = X.astype(np.float64)
    comp = np.stack([np.log(w[g]) + multivariate_normal(mu[g], np.diag(var[g])).logpdf(X64).reshape(N)
                     for g in range(G)], axis=1)
    ref = logsumexp(comp, axis=1)
    np.testing.assert_allclose(ps, ref, rtol=1e-12, atol=1e-11)
    assert abs(mean_ll - ref.mean()) <= 1e-12 * abs(ref.mean())
    # per-Gaussian log_p(X, g)
    for g in range(G):
        np.testing.assert_allclose(oracle.log_p_g(X, mu, var, g), comp[:, g] - np.log(w[g]),
                                   rtol=1e-12, atol=1e-11)


def test_loglik_matches_scipy_full(oracle):
    rng = _rng(31)
    D, G, N = 4, 3, 400
    X = rng.normal(size=(N, D)).astype(np.float32) * 2
    w = rng.dirichlet(np.ones(G))
    mu = rng.normal(size=(G, D))
    S = np.stack([_spd(rng, D) for _ in range(G)])
    mean_ll, ps = oracle.loglik(X, w, mu, S, full=True, per_sample=True)
    X64 = X.astype(np.float64)
    comp = np.stack([np.log(w[g]) + multivariate_normal(mu[g], S[g]).logpdf(X64) for g in range(G)], 1)
    np.testing.assert_allclose(ps, logsumexp(comp, axis=1), rtol=1e-12, atol=1e-11)


def test_full_rejects_non_pd(oracle):
    X = np.zeros((4, 2), dtype=np.float32)
    S = np.array([[[1.0, 2.0], [2.0, 1.0]]])
    with pytest.raises(Exception):
        oracle.loglik(X, [1.0], np.zeros((1, 2)), S, full=True)


# --------------------------------------------------------------------------- P-7
def _dec_lin_mixture(X, w, mu, var):
    """Eqs. 1-3 evaluated directly in the linear domain with 50-digit decimals."""
    getcontext().prec = 50
    two_pi = Decimal(2) * Decimal("3.14159265358979323846264338327950288419716939937510")
    N, D = X.shape
    G = len(w)
    logp, resp = [], []
    for i in range(N):
        dens = []
        for g in range(G):
            det = Decimal(1)
            q = Decimal(0)
            for d in range(D):
                v = Decimal(float(var[g][d]))
                det *= v
                t = Decimal(float(X[i][d])) - Decimal(float(mu[g][d]))
                q += t * t / v
            n = (-(q / 2)).exp() / ((two_pi ** D) * det).sqrt()
            dens.append(Decimal(float(w[g])) * n)
        tot = sum(dens)
        logp.append(float(tot.ln()))
        resp.append([float(x / tot) for x in dens])
    return np.array(logp), np.array(resp)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_linear_domain_decimal(oracle, seed):
    """Log-domain reformulation (Eqs. 15-18) == the linear-domain definition
    (Eqs. 1-3) computed with 50 significant digits, on tiny inputs."""
    rng = _rng(100 + seed)
    N, D, G = 6, 2, 3
    X = rng.normal(size=(N, D)).astype(np.float32) * 1.5
    w = rng.dirichlet(np.ones(G))
    mu = rng.normal(size=(G, D))
    var = rng.uniform(0.3, 2.0, size=(G, D))
    ref_lp, ref_r = _dec_lin_mixture(X, w, mu, var)
    _, ps = oracle.loglik(X, w, mu, var, per_sample=True)
    np.testing.assert_allclose(ps, ref_lp, rtol=1e-14, atol=1e-14)
    r = oracle.responsibilities(X, w, mu, var)
    np.testing.assert_allclose(r, ref_r, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------- P-3
def test_responsibility_and_weight_invariants(oracle):
    rng = _rng(7)
    N, D, G = 2000, 3, 6
    X = rng.normal(size=(N, D)).astype(np.float32) * 3
    w, mu, var = synth.random_params(rng, D, G)
    r = oracle.responsibilities(X, w, mu, var)
    np.testing.assert_allclose(r.sum(axis=1), 1.0, atol=1e-13)
    assert (r >= 0).all()
    res = oracle.em_iter(X, w, mu, var, 1e-10)
    assert abs(res.hefts.sum() - 1.0) <= 1e-12
    assert abs(res.L.sum() - N) <= 1e-9
    assert (res.hefts >= 0).all()


# --------------------------------------------------------------------------- P-4
@pytest.mark.parametrize("seed,floor", [(0, 1e-10), (1, 0.5), (2, 1e-10)])
def test_em_loglik_monotone(oracle, seed, floor):
    """EM never decreases the likelihood (Sec. 2); the variance floor keeps this
    because per dimension the floored value is the constrained maximiser."""
    X, truth = synth.diag_gmm(500 + seed, 3, 5, 3000, "uniform", -3, 3, "std_uniform", 0.3, 1.5)
    rng = _rng(seed)
    w = np.full(5, 0.2)
    mu = X[rng.choice(len(X), 5, replace=False)].astype(np.float64)
    var = np.ones((5, 3))
    prev = -np.inf
    for _ in range(25):
        res = oracle.em_iter(X, w, mu, var, floor)
        assert res.mean_loglik >= prev - 1e-12 * abs(prev if np.isfinite(prev) else 1.0)
        prev = res.mean_loglik
        w, mu, var = res.hefts, res.means, res.covs
        assert (var >= floor).all()


def test_em_loglik_monotone_full(oracle):
    X, _ = synth.full_gmm(77, 3, 3, 1500)
    w = np.full(3, 1 / 3)
    mu = X[[0, 500, 1000]].astype(np.float64)
    S = np.stack([np.eye(3)] * 3)
    prev = -np.inf
    for _ in range(15):
        res = oracle.em_iter(X, w, mu, S, 1e-6, full=True)
        assert res.mean_loglik >= prev - 1e-12 * abs(prev if np.isfinite(prev) else 1.0)
        prev = res.mean_loglik
        w, mu, S = res.hefts, res.means, res.covs


# --------------------------------------------------------------------------- P-8
def _comp_logpdf(X, mu, var):
    X64 = X.astype(np.float64)
    return np.stack([multivariate_normal(mu[g], np.diag(var[g])).logpdf(X64).reshape(len(X))
                     for g in range(len(mu))], axis=1)


def _Q_simplified(X, w, mu, var, post):
    """Appendix A: Q = sum_m sum_i log[w_m p(x_i|theta_m)] p(m|x_i, Theta^k)."""
    return float((post * (np.log(w)[None, :] + _comp_logpdf(X, mu, var))).sum())


def _Q_enumerated(X, w, mu, var, post):
    """Appendix A: Q as the expectation over every labelling y in {1..M}^N of
    log p(X, y | Theta), weighted by prod_j p(y_j | x_j, Theta^k)."""
    N, M = post.shape
    lc = np.log(w)[None, :] + _comp_logpdf(X, mu, var)
    total = 0.0
    for y in itertools.product(range(M), repeat=N):
        idx = np.arange(N)
        total += lc[idx, y].sum() * np.prod(post[idx, y])
    return total


@pytest.mark.parametrize("seed", [0, 1])
def test_q_function_enumeration_and_maximisation(oracle, seed):
    """Appendix A: the enumerated Q equals its simplified double sum, and the
    oracle's M-step output maximises Q over feasible parameters (weights on the
    simplex, variances >= floor): random feasible perturbations never raise it."""
    rng = _rng(900 + seed)
    N, D, M = 5, 2, 3
    X = rng.normal(size=(N, D)).astype(np.float32) * 2
    w = rng.dirichlet(np.ones(M))
    mu = rng.normal(size=(M, D))
    var = rng.uniform(0.5, 2, size=(M, D))
    X64 = X.astype(np.float64)
    lc = np.log(w)[None, :] + _comp_logpdf(X, mu, var)
    post = np.exp(lc - logsumexp(lc, axis=1, keepdims=True))  # Bayes' rule, independent of the oracle
    q_enum = _Q_enumerated(X, w, mu, var, post)
    q_simp = _Q_simplified(X, w, mu, var, post)
    assert abs(q_enum - q_simp) <= 1e-10 * abs(q_simp)
    floor = 0.05
    res = oracle.em_iter(X, w, mu, var, floor)
    q_star = _Q_simplified(X, res.hefts, res.means, res.covs, post)
    for _ in range(300):
        w2 = np.abs(res.hefts + rng.normal(size=M) * 0.05)
        w2 /= w2.sum()
        mu2 = res.means + rng.normal(size=(M, D)) * 0.1
        var2 = np.maximum(res.covs * np.exp(rng.normal(size=(M, D)) * 0.2), floor)
        assert _Q_simplified(X, w2, mu2, var2, post) <= q_star + 1e-12 * abs(q_star)


# --------------------------------------------------------------------------- P-9 / P-10
def test_affine_equivariance(oracle):
    """x -> a + s*x maps mu -> a + s*mu, var -> s^2 var, leaves w unchanged and
    shifts the mean log-likelihood by -sum log|s| (floor inactive)."""
    rng = _rng(11)
    N, D, G = 1500, 3, 4
    # samples on a 2^-10 grid so that a + s*x below is exact in float32
    X = np.round(rng.normal(size=(N, D)) * 2 * 1024) / 1024
    w, mu, var = synth.random_params(rng, D, G)
    a = np.array([1.5, -3.0, 0.25])
    s = np.array([2.0, 0.5, -4.0])  # powers of two
    X1 = X.astype(np.float32)
    X2 = (a + s * X1.astype(np.float64)).astype(np.float32)
    r1 = oracle.em_iter(X1, w, mu, var, 1e-12)
    r2 = oracle.em_iter(X2, w, a + s * mu.astype(np.float64), (s ** 2) * var.astype(np.float64), 1e-12)
    np.testing.assert_allclose(r2.hefts, r1.hefts, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(r2.means, a + s * r1.means, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(r2.covs, s ** 2 * r1.covs, rtol=1e-9)
    assert abs(r2.mean_loglik - (r1.mean_loglik - np.log(np.abs(s)).sum())) <= 1e-10 * abs(r1.mean_loglik)


def test_permutation_invariance(oracle):
    rng = _rng(12)
    N, D, G = 800, 2, 3
    X = (rng.normal(size=(N, D)) * 2).astype(np.float32)
    w, mu, var = synth.random_params(rng, D, G)
    r1 = oracle.em_iter(X, w, mu, var, 1e-10)
    perm = rng.permutation(N)
    r2 = oracle.em_iter(X[perm], w, mu, var, 1e-10)
    np.testing.assert_allclose(r2.means, r1.means, rtol=1e-11)
    np.testing.assert_allclose(r2.covs, r1.covs, rtol=1e-11)
    cp = np.array([2, 0, 1])
    r3 = oracle.em_iter(X, w[cp], mu[cp], var[cp], 1e-10)
    np.testing.assert_allclose(r3.means, r1.means[cp], rtol=1e-13)
    np.testing.assert_allclose(r3.hefts, r1.hefts[cp], rtol=1e-13)


def test_thread_count_does_not_change_results(oracle):
    X, _ = synth.config1(N=3000)
    rng = _rng(5)
    w, mu, var = synth.random_params(rng, 4, 4)
    oracle.set_threads(1)
    a = oracle.em_iter(X, w, mu, var, 1e-10)
    ka = oracle.kmeans_iter(X, mu, np.ones(4), 1e-10)
    oracle.set_threads(8)
    b = oracle.em_iter(X, w, mu, var, 1e-10)
    kb = oracle.kmeans_iter(X, mu, np.ones(4), 1e-10)
    oracle.set_threads(0)
    assert np.array_equal(a.means, b.means) and np.array_equal(a.covs, b.covs)
    assert a.mean_loglik == b.mean_loglik
    assert np.array_equal(ka.means, kb.means) and ka.inertia == kb.inertia


# --------------------------------------------------------------------------- global stats
def test_global_stats_matches_numpy(oracle):
    rng = _rng(13)
    X = (rng.normal(size=(5000, 6)) * rng.uniform(0.1, 10, 6) + rng.normal(size=6) * 100).astype(np.float32)
    mean, var = oracle.global_stats(X)
    np.testing.assert_allclose(mean, X.astype(np.float64).mean(0), rtol=1e-13)
    np.testing.assert_allclose(var, X.astype(np.float64).var(0, ddof=0), rtol=1e-11)


# --------------------------------------------------------------------------- k-means
@pytest.mark.parametrize("maha", [False, True])
def test_kmeans_bruteforce(oracle, maha):
    """Eq. 19 / Eq. 20 by brute force with scipy's distance routines; new means
    are plain averages of the assigned samples (Sec. 3)."""
    rng = _rng(14 + maha)
    N, D, G = 600, 3, 5
    X = (rng.normal(size=(N, D)) * [1, 10, 0.1] + rng.normal(size=D)).astype(np.float32)
    mu = X[rng.choice(N, G, replace=False)].astype(np.float64) + rng.normal(size=(G, D)) * 0.01
    X64 = X.astype(np.float64)
    if maha:
        var = X64.var(0)
        lam = 1.0 / var
        dist = cdist(X64, mu, metric="seuclidean", V=var) ** 2
    else:
        lam = np.ones(D)
        dist = cdist(X64, mu, metric="sqeuclidean")
    res = oracle.kmeans_iter(X, mu, lam, 1e-10)
    assign = dist.argmin(axis=1)
    assert np.array_equal(res.assign, assign)
    np.testing.assert_allclose(res.inertia, dist.min(axis=1).sum(), rtol=1e-11)
    for g in range(G):
        sel = X64[assign == g]
        assert res.counts[g] == len(sel)
        if len(sel):
            np.testing.assert_allclose(res.means[g], sel.mean(0), rtol=1e-12, atol=1e-13)
            np.testing.assert_allclose(res.dcovs[g], np.maximum(sel.var(0), 1e-10), rtol=1e-10)
    np.testing.assert_allclose(res.hefts, res.counts / N, rtol=1e-15)
    srt = np.sort(dist, axis=1)
    np.testing.assert_allclose(res.gap, (srt[:, 1] - srt[:, 0]) / srt[:, 0], rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("maha", [False, True])
def test_kmeans_dists_and_near_sets(oracle, maha):
    """The full distance matrix against scipy's weighted squared distances; its
    first argmin is the oracle's assignment; the near set of a sample always
    holds its assigned mean, and holds a second mean exactly when the oracle's
    relative gap is below the threshold (an exact tie from a duplicated mean)."""
    rng = _rng(40 + maha)
    N, D, G = 400, 4, 6
    X = (rng.normal(size=(N, D)) * [1, 3, 0.5, 2]).astype(np.float32)
    mu = X[rng.choice(N, G, replace=False)].astype(np.float64)
    mu[5] = mu[2]  # exact ties for every sample nearest to mean 2
    X64 = X.astype(np.float64)
    lam = 1.0 / X64.var(0) if maha else np.ones(D)
    d = oracle.kmeans_dists(X, mu, lam)
    ref = cdist(X64 * np.sqrt(lam), mu * np.sqrt(lam), metric="sqeuclidean")
    np.testing.assert_allclose(d, ref, rtol=1e-12, atol=1e-12)
    res = oracle.kmeans_iter(X, mu, lam, 1e-10)
    assert np.array_equal(d.argmin(axis=1), res.assign)
    dmin = d.min(axis=1, keepdims=True)
    near = (d - dmin) / np.maximum(dmin, 1e-300) < 1e-6
    assert near[np.arange(N), res.assign].all()
    assert np.array_equal(near.sum(axis=1) >= 2, res.gap < 1e-6)
    tied = res.assign == 2
    assert tied.any() and near[tied, 5].all() and (res.assign != 5).all()


def test_kmeans_single_cluster_closed_form(oracle):
    """N_G = 1: every sample in cluster 0; inertia under the input mean mu0 is
    N * sum_d lam_d (var_d + (mean_d - mu0_d)^2)."""
    rng = _rng(15)
    X = (rng.normal(size=(1000, 4)) * 3).astype(np.float32)
    X64 = X.astype(np.float64)
    mu0 = rng.normal(size=(1, 4))
    lam = rng.uniform(0.5, 2, 4)
    res = oracle.kmeans_iter(X, mu0, lam, 1e-10)
    assert (res.assign == 0).all() and res.counts[0] == 1000
    np.testing.assert_allclose(res.means[0], X64.mean(0), rtol=1e-12)
    closed = 1000 * (lam * (X64.var(0) + (X64.mean(0) - mu0[0]) ** 2)).sum()
    assert abs(res.inertia - closed) <= 1e-11 * closed


def test_kmeans_tie_goes_to_lowest_index(oracle):
    """Duplicate means give exact ties; Eq. 19's argmin takes the first."""
    X = np.array([[0.0, 0.0], [1.0, 1.0], [5.0, 5.0]], dtype=np.float32)
    mu = np.array([[5.0, 5.0], [0.5, 0.5], [0.5, 0.5]])
    res = oracle.kmeans_iter(X, mu, np.ones(2), 1e-10)
    assert list(res.assign) == [1, 1, 0]
    assert res.counts[2] == 0


def test_kmeans_resurrection_golden(oracle):
    with open(os.path.join(GOLDEN, "resurrection_1d.json")) as f:
        gd = json.load(f)
    X = np.array(gd["X"], dtype=np.float32)[:, None]
    mu = np.array(gd["means_in"])[:, None]
    res = oracle.kmeans_iter(X, mu, np.ones(1), gd["var_floor"])
    assert list(res.assign) == gd["assign"]
    assert list(res.counts) == gd["counts"]
    np.testing.assert_allclose(res.means[:, 0], gd["means_out"], rtol=1e-15)
    np.testing.assert_allclose(res.dcovs[:, 0], gd["dcovs_out"], rtol=1e-14)
    np.testing.assert_allclose(res.hefts, gd["hefts_out"], rtol=1e-15)
    assert res.inertia == gd["inertia"]


def test_kmeans_inertia_non_increasing_with_dead_means(oracle):
    """Lloyd iterations never raise the cost; a resurrected mean owns no sample
    when it moves, so resurrection keeps this."""
    X, _ = synth.diag_gmm(321, 2, 3, 2000, "uniform", -6, 6, "std_uniform", 0.3, 0.8)
    # 6 means, three of them duplicates far away -> dead clusters
    mu = np.concatenate([X[:3].astype(np.float64), np.full((3, 2), 50.0)])
    lam = np.ones(2)
    prev = np.inf
    dead_seen = False
    for _ in range(12):
        res = oracle.kmeans_iter(X, mu, lam, 1e-10)
        assert res.inertia <= prev * (1 + 1e-12)
        prev = res.inertia
        dead_seen |= bool((res.counts == 0).any())
        mu = res.means
    assert dead_seen


def test_assign_modes(oracle):
    rng = _rng(16)
    N, D, G = 400, 3, 4
    X = (rng.normal(size=(N, D)) * 2).astype(np.float32)
    w, mu, var = synth.random_params(rng, D, G)
    a0 = oracle.assign(X, w, mu, var, 0)
    assert np.array_equal(a0, cdist(X.astype(np.float64), mu.astype(np.float64), "sqeuclidean").argmin(1))
    a1 = oracle.assign(X, w, mu, var, 1)
    lc = np.log(w.astype(np.float64))[None] + _comp_logpdf(X, mu.astype(np.float64), var.astype(np.float64))
    assert np.array_equal(a1, lc.argmax(1))


# --------------------------------------------------------------------------- P-11
def test_fig1_recipe_recovery(oracle):
    """Fig. 1 program: d=5, N=10000, unit-variance clusters at 1..5 and 3..7 in
    ratio 2:1; Mahalanobis k-means (10 iterations) then 5 EM iterations, floor
    1e-10.  The paper prints no outputs, so the check is statistical: the fit
    recovers the generating parameters within a few standard errors."""
    X, truth = synth.fig1_recipe()
    _, var = oracle.global_stats(X)
    lam = oracle.maha_lambda(var, 1e-10)
    rng = _rng(17)
    mu = X[rng.choice(len(X), 2, replace=False)].astype(np.float64)  # a random subset
    for _ in range(10):
        km = oracle.kmeans_iter(X, mu, lam, 1e-10)
        mu = km.means
    w, var_g = km.hefts, km.dcovs
    for _ in range(5):
        em = oracle.em_iter(X, w, mu, var_g, 1e-10)
        w, mu, var_g = em.hefts, em.means, em.covs
    order = np.argsort(mu[:, 0])
    w, mu, var_g = w[order], mu[order], var_g[order]
    n = np.array([2 / 3, 1 / 3]) * len(X)
    assert np.all(np.abs(w - truth.hefts) < 5 * np.sqrt(truth.hefts * (1 - truth.hefts) / len(X)) + 0.01)
    assert np.all(np.abs(mu - truth.means) < 5 / np.sqrt(n)[:, None] + 0.05)
    assert np.all(np.abs(var_g - 1.0) < 5 * np.sqrt(2 / n)[:, None] + 0.1)


# ---------------------------------------------------------------- spread seeding
def test_seed_spread_closed_form_1d(oracle):
    """x = 0..10 from x = 5: distances (x - 5)^2 put 0 and 10 at 25 (the lower
    index, 0, wins), then 10 is farthest from {5, 0}, then 2, 3, 7, 8 tie at 4
    and 2 wins: seeds 5, 0, 10, 2."""
    X = np.arange(11, dtype=np.float32)[:, None]
    idx, means = oracle.seed_spread(X, 4, first=5)
    assert idx.tolist() == [5, 0, 10, 2]
    np.testing.assert_array_equal(means[:, 0], [5.0, 0.0, 10.0, 2.0])


@pytest.mark.parametrize("maha,first", [(False, 0), (True, 0), (True, 137)])
def test_seed_spread_brute_force(oracle, maha, first):
    """Greedy maximin over the full pairwise distance matrix (scipy cdist, an
    independent evaluation of the weighted distances)."""
    rng = _rng(23)
    X = (rng.standard_normal((300, 4)) * [1.0, 3.0, 0.5, 2.0]).astype(np.float32)
    lam = oracle.maha_lambda(oracle.global_stats(X)[1], 1e-10) if maha else None
    w = np.ones(4) if lam is None else lam
    D2 = cdist(X.astype(np.float64), X.astype(np.float64), "sqeuclidean", w=w)
    ref = [first]
    dmin = D2[first].copy()
    for _ in range(11):
        s = int(np.argmax(dmin))  # first index of the maximum
        ref.append(s)
        dmin = np.minimum(dmin, D2[s])
    idx, means = oracle.seed_spread(X, 12, first=first, lam=lam)
    assert idx.tolist() == ref
    np.testing.assert_array_equal(means, X[ref].astype(np.float64))
    assert len(set(ref)) == 12


def test_seed_spread_more_seeds_than_distinct_samples(oracle):
    """Three distinct points: once all are seeds every distance is 0 and the
    lowest index is taken."""
    X = np.array([[0.0], [4.0], [0.0], [9.0], [4.0]], dtype=np.float32)
    idx, _ = oracle.seed_spread(X, 5, first=1)
    assert idx.tolist() == [1, 3, 0, 0, 0]


# ------------------------------------------------------- FP64 samples (gmm_diag)
def _f64_data(seed, N, D, offset=1e6, scale=1e-3):
    """FP64 samples that FP32 cannot hold: a large offset plus deviations far
    below the FP32 spacing at that offset (0.0625 at 1e6)."""
    rng = _rng(seed)
    return offset + rng.normal(size=(N, D)) * scale * rng.uniform(0.5, 2.0, size=D)


@pytest.mark.parametrize("D,N", [(1, 40), (4, 3000)])
def test_f64_single_component_closed_form(oracle, D, N):
    """FP64 samples, N_G = 1: the EM step gives numpy's FP64 mean and population
    variance, the k-means step the same mean; the same data rounded to FP32
    would have lost the deviations entirely."""
    X = _f64_data(3 + D, N, D)
    rng = _rng(D)
    res = oracle.em_iter(X, [1.0], rng.normal(size=(1, D)) + 1e6, np.full((1, D), 1e-6), 1e-30)
    np.testing.assert_allclose(res.means[0], X.mean(axis=0), rtol=1e-15)
    np.testing.assert_allclose(res.covs[0], X.var(axis=0), rtol=1e-8)
    km = oracle.kmeans_iter(X, X[:1], np.ones(D), 1e-30)
    np.testing.assert_allclose(km.means[0], X.mean(axis=0), rtol=1e-15)
    np.testing.assert_allclose(km.dcovs[0], X.var(axis=0), rtol=1e-8)
    m, v = oracle.global_stats(X)
    np.testing.assert_allclose(m, X.mean(axis=0), rtol=1e-15)
    np.testing.assert_allclose(v, X.var(axis=0), rtol=1e-8)
    assert np.all(X.astype(np.float32).astype(np.float64).var(axis=0) == 0.0)


@pytest.mark.parametrize("seed", [0, 1])
def test_f64_bruteforce_linear_domain_decimal(oracle, seed):
    """FP64 samples through the log domain == Eqs. 1-3 in 50-digit decimals."""
    rng = _rng(200 + seed)
    N, D, G = 6, 2, 3
    X = rng.normal(size=(N, D)) * 1.5 + 1e-9 * rng.normal(size=(N, D))
    w = rng.dirichlet(np.ones(G))
    mu = rng.normal(size=(G, D))
    var = rng.uniform(0.3, 2.0, size=(G, D))
    ref_lp, ref_r = _dec_lin_mixture(X, w, mu, var)
    _, ps = oracle.loglik(X, w, mu, var, per_sample=True)
    np.testing.assert_allclose(ps, ref_lp, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(oracle.responsibilities(X, w, mu, var), ref_r, rtol=1e-13,
                               atol=1e-15)


@pytest.mark.parametrize("maha", [False, True])
def test_f64_kmeans_bruteforce(oracle, maha):
    """FP64 samples: Eq. 19 / Eq. 20 by brute force with scipy's distances."""
    rng = _rng(300 + maha)
    N, D, G = 500, 3, 4
    X = rng.normal(size=(N, D)) * [1, 10, 0.1] + 5e5
    mu = X[rng.choice(N, G, replace=False)] + rng.normal(size=(G, D)) * 0.01
    if maha:
        var = X.var(0)
        lam, dist = 1.0 / var, cdist(X, mu, metric="seuclidean", V=var) ** 2
    else:
        lam, dist = np.ones(D), cdist(X, mu, metric="sqeuclidean")
    res = oracle.kmeans_iter(X, mu, lam, 1e-30)
    assert np.array_equal(res.assign, dist.argmin(axis=1))
    for g in range(G):
        sel = X[res.assign == g]
        np.testing.assert_allclose(res.means[g], sel.mean(0), rtol=1e-15)
        np.testing.assert_allclose(res.dcovs[g], sel.var(0), rtol=1e-7)
    np.testing.assert_allclose(oracle.kmeans_dists(X, mu, lam), dist, rtol=1e-7)


def test_f64_entry_points_agree_with_fp32_on_fp32_data(oracle):
    """FP32 samples handed over as FP64 give bit-identical results (each value
    is promoted exactly in both)."""
    X, _ = synth.config1(N=3000)
    X64 = X.astype(np.float64)
    mu = synth.static_subset(X, 4).astype(np.float64)
    w, v = np.full(4, 0.25), np.ones((4, 4))
    a, b = oracle.em_iter(X, w, mu, v, 1e-10), oracle.em_iter(X64, w, mu, v, 1e-10)
    assert np.array_equal(a.means, b.means) and np.array_equal(a.covs, b.covs)
    assert a.mean_loglik == b.mean_loglik
    ka, kb = oracle.kmeans_iter(X, mu, np.ones(4), 1e-10), oracle.kmeans_iter(X64, mu, np.ones(4), 1e-10)
    assert np.array_equal(ka.assign, kb.assign) and ka.inertia == kb.inertia
    assert np.array_equal(oracle.global_stats(X)[1], oracle.global_stats(X64)[1])
