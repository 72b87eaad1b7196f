"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws random data (samples from a ground-truth mixture) and
picks initial means by index; it contains none of the training arithmetic.
Both the GPU path's tests/benchmark and the CPU oracle's tests take their
inputs from here.

Samples are returned as a C-contiguous float32 (N, D) array: row i is sample i,
which is the paper's D x N column-major data matrix (one sample per column,
Sec. 4 API) viewed from numpy.

Distribution notation: N(m, v) has mean m and VARIANCE v; log-uniform [a, b]
is exp(U(ln a, ln b)); Dirichlet(1) is flat over the simplex.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 18  # samples drawn per block of noise (fixed: part of the recipe)


@dataclass
class Truth:
    hefts: np.ndarray           # (G,)
    means: np.ndarray           # (G, D)
    dcovs: np.ndarray | None    # (G, D) diagonal variances, or None
    covs: np.ndarray | None     # (G, D, D) full covariances, or None
    labels: np.ndarray | None = field(default=None, repr=False)


def _draw(rng, N, hefts, means, scale_fn, dtype=np.float32):
    G, D = means.shape
    labels = rng.choice(G, size=N, p=hefts).astype(np.int32)
    X = np.empty((N, D), dtype=dtype)
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        z = rng.standard_normal((e - s, D))
        X[s:e] = (means[labels[s:e]] + scale_fn(labels[s:e], z)).astype(dtype)
    return X, labels


def diag_gmm(seed, D, G, N, mean_kind, mean_a, mean_b, var_kind, var_a, var_b, dtype=np.float32):
    """Ground-truth diagonal GMM and N samples from it (float32, or float64 for
    the FP64-data path: the same draw without the final rounding).

    Generation order: weights -> means -> variances -> labels -> noise.
    mean_kind 'uniform' draws U[mean_a, mean_b]; 'normal' draws N(mean_a, mean_b).
    var_kind 'loguniform' draws variances log-U[var_a, var_b]; 'std_uniform'
    draws standard deviations U[var_a, var_b].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.dirichlet(np.ones(G))
    if mean_kind == "uniform":
        mu = rng.uniform(mean_a, mean_b, size=(G, D))
    elif mean_kind == "normal":
        mu = rng.normal(mean_a, np.sqrt(mean_b), size=(G, D))
    else:
        raise ValueError(mean_kind)
    if var_kind == "loguniform":
        var = np.exp(rng.uniform(np.log(var_a), np.log(var_b), size=(G, D)))
    elif var_kind == "std_uniform":
        var = rng.uniform(var_a, var_b, size=(G, D)) ** 2
    else:
        raise ValueError(var_kind)
    sd = np.sqrt(var)
    X, labels = _draw(rng, N, w, mu, lambda lab, z: sd[lab] * z, dtype)
    return X, Truth(w, mu, var, None, labels)


def full_gmm(seed, D, G, N, mean_var=4.0, a_var=0.3, ridge=0.1):
    """Ground-truth full-covariance GMM: Sigma_g = A A^T + ridge*I, A_de ~ N(0, a_var)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.dirichlet(np.ones(G))
    mu = rng.normal(0.0, np.sqrt(mean_var), size=(G, D))
    A = rng.normal(0.0, np.sqrt(a_var), size=(G, D, D))
    S = A @ np.transpose(A, (0, 2, 1)) + ridge * np.eye(D)[None]
    Lc = np.linalg.cholesky(S)
    X, labels = _draw(rng, N, w, mu, lambda lab, z: np.einsum("nij,nj->ni", Lc[lab], z))
    return X, Truth(w, mu, None, S, labels)


# --- the five workloads -------------------------------------------------------

def seed_for(cfg_index: int) -> int:
    return 1707 * 10 + cfg_index


def config1(N=10_000, dtype=np.float32):
    """D=4, G=4, N=1e4: means U[-5,5], std U[0.5,2], weights Dirichlet(1)."""
    return diag_gmm(seed_for(1), 4, 4, N, "uniform", -5.0, 5.0, "std_uniform", 0.5, 2.0, dtype)


def config2(N=1_000_000, D=100, G=100, dtype=np.float32):
    """D=100, G=100, N=1e6: means N(0,4), variances log-U[0.1,10], weights Dirichlet(1)."""
    return diag_gmm(seed_for(2), D, G, N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0, dtype)


def config3(N=8_000_000, D=64, G=512):
    """D=64, G=512, N=8e6: means N(0,1), variances log-U[0.05,5], weights Dirichlet(1)."""
    return diag_gmm(seed_for(3), D, G, N, "normal", 0.0, 1.0, "loguniform", 0.05, 5.0)


def config4(N=2_000_000, D=32, G=64):
    """D=32, G=64, N=2e6 full covariance A A^T + 0.1 I, A_de ~ N(0, 0.3)."""
    return full_gmm(seed_for(4), D, G, N)


def model5_seed(k: int) -> int:
    h = hashlib.sha256(f"17079094:{k}".encode()).digest()
    return int.from_bytes(h[:8], "little")


def config5_shapes(n_models=2000, seed=seed_for(5)):
    """Per-model (N_k, G_k) of the batched workload: G_k uniform over
    {8,16,32,64}, N_k = round(exp U(ln 500, ln 2e5))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    G = rng.choice(np.array([8, 16, 32, 64]), size=n_models)
    N = np.rint(np.exp(rng.uniform(np.log(500.0), np.log(2e5), size=n_models))).astype(np.int64)
    return N, G


def config5_model(k, N, G, D=40):
    """Model k of the batched workload: the D=100 recipe (means N(0,4),
    variances log-U[0.1,10], Dirichlet(1) weights) at D=40."""
    return diag_gmm(model5_seed(k), D, int(G), int(N), "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)


def fig1_recipe(N=10_000, d=5, seed=seed_for(0)):
    """The example program of the paper's Fig. 1: two unit-variance clusters with
    means 1..d and (1..d)+2, drawn in the repeating order mean1, mean1, mean2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m1 = np.linspace(1.0, float(d), d)
    m2 = m1 + 2.0
    lab = (np.arange(N) % 3 == 2).astype(np.int32)
    X = (np.where(lab[:, None] == 1, m2, m1) + rng.standard_normal((N, d))).astype(np.float32)
    return X, Truth(np.array([2 / 3, 1 / 3]), np.stack([m1, m2]), np.ones((2, d)), None, lab)


# --- the same recipes drawn on the device (torch Philox), for data sets too
# large to draw on the host inside a benchmark run ---------------------------

def diag_gmm_device(seed, D, G, N, mean_var, var_lo, var_hi, device="cuda"):
    """Device twin of diag_gmm(seed, D, G, N, "normal", 0, mean_var, "loguniform",
    var_lo, var_hi): the same recipe and generation order (weights, means,
    variances, labels, noise) with torch's generator, so a different draw."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    e = -torch.log(torch.rand(G, device=device, generator=gen, dtype=torch.float64))
    w = e / e.sum()
    mu = float(np.sqrt(mean_var)) * torch.randn(G, D, device=device, generator=gen,
                                                dtype=torch.float64)
    lv = np.log(var_lo) + (np.log(var_hi) - np.log(var_lo)) * torch.rand(
        G, D, device=device, generator=gen, dtype=torch.float64)
    sd = torch.exp(0.5 * lv)
    lab = torch.multinomial(w, N, replacement=True, generator=gen)
    X = torch.empty(N, D, device=device, dtype=torch.float32)
    for s in range(0, N, CHUNK):
        e_ = min(N, s + CHUNK)
        z = torch.randn(e_ - s, D, device=device, generator=gen, dtype=torch.float64)
        X[s:e_] = (mu[lab[s:e_]] + sd[lab[s:e_]] * z).to(torch.float32)
    return X


def full_gmm_device(seed, D, G, N, mean_var=4.0, a_var=0.3, ridge=0.1, device="cuda"):
    """Device twin of full_gmm: Sigma_g = A A^T + ridge I, A_de ~ N(0, a_var)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    e = -torch.log(torch.rand(G, device=device, generator=gen, dtype=torch.float64))
    w = e / e.sum()
    mu = float(np.sqrt(mean_var)) * torch.randn(G, D, device=device, generator=gen,
                                                dtype=torch.float64)
    A = float(np.sqrt(a_var)) * torch.randn(G, D, D, device=device, generator=gen,
                                            dtype=torch.float64)
    S = A @ A.transpose(1, 2) + ridge * torch.eye(D, device=device, dtype=torch.float64)
    Lc = torch.linalg.cholesky(S)
    lab = torch.multinomial(w, N, replacement=True, generator=gen)
    X = torch.empty(N, D, device=device, dtype=torch.float32)
    for s in range(0, N, CHUNK):
        e_ = min(N, s + CHUNK)
        z = torch.randn(e_ - s, D, 1, device=device, generator=gen, dtype=torch.float64)
        X[s:e_] = (mu[lab[s:e_]] + (Lc[lab[s:e_]] @ z)[..., 0]).to(torch.float32)
    return X


def static_subset_index(N, G):
    """Indices floor(g*N/G), g = 0..G-1, of the static_subset seed mode."""
    return (np.arange(G, dtype=np.int64) * N) // G


def static_subset(X, G):
    """Initial means = samples floor(g*N/G), g = 0..G-1 (a repeatable subset of
    the training samples, the static_subset seed mode)."""
    N = X.shape[0]
    idx = (np.arange(G, dtype=np.int64) * N) // G
    return np.array(X[idx], dtype=X.dtype if X.dtype == np.float64 else np.float32)


def random_params(rng, D, G, var_lo=0.2, var_hi=3.0, mean_scale=3.0):
    """A random (not fitted) diagonal parameter set, for per-step parity inputs."""
    w = rng.dirichlet(np.ones(G))
    mu = rng.normal(0.0, mean_scale, size=(G, D))
    var = np.exp(rng.uniform(np.log(var_lo), np.log(var_hi), size=(G, D)))
    return w.astype(np.float32), mu.astype(np.float32), var.astype(np.float32)
