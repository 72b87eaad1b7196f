"""Host-side training driver over the C ABI: the learn() sequence of the
paper's Sec. 4 API (global statistics for the Mahalanobis distance, seeding,
k-means iterations, hand-off, EM iterations).  No arithmetic happens here;
every step is a call into libgmm.so on one stream.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import gmm


@dataclass
class Model:
    hefts: torch.Tensor   # (G,) float32
    means: torch.Tensor   # (G, D) float32
    covs: torch.Tensor    # (G, D) or (G, D, D) float32
    cov: int = gmm.COV_DIAG


@dataclass
class FitLog:
    inertia: list = field(default_factory=list)      # k-means, under each iteration's input means
    loglik: list = field(default_factory=list)       # EM, of each iteration's input parameters
    km_recomputed: list = field(default_factory=list)
    em_recomputed: list = field(default_factory=list)
    status: int = 0


class Trainer:
    """Owns the workspace and scalar outputs for one (N, D, G) problem."""

    def __init__(self, X, G, cov=gmm.COV_DIAG, prec=gmm.PREC_FP32):
        self.X = X
        self.N, self.D = X.shape
        self.G = int(G)
        self.cov = cov
        self.prec = prec
        dev = X.device
        self.ws = gmm.workspace(self.N, self.D, self.G, cov, prec, dev)
        self.scal = torch.zeros(4, dtype=torch.float64, device=dev)
        self.i64 = torch.zeros(2, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.counts = torch.zeros(self.G, dtype=torch.int64, device=dev)
        self.gmean = torch.zeros(self.D, dtype=torch.float64, device=dev)
        self.gvar = torch.zeros(self.D, dtype=torch.float64, device=dev)

    def global_stats(self):
        gmm.gmm_global_stats(self.X, self.gmean, self.gvar, self.ws)
        return self.gmean, self.gvar

    def kmeans_iter(self, means, dcovs, hefts, dist, var_floor, assign=None, prec=None):
        gmm.gmm_kmeans_iter(self.X, dist, self.gvar if dist == gmm.DIST_MAHA else None, var_floor,
                            means, dcovs, hefts, self.counts, assign, self.scal[0:1],
                            self.prec if prec is None else prec, self.i64[0:1], self.status,
                            self.ws)

    def em_iter(self, model: Model, var_floor, prec=None):
        gmm.gmm_em_iter(self.X, model.cov, model.hefts, model.means, model.covs, var_floor,
                        self.prec if prec is None else prec, self.scal[1:2], self.i64[1:2],
                        self.status, self.ws)

    def loglik(self, model: Model, per_sample=None, prec=None):
        gmm.gmm_loglik(self.X, model.cov, model.hefts, model.means, model.covs,
                       self.prec if prec is None else prec, self.scal[2:3], per_sample,
                       self.status, self.ws)
        return self.scal[2:3]


SEED_MODES = ("keep_existing", "static_subset", "random_subset", "static_spread",
              "random_spread")


def learn(X, G, dist=gmm.DIST_MAHA, init_means=None, km_iter=10, em_iter=10, var_floor=1e-10,
          prec=gmm.PREC_FP32, cov=gmm.COV_DIAG, record=True, seed_mode=None, rng_seed=0,
          em_tol=None):
    """Seeding, k-means, then EM (Sec. 4 learn()).

    seed_mode: one of SEED_MODES; "keep_existing" (the default when init_means,
    a (G, D) float32 device tensor, is given) starts from init_means; the other
    modes seed on the device with gmm_seed_means, the random ones from indices
    drawn on the host with NumPy's PCG64(rng_seed).  em_tol: stop EM once the
    mean log-likelihood rises by less than em_tol from one iteration to the
    next (each iteration reports that of its input parameters; this reads the
    value back to the host every iteration)."""
    import numpy as np

    tr = Trainer(X, G, cov, prec)
    N, D = X.shape
    dev = X.device
    if seed_mode is None:
        seed_mode = "keep_existing" if init_means is not None else "static_subset"
    if seed_mode not in SEED_MODES:
        raise ValueError(f"seed_mode must be one of {SEED_MODES}")
    if dist == gmm.DIST_MAHA:
        tr.global_stats()
    if seed_mode == "keep_existing":
        if init_means is None:
            raise ValueError("keep_existing needs init_means")
        means = init_means.clone().contiguous()
    else:
        means = torch.zeros(G, D, dtype=torch.float32, device=dev)
        rng = np.random.Generator(np.random.PCG64(rng_seed))
        if seed_mode == "static_subset":
            gmm.gmm_seed_means(X, gmm.SEED_SUBSET, means, tr.status, tr.ws)
        elif seed_mode == "random_subset":
            idx = rng.choice(N, G, replace=G > N)
            gmm.gmm_seed_means(X, gmm.SEED_SUBSET, means, tr.status, tr.ws,
                               idx=torch.as_tensor(idx, dtype=torch.int64, device=dev))
        else:
            first = 0 if seed_mode == "static_spread" else int(rng.integers(N))
            gmm.gmm_seed_means(X, gmm.SEED_SPREAD, means, tr.status, tr.ws,
                               gvar=tr.gvar if dist == gmm.DIST_MAHA else None,
                               var_floor=var_floor, first=first)
    dcovs = torch.ones(G, D, dtype=torch.float32, device=dev)
    hefts = torch.full((G,), 1.0 / G, dtype=torch.float32, device=dev)
    log = FitLog()
    log.status |= int(tr.status[0]) if seed_mode != "keep_existing" else 0
    for _ in range(km_iter):
        tr.kmeans_iter(means, dcovs, hefts, dist, var_floor)
        if record:
            log.inertia.append(float(tr.scal[0]))
            log.km_recomputed.append(int(tr.i64[0]))
            log.status |= int(tr.status[0])
    if cov == gmm.COV_FULL:
        covs = torch.diag_embed(dcovs).contiguous()
    else:
        covs = dcovs
    model = Model(hefts, means, covs, cov)
    prev = None
    for _ in range(em_iter):
        tr.em_iter(model, var_floor)
        if record or em_tol is not None:
            ll = float(tr.scal[1])
            log.loglik.append(ll)
            log.em_recomputed.append(int(tr.i64[1]))
            log.status |= int(tr.status[0])
            if em_tol is not None and prev is not None and ll - prev < em_tol:
                break
            prev = ll
    return model, log, tr
