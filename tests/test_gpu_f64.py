"""GPU parity of the FP64-data path (gmm_*_f64: FP64 samples and parameters,
the paper's gmm_diag precision) against the oracle's FP64-sample entry
points, element by element at FP64 tolerances: the D=4/G=4/N=1e4 and
D=100/G=100/N=1e6 shapes (k-means step, EM step, log-likelihood, global
statistics), data that FP32 cannot hold, tiles with ragged tails, the largest
supported shape, run-to-run determinism and the shape limits."""
import numpy as np
import pytest

from paper_1707_09094_amd import synth
from tests.parity import check_em, check_kmeans

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-11      # parameters: FP64 sums in another order than the oracle's
LL_TOL = 1e-12   # mean log-likelihood, relative


@pytest.fixture(scope="module")
def G_():
    from paper_1707_09094_amd import gmm
    gmm.library()
    return gmm


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


class R64:
    def __init__(self, gmm, X, G):
        self.g, self.X = gmm, X
        self.N, self.D = X.shape
        self.G = G
        self.Xd = _t(X)
        self.ws = gmm.workspace_f64(self.N, self.D, G, DEV)
        self.st = torch.zeros(1, dtype=torch.int32, device=DEV)
        self.scal = torch.zeros(1, dtype=torch.float64, device=DEV)

    def stats(self):
        m = torch.zeros(self.D, dtype=torch.float64, device=DEV)
        v = torch.zeros(self.D, dtype=torch.float64, device=DEV)
        self.g.gmm_global_stats_f64(self.Xd, m, v, self.ws)
        return m.cpu().numpy(), v.cpu().numpy()

    def kmeans(self, mu, gvar=None):
        N, D, G = self.N, self.D, self.G
        m = _t(mu)
        dc = torch.zeros(G, D, dtype=torch.float64, device=DEV)
        h = torch.zeros(G, dtype=torch.float64, device=DEV)
        cnt = torch.zeros(G, dtype=torch.int64, device=DEV)
        asg = torch.zeros(N, dtype=torch.int32, device=DEV)
        gv = None if gvar is None else _t(gvar)
        self.g.gmm_kmeans_iter_f64(self.Xd, 0 if gvar is None else 1, gv, 1e-10, m, dc, h, cnt,
                                   asg, self.scal, None, self.st, self.ws)
        torch.cuda.synchronize()
        return dict(means=m.cpu().numpy(), dcovs=dc.cpu().numpy(), hefts=h.cpu().numpy(),
                    counts=cnt.cpu().numpy(), assign=asg.cpu().numpy(),
                    inertia=float(self.scal.item()), status=int(self.st.item()))

    def em(self, w, mu, var, floor=1e-10):
        h, m, c = _t(w), _t(mu), _t(var)
        self.g.gmm_em_iter_f64(self.Xd, h, m, c, floor, self.scal, self.st, self.ws)
        torch.cuda.synchronize()
        return dict(hefts=h.cpu().numpy(), means=m.cpu().numpy(), covs=c.cpu().numpy(),
                    loglik=float(self.scal.item()), status=int(self.st.item()))

    def loglik(self, w, mu, var):
        ps = torch.zeros(self.N, dtype=torch.float64, device=DEV)
        self.g.gmm_loglik_f64(self.Xd, _t(w), _t(mu), _t(var), self.scal, ps, self.st, self.ws)
        torch.cuda.synchronize()
        return float(self.scal.item()), ps.cpu().numpy(), int(self.st.item())


def _fit_chain(oracle, r, X, G, lam, gv, km_steps):
    """k-means steps on the GPU from the static subset, the last one checked
    against the oracle; returns its hand-off."""
    mu = synth.static_subset(X, G)
    for _ in range(km_steps - 1):
        mu = r.kmeans(mu, gvar=gv)["means"]
    gk = r.kmeans(mu, gvar=gv)
    assert gk["status"] == 0
    rk = oracle.kmeans_iter(X, mu, lam, 1e-10)
    check_kmeans(gk, rk, oracle.kmeans_dists(X, mu, lam), len(X), tol=TOL, rel_gap=1e-12)
    return gk


@pytest.mark.parametrize("cfg", ["d4g4", "d100g100"])
def test_f64_config_shapes(G_, oracle, cfg):
    """Global statistics, a Mahalanobis k-means step, an EM step from its
    hand-off and the log-likelihood, each against the oracle fed the same FP64
    inputs."""
    if cfg == "d4g4":
        X, _ = synth.config1(dtype=np.float64)
        G = 4
    else:
        X, _ = synth.config2(N=1_000_000, dtype=np.float64)
        G = 100
    N, D = X.shape
    r = R64(G_, X, G)
    m, v = r.stats()
    rm, rv = oracle.global_stats(X)
    np.testing.assert_allclose(m, rm, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(v, rv, rtol=1e-12)
    lam = oracle.maha_lambda(rv, 1e-10)
    gk = _fit_chain(oracle, r, X, G, lam, rv, 3)
    w, mu, var = gk["hefts"], gk["means"], gk["dcovs"]
    gpu = r.em(w, mu, var)
    assert gpu["status"] == 0
    ref = oracle.em_iter(X, w, mu, var, 1e-10)
    check_em(gpu, ref, N, tol=TOL, ll_tol=LL_TOL)
    ll, ps, st = r.loglik(gpu["hefts"], gpu["means"], gpu["covs"])
    rll, rps = oracle.loglik(X, gpu["hefts"], gpu["means"], gpu["covs"], per_sample=True)
    assert st == 0
    assert abs(ll - rll) <= LL_TOL * abs(rll)
    np.testing.assert_allclose(ps, rps, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,D,G", [(1, 3, 2), (63, 17, 5), (3001, 128, 7), (4097, 64, 40),
                                   (2500, 8, 150), (3001, 100, 300)])
def test_f64_em_step_random_params(G_, oracle, N, D, G):
    """Unfitted parameters near the data (overlapping components), tiles with
    ragged tails, one sample, and more components than one workgroup's waves."""
    X, _ = synth.diag_gmm(800 + N + D, D, max(G, 2), N, "normal", 0.0, 4.0, "loguniform", 0.1,
                          10.0, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(N + G))
    w, mu, var = synth.random_params(rng, D, G)
    if N >= G:
        mu = X[rng.choice(N, G, replace=False)]
    r = R64(G_, X, G)
    gpu = r.em(w.astype(np.float64), mu.astype(np.float64), var.astype(np.float64))
    assert gpu["status"] == 0
    ref = oracle.em_iter(X, w, mu, var, 1e-10)
    # weights, means and log-likelihood at the FP64 bar
    check_em({**gpu, "covs": ref.covs}, ref, N, tol=TOL, ll_tol=LL_TOL)
    # variances: the one-pass moments about the old mean give S2/L - dm^2 with
    # dm the mean's move in this step, so their rounding is relative to
    # sigma^2 + dm^2 rather than sigma^2 (random starting means move far)
    live = ref.L >= 1.0
    dm2 = (ref.means - np.asarray(mu, np.float64)) ** 2 / ref.covs
    err = np.abs(gpu["covs"] - ref.covs) / ref.covs
    assert np.all(err[live] <= 1e-12 * (1.0 + dm2[live])), err[live].max()


def test_f64_data_beyond_fp32(G_, oracle):
    """Deviations of 1e-3 around an offset of 1e6 (FP32 spacing there: 0.0625):
    the EM step keeps them.  Two clusters 10 standard deviations apart, so every
    responsibility is 0 or 1 to FP64 rounding and the exact answer is each
    cluster's mean and population variance, taken here with correctly rounded
    sums (math.fsum).  The oracle's plain sequential sums of 1e4 values near 1e6
    are themselves off by ~1e-8 in the mean, ~1e-10 relative in these 1e-6
    variances, so it is held to that."""
    import math
    rng = np.random.Generator(np.random.PCG64(5))
    N, D = 20_000, 6
    X = 1e6 + rng.normal(size=(N, D)) * 1e-3 * rng.uniform(0.5, 2.0, size=D)
    X[N // 2:, :3] += 0.01
    halves = (X[:N // 2], X[N // 2:])
    w = np.array([0.5, 0.5])
    mu = np.stack([h.mean(0) for h in halves]) + 1e-4
    var = np.full((2, D), 1e-6)
    r = R64(G_, X, 2)
    gpu = r.em(w, mu, var, floor=1e-30)
    assert gpu["status"] == 0
    for g, h in enumerate(halves):
        m = np.array([math.fsum(h[:, d]) / len(h) for d in range(D)])
        v = np.array([math.fsum((h[:, d] - m[d]) ** 2) / len(h) for d in range(D)])
        np.testing.assert_allclose(gpu["means"][g], m, rtol=1e-15)
        np.testing.assert_allclose(gpu["covs"][g], v, rtol=1e-12)
        assert gpu["hefts"][g] == 0.5
    ref = oracle.em_iter(X, w, mu, var, 1e-30)
    check_em(gpu, ref, N, tol=1e-9, ll_tol=LL_TOL)
    _, v = r.stats()
    vx = np.array([math.fsum((X[:, d] - math.fsum(X[:, d]) / N) ** 2) / N for d in range(D)])
    np.testing.assert_allclose(v, vx, rtol=1e-12)
    assert X.astype(np.float32).astype(np.float64)[:, 3:].var(0).max() == 0.0


def test_f64_deterministic_and_limits(G_):
    X, _ = synth.diag_gmm(9, 32, 16, 30_000, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0,
                          dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(9))
    w, mu, var = synth.random_params(rng, 32, 16)
    mu = X[rng.choice(30_000, 16, replace=False)]
    r = R64(G_, X, 16)
    a = r.em(w.astype(np.float64), mu, var.astype(np.float64))
    b = r.em(w.astype(np.float64), mu, var.astype(np.float64))
    for k in ("hefts", "means", "covs"):
        assert np.array_equal(a[k], b[k]), k
    assert a["loglik"] == b["loglik"]
    assert G_.gmm_workspace_bytes_f64(100, 129, 4) == 0   # D beyond 128
    assert G_.gmm_workspace_bytes_f64(100, 128, 2000) == 0  # tile beyond LDS
    assert G_.gmm_workspace_bytes_f64(100, 128, 400) > 0
    with pytest.raises(G_.GmmError):
        G_.gmm_em_iter_f64(r.Xd, _t(w), _t(mu), _t(var), -1.0, r.scal, r.st, r.ws)
