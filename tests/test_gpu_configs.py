"""GPU parity at the benchmark configurations' own shapes, through the C ABI:
one k-means step and one EM step of the D=100/G=100/N=1e6 headline data set
(both arithmetic forms), the D=64/G=512 workload on a grid of 512 workgroups
(with run-to-run determinism of its atomic partials), full covariances at
D=32/G=64 (the LDS-staged flush of the map step) and at D=128, the
full-covariance log-likelihood, constructed k-means near ties, and graph
capture of single-model calls replayed against the eager results."""
import numpy as np
import pytest

from paper_1707_09094_amd import synth
from tests.parity import check_em, check_kmeans

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def G_():
    from paper_1707_09094_amd import gmm
    gmm.library()
    return gmm


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


class Runner:
    """Device copies of one data set plus the buffers of the single-model calls."""

    def __init__(self, gmm, X, G, cov=0):
        self.g = gmm
        self.X = X
        self.N, self.D = X.shape
        self.G = G
        self.cov = cov
        self.Xd = _t(X)
        self.ws = gmm.workspace(self.N, self.D, G, cov, 1, DEV)
        self.st = torch.zeros(1, dtype=torch.int32, device=DEV)
        self.nrec = torch.zeros(1, dtype=torch.int64, device=DEV)
        self.scal = torch.zeros(1, dtype=torch.float64, device=DEV)

    def kmeans(self, mu, gvar=None, prec=0):
        N, D, G = self.N, self.D, self.G
        m = _t(mu)
        dc = torch.zeros(G, D, device=DEV)
        h = torch.zeros(G, device=DEV)
        cnt = torch.zeros(G, dtype=torch.int64, device=DEV)
        asg = torch.zeros(N, dtype=torch.int32, device=DEV)
        gv = None if gvar is None else _t(gvar, torch.float64)
        self.g.gmm_kmeans_iter(self.Xd, 0 if gvar is None else 1, gv, 1e-10, m, dc, h, cnt, asg,
                               self.scal, prec, self.nrec, self.st, self.ws)
        torch.cuda.synchronize()
        return dict(means=m.cpu().numpy(), dcovs=dc.cpu().numpy(), hefts=h.cpu().numpy(),
                    counts=cnt.cpu().numpy(), assign=asg.cpu().numpy(),
                    inertia=float(self.scal.item()), nrec=int(self.nrec.item()),
                    status=int(self.st.item()))

    def em(self, w, mu, var, prec=0, floor=1e-10):
        h, m, c = _t(w), _t(mu), _t(var)
        self.g.gmm_em_iter(self.Xd, self.cov, h, m, c, floor, prec, self.scal, self.nrec, self.st,
                           self.ws)
        torch.cuda.synchronize()
        return dict(hefts=h.cpu().numpy(), means=m.cpu().numpy(), covs=c.cpu().numpy(),
                    loglik=float(self.scal.item()), nrec=int(self.nrec.item()),
                    status=int(self.st.item()))


def _same(a, b):
    for k in ("hefts", "means", "covs"):
        assert np.array_equal(a[k], b[k]), k
    assert a["loglik"] == b["loglik"]


# ------------------------------------------------ D=100, G=100, N=1e6 (headline)
def test_headline_size_kmeans_and_em_steps(G_, oracle):
    """The benchmark's data set at full size: a Mahalanobis k-means step after
    three k-means iterations, then one EM step of each arithmetic form from the
    k-means hand-off, each against the oracle on the same FP32 inputs (about
    3,900 samples per workgroup in the FP32 Welford runs)."""
    X, _ = synth.config2(N=1_000_000)
    N, D = X.shape
    G = 100
    r = Runner(G_, X, G)
    _, gv = oracle.global_stats(X)
    lam = oracle.maha_lambda(gv, 1e-10)
    mu = synth.static_subset(X, G)
    for _ in range(3):
        mu = r.kmeans(mu, gvar=gv, prec=1)["means"]
    rk = oracle.kmeans_iter(X, mu, lam, 1e-10)
    dists = oracle.kmeans_dists(X, mu, lam)
    for prec in (0, 1):
        gk = r.kmeans(mu, gvar=gv, prec=prec)
        assert gk["status"] == 0
        check_kmeans(gk, rk, dists, N)
    del dists
    w, mu1, var = gk["hefts"], gk["means"], gk["dcovs"]
    ref = oracle.em_iter(X, w, mu1, var, 1e-10)
    out = {}
    for prec in (0, 1):
        out[prec] = r.em(w, mu1, var, prec=prec)
        assert out[prec]["status"] == 0
        check_em(out[prec], ref, N)
    assert abs(out[0]["loglik"] - out[1]["loglik"]) <= 1e-7 * abs(ref.mean_loglik)
    assert out[1]["nrec"] >= N


# ------------------------------------------------ D=64, G=512 on 512 workgroups
def test_wide_config_on_full_grid_and_determinism(G_, oracle):
    """The D=64/G=512 recipe at N=65,536 (the 512-workgroup grid of the FP64
    matrix-core kernels): a Mahalanobis k-means step and an EM step of each
    arithmetic form from its hand-off against the oracle (FP32 form: the FP64
    matrix-core kernel; BF16x3 form: the sliced split-BF16 kernels, four
    slices of 128), the two forms' log-likelihoods within 1e-7 of each other,
    and each EM step run twice bit for bit (the FP64 kernel's map step adds
    partials with order-fixed atomics)."""
    X, _ = synth.config3(N=65_536)
    N, D = X.shape
    G = 512
    assert G_.gmm_em_path(D, G, G_.COV_DIAG, 0) == G_.PATH_WIDE_FP64
    assert G_.gmm_em_path(D, G, G_.COV_DIAG, 1) == G_.PATH_SLICED_BF16X3
    for prec in (0, 1):
        assert G_.gmm_kmeans_path(D, G, prec) == G_.PATH_WIDE_FP64
    r = Runner(G_, X, G)
    _, gv = oracle.global_stats(X)
    lam = oracle.maha_lambda(gv, 1e-10)
    mu = synth.static_subset(X, G)
    mu = r.kmeans(mu, gvar=gv)["means"]
    gk = r.kmeans(mu, gvar=gv)
    assert gk["status"] == 0
    check_kmeans(gk, oracle.kmeans_iter(X, mu, lam, 1e-10), oracle.kmeans_dists(X, mu, lam), N)
    w, mu1, var = gk["hefts"], gk["means"], gk["dcovs"]
    ref = oracle.em_iter(X, w, mu1, var, 1e-10)
    out = {}
    for prec in (0, 1):
        a = r.em(w, mu1, var, prec=prec)
        assert a["status"] == 0
        check_em(a, ref, N)
        b = r.em(w, mu1, var, prec=prec)
        _same(a, b)
        out[prec] = a
    assert abs(out[0]["loglik"] - out[1]["loglik"]) <= 1e-7 * abs(ref.mean_loglik)
    assert out[1]["nrec"] >= N


# ------------------------------------------------ full covariances
def _full_case(D, G, N, seed):
    X, truth = synth.full_gmm(seed + D, D, G, N)
    rng = np.random.Generator(np.random.PCG64(D * 1000 + G))
    w = rng.dirichlet(np.ones(G)).astype(np.float32)
    mu = X[rng.choice(N, G, replace=False)].astype(np.float32)
    S = truth.covs.astype(np.float32)
    S = (S + np.transpose(S, (0, 2, 1))) / 2
    return X, w, mu, S


@pytest.mark.parametrize("N,D,G", [(20_000, 32, 64), (2000, 20, 40), (3000, 128, 3)])
def test_em_step_full_config_shapes(G_, oracle, N, D, G):
    """D=32/G=64 and D=20/G=40 take the map step's LDS-staged flush (tile rows
    times components at least four times the per-component entries); D=128 is
    the largest full covariance the library takes (its reduce step needs more
    than 64 KB of LDS).  The D=32/G=64 step is also run twice bit for bit."""
    X, w, mu, S = _full_case(D, G, N, 900)
    r = Runner(G_, X, G, cov=G_.COV_FULL)
    gpu = r.em(w, mu, S, floor=1e-6)
    assert gpu["status"] == 0
    check_em(gpu, oracle.em_iter(X, w, mu, S, 1e-6, full=True), N, full=True)
    if D == 32:
        _same(gpu, r.em(w, mu, S, floor=1e-6))


@pytest.mark.parametrize("N,D,G", [(5000, 4, 3), (3000, 32, 8), (2000, 48, 5), (1500, 80, 3)])
def test_loglik_full(G_, oracle, N, D, G):
    """gmm_loglik with full covariances: the mean and every per-sample value."""
    X, w, mu, S = _full_case(D, G, N, 950)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    ps = torch.zeros(N, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = G_.workspace(N, D, G, G_.COV_FULL, 0, DEV)
    G_.gmm_loglik(_t(X), G_.COV_FULL, _t(w), _t(mu), _t(S), 0, ll, ps, st, ws)
    torch.cuda.synchronize()
    assert st.item() == 0
    ref, rps = oracle.loglik(X, w, mu, S, full=True, per_sample=True)
    assert abs(ll.item() - ref) <= 1e-6 * abs(ref)
    np.testing.assert_allclose(ps.cpu().numpy(), rps, rtol=2e-6, atol=2e-5)


# ------------------------------------------------ k-means near ties
def _tie_data(seed, D, G, n_mid):
    """Well separated integer-valued means, samples around them, and n_mid
    samples at (or one FP32 ulp off) the midpoint of two means: exact ties and
    gaps far below 1e-6 relative."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.integers(-40, 41, size=(G, D)).astype(np.float32)
    lab = rng.integers(0, G, size=4000)
    X = (mu[lab] + rng.normal(size=(4000, D))).astype(np.float32)
    a = rng.integers(0, G, size=n_mid)
    b = (a + 1 + rng.integers(0, G - 1, size=n_mid)) % G
    mid = ((mu[a] + mu[b]) / 2).astype(np.float32)
    bump = rng.integers(0, 3, size=n_mid)  # 0: exact midpoint; 1, 2: one ulp off
    d0 = rng.integers(0, D, size=n_mid)
    for k in range(n_mid):
        if bump[k]:
            v = mid[k, d0[k]]
            mid[k, d0[k]] = np.nextafter(v, np.float32(np.inf if bump[k] == 1 else -np.inf))
    X = np.concatenate([X, mid]).astype(np.float32)
    return X[rng.permutation(len(X))], mu


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("D,G,maha", [(8, 16, False), (8, 16, True), (40, 100, True),
                                      (8, 150, False)])
def test_kmeans_near_ties(G_, oracle, D, G, maha, prec):
    X, mu = _tie_data(D * 100 + G, D, G, 600)
    N = len(X)
    gv = oracle.global_stats(X)[1] if maha else None
    lam = oracle.maha_lambda(gv, 1e-10) if maha else np.ones(D)
    r = Runner(G_, X, G)
    gk = r.kmeans(mu, gvar=gv, prec=prec)
    assert gk["status"] == 0
    rk = oracle.kmeans_iter(X, mu, lam, 1e-10)
    n_amb = check_kmeans(gk, rk, oracle.kmeans_dists(X, mu, lam), N)
    assert n_amb >= 50  # the ambiguous branch of the check is exercised


# ------------------------------------------------ graph capture (single model)
@pytest.mark.parametrize("D,G,cov", [(40, 16, 0), (64, 200, 0), (6, 4, 1)])
def test_graph_capture_replay_single_model(G_, D, G, cov):
    """One k-means iteration and two EM iterations of the single-model calls
    captured into a graph; every replay, with eager work and synchronisation
    between replays, reproduces the eager sequence bit for bit."""
    N = 20_000
    X, _ = synth.diag_gmm(31 + D, D, min(G, 16), N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    Xd = _t(X)
    ws = G_.workspace(N, D, G, cov, 1, DEV)
    mu0 = _t(synth.static_subset(X, G))
    means, dcovs = mu0.clone(), torch.ones(G, D, device=DEV)
    hefts = torch.zeros(G, device=DEV)
    covs = torch.zeros((G, D, D) if cov else (G, D), device=DEV)
    counts = torch.zeros(G, dtype=torch.int64, device=DEV)
    inertia = torch.zeros(1, dtype=torch.float64, device=DEV)
    ll = torch.zeros(2, dtype=torch.float64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    gm = torch.zeros(D, dtype=torch.float64, device=DEV)
    gv = torch.zeros(D, dtype=torch.float64, device=DEV)
    G_.gmm_global_stats(Xd, gm, gv, ws)

    def reset():
        means.copy_(mu0)

    def seq():
        G_.gmm_kmeans_iter(Xd, G_.DIST_MAHA, gv, 1e-10, means, dcovs, hefts, counts, None,
                           inertia, 1, None, st, ws)
        if cov:
            covs.copy_(torch.diag_embed(dcovs))
        else:
            covs.copy_(dcovs)
        G_.gmm_em_iter(Xd, cov, hefts, means, covs, 1e-10, 1, ll[0:1], None, st, ws)
        G_.gmm_em_iter(Xd, cov, hefts, means, covs, 1e-10, 1, ll[1:2], None, st, ws)

    def snap():
        return [t.cpu().numpy().copy() for t in (hefts, means, covs, counts, inertia, ll, st)]

    reset()
    seq()
    torch.cuda.synchronize()
    eager = snap()
    assert eager[-1][0] == 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the side stream before capture
        reset()
        seq()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        seq()
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, e in zip(snap(), eager):
            np.testing.assert_array_equal(a, e, err_msg=f"replay {rep}")
        _ = torch.ones(1000, device=DEV).sum().item()  # eager work between replays
