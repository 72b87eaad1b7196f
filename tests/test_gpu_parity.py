"""GPU parity: the HIP path through the C ABI vs the FP64 oracle, element by
element on the same seeded inputs (same FP32 parameters into both, one
iteration), plus edge cases, error paths and run-to-run determinism."""
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


def gpu_em_step(gmm, X, w, mu, var, floor, prec=0, full=False, ws=None):
    N, D = X.shape
    G = len(w)
    cov = gmm.COV_FULL if full else gmm.COV_DIAG
    Xd = _t(X)
    h, m, c = _t(w), _t(mu), _t(var)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    nrec = torch.zeros(1, dtype=torch.int64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    if ws is None:
        ws = gmm.workspace(N, D, G, cov, prec, DEV)
    gmm.gmm_em_iter(Xd, cov, h, m, c, floor, prec, ll, nrec, st, ws)
    torch.cuda.synchronize()
    return dict(hefts=h.cpu().numpy(), means=m.cpu().numpy(), covs=c.cpu().numpy(),
                loglik=float(ll.item()), nrec=int(nrec.item()), status=int(st.item()))


def gpu_kmeans_step(gmm, X, mu, dist, floor, gvar=None, prec=0, ldx=None):
    N, D = X.shape
    G = mu.shape[0]
    if ldx is None or ldx == D:
        Xd = _t(X)
    else:  # rows ldx floats apart
        wide = np.zeros((N, ldx), np.float32)
        wide[:, :D] = X
        Xd = _t(wide)[:, :D]
    m = _t(mu)
    dc = torch.zeros(G, D, device=DEV)
    h = torch.zeros(G, device=DEV)
    cnt = torch.zeros(G, dtype=torch.int64, device=DEV)
    asg = torch.zeros(N, dtype=torch.int32, device=DEV)
    inr = torch.zeros(1, dtype=torch.float64, device=DEV)
    nrec = torch.zeros(1, dtype=torch.int64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = gmm.workspace(N, D, G, gmm.COV_DIAG, prec, DEV)
    gv = None if gvar is None else _t(gvar, torch.float64)
    gmm.gmm_kmeans_iter(Xd, dist, gv, floor, m, dc, h, cnt, asg, inr, prec, nrec, st, ws)
    torch.cuda.synchronize()
    return dict(means=m.cpu().numpy(), dcovs=dc.cpu().numpy(), hefts=h.cpu().numpy(),
                counts=cnt.cpu().numpy(), assign=asg.cpu().numpy(), inertia=float(inr.item()),
                nrec=int(nrec.item()), status=int(st.item()))


def _params(seed, D, G, X=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    w, mu, var = synth.random_params(rng, D, G)
    if X is not None:  # means near data so components own samples
        mu = X[rng.choice(len(X), G, replace=False)].astype(np.float32)
    return w, mu, var


# ---------------------------------------------------------------- global stats
@pytest.mark.parametrize("N,D", [(1, 3), (10_000, 4), (50_001, 100), (777, 1)])
def test_global_stats(G_, oracle, N, D):
    rng = np.random.Generator(np.random.PCG64(N + D))
    X = (rng.normal(size=(N, D)) * rng.uniform(0.1, 10, D) + rng.normal(size=D) * 50).astype(np.float32)
    m = torch.zeros(D, dtype=torch.float64, device=DEV)
    v = torch.zeros(D, dtype=torch.float64, device=DEV)
    ws = G_.workspace(N, D, 1, device=DEV)
    G_.gmm_global_stats(_t(X), m, v, ws)
    rm, rv = oracle.global_stats(X)
    np.testing.assert_allclose(m.cpu().numpy(), rm, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(v.cpu().numpy(), rv, rtol=1e-10, atol=1e-300)


# ---------------------------------------------------------------- EM, diagonal
# (N, D, G) spanning several tiles, ragged tails and the degenerate shapes of
# the one-pass kernels (D, G <= 128), run in both arithmetic forms
EM_ONEPASS = [
    (10_000, 4, 4),
    (1, 3, 2),
    (5, 2, 3),
    (63, 17, 5),
    (1000, 1, 3),
    (3001, 128, 7),
    (20_000, 100, 100),
    (4097, 64, 40),
    (2000, 40, 128),
    (50_000, 64, 16),   # per-wave map-step states, largest LDS layout
    (20_000, 40, 9),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("N,D,G", EM_ONEPASS)
def test_em_step_diag(G_, oracle, N, D, G, prec):
    assert G_.gmm_em_path(D, G, G_.COV_DIAG, prec) == (
        G_.PATH_ONEPASS_BF16X3 if prec else G_.PATH_ONEPASS_FP32)
    X, _ = synth.diag_gmm(1000 + N + D, D, max(G, 2), N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    w, mu, var = _params(N * 7 + G, D, G, X if N >= G else None)
    floor = 1e-10
    gpu = gpu_em_step(G_, X, w, mu, var, floor, prec=prec)
    assert gpu["status"] == 0
    ref = oracle.em_iter(X, w, mu, var, floor)
    check_em(gpu, ref, N)


# shapes outside the one-pass envelope: G > 128 runs the FP64 matrix-core
# kernel for the FP32 form and the sliced split-BF16 kernels for the BF16x3
# form; D > 128 runs the generic kernel for both (asserted through the
# dispatch query)
EM_OTHER = [
    (1500, 200, 5, "generic"),
    (2500, 8, 150, "wide"),
    (5000, 64, 512, "wide"),
    (3001, 100, 300, "wide"),
    (3001, 128, 200, "wide"),   # two dimensions per lane, slices below 128
    (129, 33, 129, "wide"),     # slices of 80 and 49, ragged round
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("N,D,G,path", EM_OTHER)
def test_em_step_diag_beyond_onepass(G_, oracle, N, D, G, path, prec):
    if path == "generic":
        want = G_.PATH_GENERIC
    else:
        want = G_.PATH_SLICED_BF16X3 if prec else G_.PATH_WIDE_FP64
    assert G_.gmm_em_path(D, G, G_.COV_DIAG, prec) == want
    X, _ = synth.diag_gmm(1000 + N + D, D, max(G, 2), N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    w, mu, var = _params(N * 7 + G, D, G, X if N >= G else None)
    gpu = gpu_em_step(G_, X, w, mu, var, 1e-10, prec=prec)
    assert gpu["status"] == 0
    check_em(gpu, oracle.em_iter(X, w, mu, var, 1e-10), N)
    if want == G_.PATH_SLICED_BF16X3:
        assert gpu["nrec"] >= N  # every sample's best component is recomputed


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("N,D,G", [(777, 64, 128), (777, 64, 130), (777, 64, 200), (777, 64, 16),
                                   (5000, 40, 12), (777, 40, 64)])
def test_em_heavy_sample_after_tiny_weights(G_, oracle, N, D, G, prec):
    """Unfitted components that collapse onto one or two samples: far-off
    samples with responsibilities ~1e-11 can open a component's run in a
    workgroup, and the heavy sample that follows must not inherit their
    rounding in the running mean (variances of ~1e-6 against a data spread of
    ~16; one-pass kernels at G <= 128, sliced kernels beyond, FP64 kernel for
    the FP32 form beyond)."""
    X, _ = synth.diag_gmm(7000 + 13 + D, D, G, N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    rng = np.random.Generator(np.random.PCG64(7000 + 13 + D + 1))
    w = rng.dirichlet(np.ones(G)).astype(np.float32)
    mu = X[rng.choice(N, G, replace=False)].astype(np.float32)
    var = np.exp(rng.uniform(np.log(0.5), np.log(5.0), size=(G, D))).astype(np.float32)
    gpu = gpu_em_step(G_, X, w, mu, var, 1e-10, prec=prec)
    assert gpu["status"] == 0
    check_em(gpu, oracle.em_iter(X, w, mu, var, 1e-10), N)


@pytest.mark.parametrize("N,D,G", [(200_000, 100, 100), (50_000, 40, 64), (100_000, 40, 16)])
def test_em_forms_agree_on_fitted_model(G_, oracle, N, D, G):
    """From a k-means hand-off (the realistic regime: most samples have one
    near component), both arithmetic forms match the oracle and each other."""
    X, _ = synth.diag_gmm(4242 + D, D, G, N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    _, gv = oracle.global_stats(X)
    mu = synth.static_subset(X, G)
    for _ in range(3):
        gk = gpu_kmeans_step(G_, X, mu, 1, 1e-10, gvar=gv)
        mu = gk["means"]
    w, var = gk["hefts"], gk["dcovs"]
    ref = oracle.em_iter(X, w, mu, var, 1e-10)
    a = gpu_em_step(G_, X, w, mu, var, 1e-10, prec=0)
    b = gpu_em_step(G_, X, w, mu, var, 1e-10, prec=1)
    check_em(a, ref, N)
    check_em(b, ref, N)
    assert abs(a["loglik"] - b["loglik"]) <= 1e-7 * abs(a["loglik"])
    assert b["nrec"] >= N  # every sample's best component is recomputed


def test_em_step_config1_and_trajectory(G_, oracle):
    """Config 1 (D=4, G=4, N=1e4): 10 Mahalanobis k-means + 10 EM iterations;
    every step compared with the oracle fed the same FP32 inputs, and the
    trajectories' log-likelihood non-decreasing."""
    X, _ = synth.config1()
    N, D = X.shape
    G = 4
    _, gv = oracle.global_stats(X)
    lam = oracle.maha_lambda(gv, 1e-10)
    mu = synth.static_subset(X, G)
    for _ in range(10):
        gk = gpu_kmeans_step(G_, X, mu, 1, 1e-10, gvar=gv)
        rk = oracle.kmeans_iter(X, mu, lam, 1e-10)
        ok = rk.gap >= 1e-6
        assert np.array_equal(gk["assign"][ok], rk.assign[ok])
        mu = gk["means"]
    w, var = gk["hefts"], gk["dcovs"]
    prev = -np.inf
    for _ in range(10):
        gpu = gpu_em_step(G_, X, w, mu, var, 1e-10)
        ref = oracle.em_iter(X, w, mu, var, 1e-10)
        check_em(gpu, ref, N)
        assert gpu["loglik"] >= prev - 1e-6 * abs(gpu["loglik"])
        prev = gpu["loglik"]
        w, mu, var = gpu["hefts"], gpu["means"], gpu["covs"]


def test_em_single_component_closed_form(G_):
    """N_G = 1 (Eqs. 5-7 with l = 1): sample mean and population variance."""
    rng = np.random.Generator(np.random.PCG64(3))
    X = (rng.normal(size=(5000, 6)) * 2 + 3).astype(np.float32)
    gpu = gpu_em_step(G_, X, np.ones(1, np.float32), np.zeros((1, 6), np.float32),
                      np.ones((1, 6), np.float32), 1e-10)
    X64 = X.astype(np.float64)
    assert abs(gpu["hefts"][0] - 1.0) <= 1e-6
    np.testing.assert_allclose(gpu["means"][0], X64.mean(0), rtol=1e-5)
    np.testing.assert_allclose(gpu["covs"][0], X64.var(0), rtol=1e-5)


def test_em_floor_and_zero_weight(G_, oracle):
    """Constant dimension -> variance exactly the floor; a zero-weight component
    gets no responsibility, weight 0, and keeps its parameters."""
    rng = np.random.Generator(np.random.PCG64(4))
    X = rng.normal(size=(3000, 3)).astype(np.float32)
    X[:, 2] = 1.25
    w = np.array([0.5, 0.5, 0.0], np.float32)
    mu = np.array([[-1, 0, 1.25], [1, 0, 1.25], [5, 5, 5]], np.float32)
    var = np.ones((3, 3), np.float32)
    gpu = gpu_em_step(G_, X, w, mu, var, 1e-3)
    ref = oracle.em_iter(X, w, mu, var, 1e-3)
    assert gpu["covs"][0, 2] == np.float32(1e-3) and gpu["covs"][1, 2] == np.float32(1e-3)
    assert gpu["hefts"][2] == 0.0
    np.testing.assert_array_equal(gpu["means"][2], mu[2])
    check_em(gpu, ref, len(X))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("N,D,G", [(3000, 40, 16), (2000, 100, 100), (1500, 8, 150)])
def test_em_floored_singleton_component(G_, oracle, N, D, G, prec):
    """A k-means hand-off can leave a one-sample cluster whose variances sit at
    the floor: its log-density spans ~1e10 nats over the data, far beyond the
    near window, so the screening form's rounding error must widen the window
    for that component (and the reference of the log-sum-exp must not come
    from its screened value)."""
    X, _ = synth.diag_gmm(77 + D, D, 8, N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    w, mu, var = _params(G + D, D, G, X)
    mu[3] = X[11]
    var[3] = 1e-10
    mu[5] = X[200] + 0.01
    var[5] = 1e-8
    w = (w / w.sum()).astype(np.float32)
    for floor in (1e-10,):
        gpu = gpu_em_step(G_, X, w, mu, var, floor, prec=prec)
        assert gpu["status"] == 0
        ref = oracle.em_iter(X, w, mu, var, floor)
        assert ref.L[3] > 0.5  # the floored component keeps its own sample
        check_em(gpu, ref, N)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    G_.gmm_loglik(_t(X), G_.COV_DIAG, _t(w), _t(mu), _t(var), prec, ll, None, st,
                  G_.workspace(N, D, G, G_.COV_DIAG, prec, DEV))
    ref_ll = oracle.loglik(X, w, mu, var)
    assert abs(ll.item() - ref_ll) <= 1e-6 * abs(ref_ll)


def test_em_nan_sets_status(G_):
    X = np.ones((100, 3), np.float32)
    X[17, 1] = np.nan
    gpu = gpu_em_step(G_, X, np.ones(1, np.float32), np.zeros((1, 3), np.float32),
                      np.ones((1, 3), np.float32), 1e-6)
    assert gpu["status"] & 1


def test_em_nonpositive_variance_sets_status(G_):
    X = np.zeros((50, 2), np.float32)
    gpu = gpu_em_step(G_, X, np.ones(2, np.float32) / 2, np.zeros((2, 2), np.float32),
                      np.array([[1, 1], [1, 0]], np.float32), 1e-6)
    assert gpu["status"] & 1


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_em_deterministic(G_, prec):
    X, _ = synth.diag_gmm(55, 32, 16, 30_000, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    w, mu, var = _params(5, 32, 16, X)
    a = gpu_em_step(G_, X, w, mu, var, 1e-10, prec=prec)
    b = gpu_em_step(G_, X, w, mu, var, 1e-10, prec=prec)
    for k in ("hefts", "means", "covs"):
        assert np.array_equal(a[k], b[k]), k
    assert a["loglik"] == b["loglik"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("D,G,ldx", [(5, 3, 8), (40, 12, 41), (40, 40, 48)])
def test_em_row_stride(G_, oracle, D, G, ldx, prec):
    """X with a row stride larger than D (ldx > D); in the BF16x3 form these
    shapes run the staged E-step (per-wave map step at G=12, owners at G=40)."""
    N = 2000
    X, _ = synth.diag_gmm(56 + D, D, G, N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    w, mu, var = _params(6, D, G, X)
    wide = np.zeros((N, ldx), np.float32)
    wide[:, :D] = X
    Xd = _t(wide)[:, :D]
    cov = G_.COV_DIAG
    h, m, c = _t(w), _t(mu), _t(var)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = G_.workspace(N, D, G, cov, prec, DEV)
    G_.gmm_em_iter(Xd, cov, h, m, c, 1e-10, prec, ll, None, st, ws)
    assert int(st.item()) == 0
    gpu = dict(hefts=h.cpu().numpy(), means=m.cpu().numpy(), covs=c.cpu().numpy(),
               loglik=float(ll.item()))
    check_em(gpu, oracle.em_iter(X, w, mu, var, 1e-10), N)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("D,G,ldx", [(40, 12, 41), (40, 40, 48)])
def test_kmeans_row_stride(G_, oracle, D, G, ldx, prec):
    """k-means on X with a row stride larger than D (the staged matrix-core
    form in BF16x3: per-wave accumulation at G=12, owners at G=40)."""
    X, _ = synth.diag_gmm(88 + D, D, G, 3001, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    mu = synth.static_subset(X, G)
    gv = oracle.global_stats(X)[1]
    lam = oracle.maha_lambda(gv, 1e-10)
    gk = gpu_kmeans_step(G_, X, mu, 1, 1e-10, gvar=gv, prec=prec, ldx=ldx)
    assert gk["status"] == 0
    check_kmeans(gk, oracle.kmeans_iter(X, mu, lam, 1e-10), oracle.kmeans_dists(X, mu, lam), len(X))


# ---------------------------------------------------------------- loglik
@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("N,D,G", [(10_000, 4, 4), (777, 33, 9), (1, 2, 1), (3000, 100, 100),
                                   (900, 150, 3), (3001, 64, 300), (2000, 100, 260),
                                   (1, 5, 140)])
def test_loglik_diag(G_, oracle, N, D, G, prec):
    X, _ = synth.diag_gmm(77 + N, D, max(G, 2), N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    w, mu, var = _params(8, D, G, X if N >= G else None)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    ps = torch.zeros(N, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = G_.workspace(N, D, G, device=DEV)
    G_.gmm_loglik(_t(X), 0, _t(w), _t(mu), _t(var), prec, ll, ps, st, ws)
    ref, rps = oracle.loglik(X, w, mu, var, per_sample=True)
    assert abs(ll.item() - ref) <= 1e-6 * abs(ref)
    np.testing.assert_allclose(ps.cpu().numpy(), rps, rtol=2e-6, atol=2e-5)


# ---------------------------------------------------------------- k-means
@pytest.mark.parametrize("N,D,G,maha", [(10_000, 4, 4, True), (20_000, 100, 100, True),
                                        (999, 3, 7, False), (1, 2, 1, False), (4, 2, 9, False),
                                        (3000, 40, 128, True), (2000, 150, 6, True),
                                        (2500, 8, 160, False), (777, 1, 5, True),
                                        (5000, 128, 128, True), (3001, 65, 17, False),
                                        (1025, 40, 64, False), (129, 40, 16, True),
                                        (6000, 64, 512, True), (3001, 100, 300, False),
                                        (2000, 64, 1100, True), (1000, 300, 3, True),
                                        (50_000, 64, 16, True), (20_000, 40, 9, False)])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_kmeans_step(G_, oracle, N, D, G, maha, prec):
    X, _ = synth.diag_gmm(300 + N, D, max(G, 2), N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    mu = synth.static_subset(X, G) if N >= G else np.concatenate(
        [X, np.full((G - N, D), 100.0, np.float32)])
    gv = oracle.global_stats(X)[1] if maha else None
    lam = oracle.maha_lambda(gv, 1e-10) if maha else np.ones(D)
    gk = gpu_kmeans_step(G_, X, mu, 1 if maha else 0, 1e-10, gvar=gv, prec=prec)
    rk = oracle.kmeans_iter(X, mu, lam, 1e-10)
    assert gk["status"] == 0
    check_kmeans(gk, rk, oracle.kmeans_dists(X, mu, lam), N)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_kmeans_resurrection_golden(G_, prec):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "resurrection_1d.json")) as f:
        gd = json.load(f)
    X = np.array(gd["X"], np.float32)[:, None]
    mu = np.array(gd["means_in"], np.float32)[:, None]
    gk = gpu_kmeans_step(G_, X, mu, 0, gd["var_floor"], prec=prec)
    assert list(gk["assign"]) == gd["assign"]
    assert list(gk["counts"]) == gd["counts"]
    np.testing.assert_allclose(gk["means"][:, 0], gd["means_out"], rtol=1e-7)
    np.testing.assert_allclose(gk["dcovs"][:, 0], gd["dcovs_out"], rtol=1e-6)
    np.testing.assert_allclose(gk["hefts"], gd["hefts_out"], rtol=1e-7)
    assert abs(gk["inertia"] - gd["inertia"]) <= 1e-9 * gd["inertia"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_kmeans_duplicate_means_tie(G_, prec):
    X = np.array([[0.0, 0.0], [1.0, 1.0], [5.0, 5.0]], np.float32)
    mu = np.array([[5.0, 5.0], [0.5, 0.5], [0.5, 0.5]], np.float32)
    gk = gpu_kmeans_step(G_, X, mu, 0, 1e-10, prec=prec)
    assert list(gk["assign"]) == [1, 1, 0]
    assert gk["nrec"] >= 2


@pytest.mark.parametrize("D,G", [(16, 200), (100, 260)])
def test_kmeans_duplicate_means_tie_wide(G_, oracle, D, G):
    """Many components (the register-blocked screening): means duplicated
    exactly tie in every precision, so the lowest index must win for every
    sample, as in the oracle's first-minimum rule."""
    X, _ = synth.diag_gmm(17 + D, D, 8, 3000, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    base = synth.static_subset(X, G - 60)
    mu = np.concatenate([base, base[:60]])  # components G-60.. repeat 0..59
    gk = gpu_kmeans_step(G_, X, mu, 0, 1e-10)
    rk = oracle.kmeans_iter(X, mu, np.ones(D), 1e-10)
    assert gk["status"] == 0
    assert np.array_equal(gk["assign"], rk.assign)
    assert (gk["assign"] < G - 60).all()
    np.testing.assert_array_equal(gk["counts"], rk.counts)


# ---------------------------------------------------------------- assign()
@pytest.mark.parametrize("mode", [0, 1])
def test_assign_and_hist(G_, oracle, mode):
    X, _ = synth.diag_gmm(91, 6, 5, 5000, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    w, mu, var = _params(9, 6, 5, X)
    asg = torch.zeros(5000, dtype=torch.int32, device=DEV)
    hist = torch.zeros(5, dtype=torch.int64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = G_.workspace(5000, 6, 5, device=DEV)
    G_.gmm_assign(_t(X), mode, _t(w), _t(mu), _t(var), asg, hist, st, ws)
    ref = oracle.assign(X, w, mu, var, mode)
    assert np.array_equal(asg.cpu().numpy(), ref)
    assert np.array_equal(hist.cpu().numpy(), np.bincount(ref, minlength=5))


# ---------------------------------------------------------------- seeding
# one sample; several workgroups with ragged tiles; one and several LDS
# dimension chunks; static and random starts; Euclidean and Mahalanobis
@pytest.mark.parametrize("N,D,G,first,maha", [(1, 3, 4, 0, False), (5000, 7, 20, 0, False),
                                              (3001, 40, 16, 123, True), (700, 100, 64, 0, True),
                                              (20_000, 33, 8, 19_999, False)])
def test_seed_spread(G_, oracle, N, D, G, first, maha):
    X, _ = synth.diag_gmm(40 + D, D, 6, N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    gvar = oracle.global_stats(X)[1] if maha else None
    lam = oracle.maha_lambda(gvar, 1e-10) if maha else None
    ref_idx, _ = oracle.seed_spread(X, G, first=first, lam=lam)
    means = torch.full((G, D), float("nan"), device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = G_.workspace(N, D, G, device=DEV)
    G_.gmm_seed_means(_t(X), G_.SEED_SPREAD, means, st, ws,
                      gvar=None if gvar is None else _t(gvar, torch.float64), var_floor=1e-10,
                      first=first)
    assert st.item() == 0
    np.testing.assert_array_equal(means.cpu().numpy(), X[ref_idx])


def test_seed_subset(G_):
    X, _ = synth.diag_gmm(5, 9, 3, 1234, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    ws = G_.workspace(1234, 9, 37, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    means = torch.zeros(37, 9, device=DEV)
    G_.gmm_seed_means(_t(X), G_.SEED_SUBSET, means, st, ws)  # static: floor(g N / G)
    np.testing.assert_array_equal(means.cpu().numpy(), synth.static_subset(X, 37))
    rng = np.random.Generator(np.random.PCG64(3))
    idx = rng.choice(1234, 37, replace=False)
    G_.gmm_seed_means(_t(X), G_.SEED_SUBSET, means, st, ws, idx=_t(idx, torch.int64))
    np.testing.assert_array_equal(means.cpu().numpy(), X[idx])
    assert st.item() == 0
    idx[5] = 1234  # out of range: flagged, row kept
    before = means.cpu().numpy().copy()
    G_.gmm_seed_means(_t(X), G_.SEED_SUBSET, means, st, ws, idx=_t(idx, torch.int64))
    assert st.item() & G_.GMM_DEV_BADDESC
    np.testing.assert_array_equal(means.cpu().numpy()[5], before[5])


@pytest.mark.parametrize("mode", ["static_subset", "random_subset", "static_spread",
                                  "random_spread"])
def test_learn_seed_modes_and_loglik_stop(G_, mode):
    """The learn() driver end to end: each seed mode, then k-means and EM with
    the log-likelihood-increase stop (EM log-likelihoods never decrease)."""
    from paper_1707_09094_amd import train
    X, _ = synth.diag_gmm(3, 5, 4, 4000, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    tol = 1e-4
    model, log, _ = train.learn(_t(X), 4, seed_mode=mode, rng_seed=1, km_iter=5, em_iter=40,
                                em_tol=tol)
    assert log.status == 0
    ll = np.array(log.loglik)
    assert len(ll) >= 2 and np.all(np.isfinite(ll))
    inc = np.diff(ll)
    assert np.all(inc >= -1e-9 * np.abs(ll[1:]))
    if len(ll) < 40:  # stopped by the rule: only the last increase is below tol
        assert inc[-1] < tol and np.all(inc[:-1] >= tol)
    assert abs(float(model.hefts.sum()) - 1.0) < 1e-5


# ---------------------------------------------------------------- log_p(X, g)
# N = 1; several tiles with a ragged tail; D = 1, one LDS dimension chunk with
# a ragged tail (33), several chunks (100, 300); first and last Gaussian
@pytest.mark.parametrize("N,D,G,g", [(1, 1, 1, 0), (257, 5, 3, 2), (3001, 33, 4, 3),
                                     (10_000, 100, 7, 0), (2000, 300, 2, 1)])
def test_log_p_gaussian(G_, oracle, N, D, G, g):
    X, _ = synth.diag_gmm(300 + D, D, max(G, 2), N, "normal", 0.0, 4.0, "loguniform", 0.1,
                          10.0)
    _, mu, var = _params(7 + D, D, G, X if N >= G else None)
    per = torch.full((N,), float("nan"), dtype=torch.float32, device=DEV)
    mo = torch.zeros(1, dtype=torch.float64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = G_.workspace(N, D, G, device=DEV)
    G_.gmm_log_p_gaussian(_t(X), g, _t(mu), _t(var), mo, per, st, ws)
    ref = oracle.log_p_g(X, mu, var, g)
    assert st.item() == 0
    got = per.cpu().numpy().astype(np.float64)
    # FP32 output of an FP64 value: half an ulp plus FP64 reordering
    assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-12), g
    m = ref.mean()
    assert abs(mo.item() - m) <= 1e-12 * abs(m) + 1e-12
    # mean alone, and a row stride above D: the same mean to rounding
    Xw = torch.zeros(N, D + 3, device=DEV)
    Xw[:, :D] = _t(X)
    mo2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    G_.gmm_log_p_gaussian(Xw[:, :D], g, _t(mu), _t(var), mo2, None, st, ws)
    assert abs(mo2.item() - m) <= 1e-12 * abs(m) + 1e-12
    with pytest.raises(G_.GmmError):
        G_.gmm_log_p_gaussian(_t(X), G, _t(mu), _t(var), mo, per, st, ws)  # g out of range


def test_log_p_gaussian_nonpositive_variance_sets_status(G_):
    X = torch.zeros(100, 3, device=DEV)
    mu = torch.zeros(2, 3, device=DEV)
    var = torch.ones(2, 3, device=DEV)
    var[1, 2] = 0.0
    mo = torch.zeros(1, dtype=torch.float64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = G_.workspace(100, 3, 2, device=DEV)
    G_.gmm_log_p_gaussian(X, 0, mu, var, mo, None, st, ws)
    assert st.item() == 0
    G_.gmm_log_p_gaussian(X, 1, mu, var, mo, None, st, ws)
    assert st.item() & G_.GMM_DEV_NONFINITE


# ---------------------------------------------------------------- errors
def test_binding_raises_on_invalid(G_):
    X = torch.zeros(10, 3, device=DEV)
    ws = G_.workspace(10, 3, 2, device=DEV)
    h = torch.zeros(2, device=DEV)
    m = torch.zeros(2, 3, device=DEV)
    c = torch.ones(2, 3, device=DEV)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(G_.GmmError):
        G_.gmm_em_iter(X, 0, h, m, c, -1.0, 0, ll, None, st, ws)  # negative floor
    with pytest.raises(G_.GmmError):
        G_.gmm_em_iter(X, 0, h, m, c, 0.0, 0, ll, None, st, ws[:64])  # workspace too small


# ---------------------------------------------------------------- full covariance
# D <= 32 and D <= 64 screen on the matrix cores (one and two k-steps), D > 64
# on the vector ALUs; N = 70 leaves a tile of 6 samples
@pytest.mark.parametrize("N,D,G", [(5000, 4, 3), (3000, 32, 8), (257, 7, 2), (70, 33, 5),
                                   (4000, 48, 6), (3001, 64, 17), (1500, 80, 3)])
def test_em_step_full(G_, oracle, N, D, G):
    X, truth = synth.full_gmm(500 + D, D, G, N)
    rng = np.random.Generator(np.random.PCG64(D))
    w = rng.dirichlet(np.ones(G)).astype(np.float32)
    mu = X[rng.choice(N, G, replace=False)].astype(np.float32)
    S = truth.covs.astype(np.float32)
    S = (S + np.transpose(S, (0, 2, 1))) / 2
    gpu = gpu_em_step(G_, X, w, mu, S, 1e-6, full=True)
    assert gpu["status"] == 0
    ref = oracle.em_iter(X, w, mu, S, 1e-6, full=True)
    check_em(gpu, ref, N, full=True)


def test_full_not_pd_sets_status(G_):
    X = np.zeros((20, 2), np.float32)
    S = np.array([[[1.0, 2.0], [2.0, 1.0]]], np.float32)
    gpu = gpu_em_step(G_, X, np.ones(1, np.float32), np.zeros((1, 2), np.float32), S, 1e-6,
                      full=True)
    assert gpu["status"] & 2
