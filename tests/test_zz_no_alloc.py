"""gmm_em_iter_noalloc (the library's static per-GPU scratch instead of a
caller workspace) against gmm_em_iter through the C ABI: the same parameters
and log-likelihood, on two calls in a row, the second with a smaller input;
a shape whose workspace exceeds the static scratch is rejected on the host."""
import numpy as np
import pytest

from paper_1707_09094_amd import synth
from tests.parity import check_em

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def G_():
    from paper_1707_09094_amd import gmm
    gmm.library()
    return gmm


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=torch.float32)


def _run(G_, X, w, mu, var, prec, noalloc, full=False):
    N, D = X.shape
    G = len(w)
    cov = G_.COV_FULL if full else G_.COV_DIAG
    h, m, c = _t(w), _t(mu), _t(var)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    nrec = torch.zeros(1, dtype=torch.int64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    if noalloc:
        G_.gmm_em_iter_noalloc(_t(X), cov, h, m, c, 1e-10, prec, ll, nrec, st)
    else:
        ws = G_.workspace(N, D, G, cov, prec, DEV)
        G_.gmm_em_iter(_t(X), cov, h, m, c, 1e-10, prec, ll, nrec, st, ws)
    torch.cuda.synchronize()
    return dict(hefts=h.cpu().numpy(), means=m.cpu().numpy(), covs=c.cpu().numpy(),
                loglik=float(ll.item()), nrec=int(nrec.item()), status=int(st.item()))


def _case(seed, N, D, G):
    X, _ = synth.diag_gmm(seed, D, G, N, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    w = rng.dirichlet(np.ones(G)).astype(np.float32)
    mu = X[rng.choice(N, G, replace=False)].astype(np.float32)
    var = np.exp(rng.uniform(np.log(0.5), np.log(5.0), size=(G, D))).astype(np.float32)
    return X, w, mu, var


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("big,small", [((200_000, 100, 100), (3001, 40, 16)),
                                       ((20_000, 64, 200), (777, 64, 130))])
def test_noalloc_matches_workspace_call(G_, oracle, prec, big, small):
    for k, (N, D, G) in enumerate((big, small)):  # two calls in a row, the second smaller
        X, w, mu, var = _case(7000 + 13 * k + D, N, D, G)
        a = _run(G_, X, w, mu, var, prec, noalloc=True)
        b = _run(G_, X, w, mu, var, prec, noalloc=False)
        assert a["status"] == 0 and b["status"] == 0
        # the same kernels on the same inputs: identical results
        for key in ("hefts", "means", "covs"):
            assert np.array_equal(a[key], b[key]), (key, N, D, G)
        assert a["loglik"] == b["loglik"] and a["nrec"] == b["nrec"]
        if k == 1:  # and the oracle's bar, on the smaller call
            check_em(a, oracle.em_iter(X, w, mu, var, 1e-10), N)


def test_noalloc_full_covariance(G_, oracle):
    X, truth = synth.full_gmm(77, 8, 4, 5000)
    rng = np.random.Generator(np.random.PCG64(78))
    w = rng.dirichlet(np.ones(4)).astype(np.float32)
    mu = X[rng.choice(5000, 4, replace=False)].astype(np.float32)
    S = truth.covs.astype(np.float32)
    S = (S + np.transpose(S, (0, 2, 1))) / 2
    a = _run(G_, X, w, mu, S, 0, noalloc=True, full=True)
    b = _run(G_, X, w, mu, S, 0, noalloc=False, full=True)
    assert a["status"] == 0
    for key in ("hefts", "means", "covs"):
        assert np.array_equal(a[key], b[key]), key
    check_em(a, oracle.em_iter(X, w, mu, S, 1e-10, full=True), 5000, full=True)


def test_noalloc_rejects_shape_beyond_scratch(G_):
    N, D, G = 10, 64, 512  # its FP64 partials alone need more than the static scratch
    assert G_.gmm_workspace_bytes(N, D, G, G_.COV_DIAG, 0) > G_.NOALLOC_SCRATCH_BYTES
    X = torch.zeros(N, D, device=DEV)
    h = torch.full((G,), 1.0 / G, device=DEV)
    m = torch.zeros(G, D, device=DEV)
    c = torch.ones(G, D, device=DEV)
    ll = torch.zeros(1, dtype=torch.float64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(G_.GmmError) as e:
        G_.gmm_em_iter_noalloc(X, G_.COV_DIAG, h, m, c, 1e-10, 0, ll, None, st)
    assert e.value.code == G_.GMM_EINVAL
    assert torch.equal(m, torch.zeros(G, D, device=DEV))  # nothing written
