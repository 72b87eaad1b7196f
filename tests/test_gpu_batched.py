"""GPU parity of the many-model entry points (gmm_*_batched): every model of a
batch against the FP64 oracle on its own data and parameters, the batched
result against the single-model call, chunk invariance, the dead-cluster rule
inside a batch, and capture of a batched iteration sequence into a graph that
is replayed several times."""
import numpy as np
import pytest

from paper_1707_09094_amd import synth
from tests.parity import check_em, rel_means, rel_vars, rel_weights

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (N, G) per model: N below, at and just above the item size, G = 1 and the
# maximum 128, models smaller than their G
SHAPES_D40 = [(1, 1), (31, 2), (33, 8), (500, 16), (1024, 32), (1025, 64), (5000, 64),
              (20_000, 128), (7, 5), (2047, 3), (4096, 8), (12_345, 16)]
SHAPES_D100 = [(3000, 100), (100, 10), (4097, 1), (1, 3)]
# at most 64 components: the matrix-core passes keep each round's rows and the
# FP64 constants in LDS (models with G <= 16 accumulate their map step per wave)
SHAPES_D40_S = [s for s in SHAPES_D40 if s[1] <= 64]
SHAPES_D5 = [(10_000, 4), (999, 7), (2, 2)]


@pytest.fixture(scope="module")
def G_():
    from paper_1707_09094_amd import gmm
    gmm.library()
    return gmm


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def _data(seed, D, shapes):
    Xs, params = [], []
    for k, (N, G) in enumerate(shapes):
        X, _ = synth.diag_gmm(seed + k, D, max(G, 2), N, "normal", 0.0, 4.0, "loguniform",
                              0.1, 10.0)
        rng = np.random.Generator(np.random.PCG64(seed * 31 + k))
        w, mu, var = synth.random_params(rng, D, G)
        if N >= G:
            mu = X[rng.choice(N, G, replace=False)].astype(np.float32)
        Xs.append(X)
        params.append((w.astype(np.float32), mu.astype(np.float32), var.astype(np.float32)))
    return Xs, params


def _batch(G_, Xs, params):
    b = G_.ModelBatch([_t(X) for X in Xs], [len(p[0]) for p in params], device=DEV)
    for m, (w, mu, var) in enumerate(params):
        b.set_params(m, _t(w), _t(mu), _t(var))
    return b


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("D,shapes,chunk", [(40, SHAPES_D40, 1024), (100, SHAPES_D100, 2048),
                                            (5, SHAPES_D5, 32), (40, SHAPES_D40_S, 1024)])
def test_em_batched_vs_oracle(G_, oracle, D, shapes, chunk, prec):
    Xs, params = _data(500 + D, D, shapes)
    b = _batch(G_, Xs, params)
    ws = b.workspace(chunk)
    G_.gmm_em_iter_batched(b, 1e-10, prec, chunk, ws)
    torch.cuda.synchronize()
    assert not _np(b.dev_status).any()
    for m, (X, (w, mu, var)) in enumerate(zip(Xs, params)):
        ref = oracle.em_iter(X, w, mu, var, 1e-10)
        gpu = dict(hefts=_np(b.hefts[m]), means=_np(b.means[m]), covs=_np(b.covs[m]),
                   loglik=float(b.loglik[m].item()))
        check_em(gpu, ref, len(X))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_loglik_batched_vs_oracle(G_, oracle, prec):
    Xs, params = _data(71, 40, SHAPES_D40)
    b = _batch(G_, Xs, params)
    ws = b.workspace(1024)
    G_.gmm_loglik_batched(b, prec, 1024, ws)
    torch.cuda.synchronize()
    assert not _np(b.dev_status).any()
    for m, (X, (w, mu, var)) in enumerate(zip(Xs, params)):
        ref = oracle.loglik(X, w, mu, var)
        assert abs(b.loglik[m].item() - ref) <= 1e-6 * abs(ref), m
        # parameters untouched
        np.testing.assert_array_equal(_np(b.means[m]), mu)
        np.testing.assert_array_equal(_np(b.covs[m]), var)


def test_em_batched_matches_single_model_call(G_):
    """Same arithmetic as gmm_em_iter: only the partial-sum cut differs."""
    Xs, params = _data(93, 40, SHAPES_D40[:8])
    b = _batch(G_, Xs, params)
    ws = b.workspace(1024)
    G_.gmm_em_iter_batched(b, 1e-10, 1, 1024, ws)
    torch.cuda.synchronize()
    for m, (X, (w, mu, var)) in enumerate(zip(Xs, params)):
        N, D = X.shape
        G = len(w)
        h, mm, c = _t(w), _t(mu), _t(var)
        ll = torch.zeros(1, dtype=torch.float64, device=DEV)
        st = torch.zeros(1, dtype=torch.int32, device=DEV)
        G_.gmm_em_iter(_t(X), G_.COV_DIAG, h, mm, c, 1e-10, 1, ll, None, st,
                       G_.workspace(N, D, G, G_.COV_DIAG, 1, DEV))
        torch.cuda.synchronize()
        np.testing.assert_allclose(_np(b.hefts[m]), _np(h), rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(_np(b.means[m]), _np(mm), rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(_np(b.covs[m]), _np(c), rtol=1e-5, atol=1e-7)
        assert abs(b.loglik[m].item() - ll.item()) <= 1e-9 * abs(ll.item())


def test_em_batched_chunk_invariance_and_determinism(G_):
    Xs, params = _data(17, 40, SHAPES_D40)
    outs = []
    for chunk in (1024, 4096, 4096):
        b = _batch(G_, Xs, params)
        G_.gmm_em_iter_batched(b, 1e-10, 0, chunk, b.workspace(chunk))
        torch.cuda.synchronize()
        outs.append((_np(b.hefts_flat), _np(b.means_flat), _np(b.covs_flat), _np(b.loglik)))
    for a, c in zip(outs[1], outs[2]):  # same chunk: bitwise
        np.testing.assert_array_equal(a, c)
    (h1, m1, c1, l1), (h4, m4, c4, l4) = outs[0], outs[1]
    N = sum(len(X) for X in Xs)
    assert rel_weights(h4, h1, N).max() <= 1e-5
    assert rel_means(m4, m1, c1).max() <= 1e-5
    assert rel_vars(c4, c1).max() <= 1e-5
    np.testing.assert_allclose(l4, l1, rtol=1e-9)


def _km_check(oracle, X, mu, gv, got, k):
    lam = oracle.maha_lambda(gv, 1e-10) if gv is not None else np.ones(X.shape[1])
    rk = oracle.kmeans_iter(X, mu, lam, 1e-10)
    ok = rk.gap >= 1e-6
    assign, counts, means, dcovs, hefts, inertia = got
    assert np.array_equal(assign[ok], rk.assign[ok]), k
    assert abs(inertia - rk.inertia) <= 1e-9 * abs(rk.inertia) + 1e-12, k
    if ok.all():
        np.testing.assert_array_equal(counts, rk.counts)
        live = rk.counts > 0
        assert rel_means(means[live], rk.means[live], rk.dcovs[live]).max(initial=0) <= 1e-5
        assert rel_vars(dcovs[live], rk.dcovs[live]).max(initial=0) <= 1e-5
        assert rel_weights(hefts, rk.hefts, len(X)).max() <= 1e-6
        np.testing.assert_array_equal(means[~live], rk.means[~live].astype(np.float32))
        np.testing.assert_array_equal(dcovs[~live], rk.dcovs[~live].astype(np.float32))


@pytest.mark.parametrize("maha", [True, False], ids=["maha", "eucl"])
@pytest.mark.parametrize("D,shapes,chunk", [(40, SHAPES_D40, 1024), (5, SHAPES_D5, 32)],
                         ids=["d40", "d5-313items"])
def test_kmeans_batched_vs_oracle(G_, oracle, maha, D, shapes, chunk):
    # d5-313items: 10000 samples in items of 32, so the reduce step combines
    # more than 256 partials of one model (two passes of its weight table)
    Xs, _ = _data(211, D, shapes)
    means = []
    for X, (N, G) in zip(Xs, shapes):
        # more means than samples: the surplus are dead and get resurrected
        means.append(synth.static_subset(X, G) if N >= G else np.concatenate(
            [X, np.full((G - N, X.shape[1]), 100.0, np.float32)]))
    b = G_.ModelBatch([_t(X) for X in Xs], [G for _, G in shapes], device=DEV)
    for m, mu in enumerate(means):
        b.means[m].copy_(_t(mu))
    if maha:
        G_.gmm_global_stats_batched(b, b.gmean, b.gvar)
    ws = b.workspace(chunk)
    G_.gmm_kmeans_iter_batched(b, 1 if maha else 0, 1e-10, chunk, ws)
    torch.cuda.synchronize()
    assert not _np(b.dev_status).any()
    for m, (X, mu) in enumerate(zip(Xs, means)):
        gv = oracle.global_stats(X)[1] if maha else None
        if maha:
            np.testing.assert_allclose(_np(b.gvar[m]), gv, rtol=1e-10, atol=1e-300)
            np.testing.assert_allclose(_np(b.gmean[m]), oracle.global_stats(X)[0], rtol=1e-12,
                                       atol=1e-12)
        got = (_np(b.assign[m]), _np(b.counts[m]), _np(b.means[m]), _np(b.covs[m]),
               _np(b.hefts[m]), float(b.inertia[m].item()))
        _km_check(oracle, X, mu, gv, got, m)


def test_kmeans_batched_resurrection_golden(G_):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "resurrection_1d.json")) as f:
        gd = json.load(f)
    X = np.array(gd["X"], np.float32)[:, None]
    mu = np.array(gd["means_in"], np.float32)[:, None]
    # the golden model twice, with an unrelated model between them
    Xo, _ = synth.diag_gmm(5, 1, 3, 3000, "normal", 0.0, 4.0, "loguniform", 0.1, 10.0)
    b = G_.ModelBatch([_t(X), _t(Xo), _t(X)], [len(mu), 3, len(mu)], device=DEV)
    b.means[0].copy_(_t(mu))
    b.means[1].copy_(_t(synth.static_subset(Xo, 3)))
    b.means[2].copy_(_t(mu))
    G_.gmm_kmeans_iter_batched(b, 0, gd["var_floor"], 32, b.workspace(32))
    torch.cuda.synchronize()
    for m in (0, 2):
        assert list(_np(b.assign[m])) == gd["assign"]
        assert list(_np(b.counts[m])) == gd["counts"]
        np.testing.assert_allclose(_np(b.means[m])[:, 0], gd["means_out"], rtol=1e-7)
        np.testing.assert_allclose(_np(b.covs[m])[:, 0], gd["dcovs_out"], rtol=1e-6)
        np.testing.assert_allclose(_np(b.hefts[m]), gd["hefts_out"], rtol=1e-7)
        assert abs(b.inertia[m].item() - gd["inertia"]) <= 1e-9 * gd["inertia"]


def test_batched_realistic_subset(G_, oracle):
    """Twelve models of the many-model workload (D=40, G in {8,16,32,64},
    N log-uniform in [500, 2e5]): k-means hand-off, then EM in BF16x3."""
    Ns, Gs = synth.config5_shapes()
    pick = list(range(12))
    Xs = [synth.config5_model(k, Ns[k], Gs[k])[0] for k in pick]
    b = G_.ModelBatch([_t(X) for X in Xs], [int(Gs[k]) for k in pick], device=DEV)
    for m, X in enumerate(Xs):
        b.means[m].copy_(_t(synth.static_subset(X, int(Gs[pick[m]]))))
    G_.gmm_global_stats_batched(b, b.gmean, b.gvar)
    ws = b.workspace(1024)
    chunk = G_.gmm_batched_autotune(b, 1, ws)
    assert chunk in (1024, 2048, 4096, 8192, 16384)
    mu0 = [_np(b.means[m]).copy() for m in range(len(pick))]
    G_.gmm_kmeans_iter_batched(b, 1, 1e-10, chunk, ws)
    torch.cuda.synchronize()
    for m, X in enumerate(Xs):
        got = (_np(b.assign[m]), _np(b.counts[m]), _np(b.means[m]), _np(b.covs[m]),
               _np(b.hefts[m]), float(b.inertia[m].item()))
        _km_check(oracle, X, mu0[m], oracle.global_stats(X)[1], got, m)
    p0 = [(_np(b.hefts[m]).copy(), _np(b.means[m]).copy(), _np(b.covs[m]).copy())
          for m in range(len(pick))]
    G_.gmm_em_iter_batched(b, 1e-10, 1, chunk, ws)
    torch.cuda.synchronize()
    assert not _np(b.dev_status).any()
    for m, X in enumerate(Xs):
        ref = oracle.em_iter(X, *p0[m], 1e-10)
        gpu = dict(hefts=_np(b.hefts[m]), means=_np(b.means[m]), covs=_np(b.covs[m]),
                   loglik=float(b.loglik[m].item()))
        check_em(gpu, ref, len(X))


@pytest.mark.parametrize("shapes", [SHAPES_D40[4:10], SHAPES_D40_S[2:9]], ids=["g128", "g64"])
def test_batched_graph_capture_replay(G_, shapes):
    """One k-means iteration and two EM iterations captured into a graph;
    each replay (with eager work and synchronisation between replays) must
    reproduce the eager sequence bit for bit."""
    Xs, _ = _data(333, 40, shapes)
    Gs = [G for _, G in shapes]
    b = G_.ModelBatch([_t(X) for X in Xs], Gs, device=DEV)
    init = [_t(synth.static_subset(X, G) if len(X) >= G else np.resize(X, (G, 40)))
            for X, G in zip(Xs, Gs)]
    ws = b.workspace(1024)

    def reset():
        for m, mu in enumerate(init):
            b.means[m].copy_(mu)

    def seq():
        G_.gmm_kmeans_iter_batched(b, 1, 1e-10, 1024, ws)
        G_.gmm_em_iter_batched(b, 1e-10, 1, 1024, ws)
        G_.gmm_em_iter_batched(b, 1e-10, 1, 1024, ws)

    G_.gmm_global_stats_batched(b, b.gmean, b.gvar)
    reset()
    seq()
    torch.cuda.synchronize()
    eager = [_np(t).copy() for t in (b.hefts_flat, b.means_flat, b.covs_flat, b.assign_flat,
                                     b.loglik)]
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
        got = [_np(t) for t in (b.hefts_flat, b.means_flat, b.covs_flat, b.assign_flat,
                                b.loglik)]
        for a, e in zip(got, eager):
            np.testing.assert_array_equal(a, e, err_msg=f"replay {rep}")
        _ = torch.ones(1000, device=DEV).sum().item()  # eager work between replays


def test_batched_binding_raises(G_):
    X = torch.zeros(10, 3, device=DEV)
    b = G_.ModelBatch([X], [2], device=DEV)
    ws = b.workspace(1024)
    with pytest.raises(G_.GmmError):
        G_.gmm_em_iter_batched(b, 1e-10, 0, 1000, ws)  # chunk not a multiple of 32
    with pytest.raises(G_.GmmError):
        G_.gmm_em_iter_batched(b, -1.0, 0, 1024, ws)
    with pytest.raises(G_.GmmError):
        G_.gmm_em_iter_batched(b, 1e-10, 0, 32, ws[:64])  # workspace too small
    big = G_.ModelBatch([torch.zeros(10, 129, device=DEV)], [2], device=DEV)
    with pytest.raises(G_.GmmError):
        G_.gmm_em_iter_batched(big, 1e-10, 0, 1024, ws)  # D beyond the batched envelope


def test_autotune_cache(G_, tmp_path, monkeypatch):
    """gmm_batched_autotune keeps its choice per (arch, D, largest G, N and
    model-count buckets, form, covariance type): a repeated call launches
    nothing and returns the same work-item size; the cache file named by
    GMM_AUTOTUNE_CACHE gets one "key chunk" line per new choice and refills
    the table after a clear."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GMM_AUTOTUNE_CACHE", str(path))
    G_.gmm_autotune_cache_clear()
    assert G_.gmm_autotune_cache_size() == 0
    Xs, params = _data(97, 40, SHAPES_D40[:6])
    b = _batch(G_, Xs, params)
    ws = b.workspace(1024)
    c1 = G_.gmm_batched_autotune(b, 1, ws)
    assert c1 in (1024, 2048, 4096, 8192, 16384)
    assert G_.gmm_autotune_cache_size() == 1
    (line,) = path.read_text().splitlines()
    key, val = line.split()
    assert int(val) == c1 and "|D40|G64|" in key and key.endswith("|p1|diag")

    def launches(fn):
        G_.gmm_profile_enable(True)
        out = fn()
        torch.cuda.synchronize()
        n = G_.gmm_profile_read(G_.PROF_BATCHED)[1]
        G_.gmm_profile_enable(False)
        return out, n

    c2, n2 = launches(lambda: G_.gmm_batched_autotune(b, 1, ws))
    assert c2 == c1 and n2 == 0
    G_.gmm_autotune_cache_clear()
    c3, n3 = launches(lambda: G_.gmm_batched_autotune(b, 1, ws))
    assert c3 == c1 and n3 == 0 and G_.gmm_autotune_cache_size() == 1
    # the other arithmetic form is another key: timed, then cached
    c4, n4 = launches(lambda: G_.gmm_batched_autotune(b, 0, ws))
    assert n4 > 0 and G_.gmm_autotune_cache_size() == 2
    assert len(path.read_text().splitlines()) == 2
    G_.gmm_autotune_cache_clear()
