"""Benchmark: diagonal GMM training at D=100, G=100, N=1e6 on one GPU.

One step = one full training pass over the resident synthetic data set:
global per-dimension statistics, 10 Mahalanobis k-means iterations and 10 EM
iterations (the paper's speed-up experiment, Sec. 5.1), all through the C ABI.
The headline value is EM iterations per second of the EM phase inside the
timed steps; the GPU's other arithmetic form is timed separately on the same
k-means output, and both forms' final log-likelihoods are compared.

Prints ONE JSON line (rank 0).  Extra keys: the roofline of the dominant
kernel (the fused E/M pass) timed live with HIP events recorded by the library
on the launch stream, and the FP64 CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D_, G_, N_ = 100, 100, 1_000_000
KM_ITERS, EM_ITERS = 10, 10
VAR_FLOOR = 1e-10
FP32_VALU_PEAK_TF = 157.3     # MI355X published FP32 vector peak
BF16_MFMA_PEAK_TF = 2500.0    # MI355X published dense BF16 matrix peak
FP64_PEAK_TF = 78.6           # MI355X published FP64 peak (matrix and vector alike)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--N", type=int, default=N_)
    p.add_argument("--prec", choices=["fp32", "bf16x3"], default="bf16x3",
                   help="arithmetic form of the timed EM phase (headline)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--workload", choices=["d100", "d64g512", "full32"], default="d100",
                   help="d100: the headline workload (default); d64g512: D=64, G=512, N=8e6; "
                        "full32: full covariances D=32, G=64, N=2e6")
    p.add_argument("--no-batched", action="store_true",
                   help="skip the many-model (2000 models, D=40) measurement")
    p.add_argument("--profile-only", action="store_true",
                   help="run warmup + timed steps only (for rocprofv3)")
    return p.parse_args()


def em_flops(N, D, G):
    # algorithmic count per EM iteration: E-step 4NGD + M-step 4NGD
    return 8.0 * N * G * D


def measured_traffic(kernel_src, key_sha="source_sha16", key_f="fetch_bytes", key_w="write_bytes"):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_em_diag_D100_G100_N1e6.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, kernel_src), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    if rec.get(key_sha) != sha:
        return None
    return rec[key_f] + rec[key_w]


def batched_workload(gmm, synth, torch, dev, km_iters=KM_ITERS, em_iters=EM_ITERS):
    """The many-model workload: 2000 diagonal models, D=40, G_k uniform over
    {8,16,32,64}, N_k log-uniform in [500, 2e5], each drawn from the D=100
    recipe at D=40 (weights Dirichlet(1), means N(0,4), variances
    log-U[0.1,10]).  The samples are drawn on the device (torch Philox, seeded)
    because the 10.7 GB data set is too large to draw on the host in a
    benchmark run.  One step = global stats + 10 Mahalanobis k-means + 10 EM
    iterations (BF16X3) of every model, through the batched entry points."""
    import numpy as np
    Ns, Gs = synth.config5_shapes()
    D = 40
    gen = torch.Generator(device=dev)
    gen.manual_seed(17079094)
    Xs, inits = [], []
    for N, G in zip(Ns.tolist(), Gs.tolist()):
        e = -torch.log(torch.rand(G, device=dev, generator=gen))
        w = e / e.sum()
        mu = 2.0 * torch.randn(G, D, device=dev, generator=gen)
        var = torch.exp(np.log(0.1) + (np.log(10.0) - np.log(0.1)) *
                        torch.rand(G, D, device=dev, generator=gen))
        lab = torch.multinomial(w, N, replacement=True, generator=gen)
        X = (mu[lab] + var[lab].sqrt() * torch.randn(N, D, device=dev, generator=gen)).contiguous()
        Xs.append(X)
        inits.append(X[(torch.arange(G, device=dev) * N) // G].clone())
    b = gmm.ModelBatch(Xs, Gs.tolist(), device=dev)
    ws = b.workspace(1024)
    chunk = gmm.gmm_batched_autotune(b, gmm.PREC_BF16X3, ws)
    sum_ng = float(np.sum(Ns.astype(np.float64) * Gs))

    def step():
        for m, mu0 in enumerate(inits):
            b.means[m].copy_(mu0)
        gmm.gmm_global_stats_batched(b, b.gmean, b.gvar)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(km_iters):
            gmm.gmm_kmeans_iter_batched(b, gmm.DIST_MAHA, VAR_FLOOR, chunk, ws)
        e1.record()
        for _ in range(em_iters):
            gmm.gmm_em_iter_batched(b, VAR_FLOOR, gmm.PREC_BF16X3, chunk, ws)
        e2.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / km_iters, e1.elapsed_time(e2) / em_iters

    step()  # warm-up
    km_ms, em_ms = step()
    status = int((b.dev_status != 0).sum().item())
    return {"models": len(Ns), "D": D, "sum_N": int(Ns.sum()), "sum_NG": sum_ng, "chunk": chunk,
            "km_iter_ms": round(km_ms, 3), "em_iter_ms": round(em_ms, 3),
            "em_sample_components_per_s": round(sum_ng / (em_ms / 1e3), 1),
            "km_sample_components_per_s": round(sum_ng / (km_ms / 1e3), 1),
            "models_with_status": status,
            "data": "synthetic, drawn on the device (torch Philox) from the stated recipe"}


def other_workload(args, gmm, synth, torch, np):
    """D=64/G=512/N=8e6 (diagonal) or full covariances D=32/G=64/N=2e6: one step =
    global stats + 10 Mahalanobis k-means + 10 EM iterations, timed with HIP events;
    the same JSON layout as the headline line."""
    from paper_1707_09094_amd.train import Model, Trainer
    dev = "cuda:0"
    full = args.workload == "full32"
    if full:
        X, _ = synth.config4(N=args.N if args.N != N_ else 2_000_000)
        G = 64
    else:
        X, _ = synth.config3(N=args.N if args.N != N_ else 8_000_000)
        G = 512
    N, D = X.shape
    Xd = torch.as_tensor(X).to(dev)
    seed_means = torch.as_tensor(synth.static_subset(X, G)).to(dev)
    head = gmm.PREC_BF16X3 if args.prec == "bf16x3" else gmm.PREC_FP32
    cov = gmm.COV_FULL if full else gmm.COV_DIAG
    tr = Trainer(Xd, G, cov, head)
    tr_km = Trainer(Xd, G, gmm.COV_DIAG, head) if full else tr

    def fit(em_prec):
        means = seed_means.clone()
        dcovs = torch.ones(G, D, device=dev)
        hefts = torch.full((G,), 1.0 / G, device=dev)
        tr_km.global_stats()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(KM_ITERS):
            tr_km.kmeans_iter(means, dcovs, hefts, gmm.DIST_MAHA, VAR_FLOOR, prec=head)
        e1.record()
        covs = torch.diag_embed(dcovs).contiguous() if full else dcovs
        model = Model(hefts, means, covs, cov)
        for _ in range(EM_ITERS):
            tr.em_iter(model, VAR_FLOOR, prec=em_prec)
        e2.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), e1.elapsed_time(e2), float(tr.scal[1].item())

    for _ in range(args.warmup):
        fit(head)
    kms, ems, lls = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b, ll = fit(head)
        kms.append(a)
        ems.append(b)
        lls.append(ll)
    wall = time.perf_counter() - t0
    _, em_fp32, ll32 = fit(gmm.PREC_FP32)
    em_ms = float(np.mean(ems)) / EM_ITERS
    # both kernels compute in FP64 (E-step on the matrix cores; map step on the
    # matrix cores for full covariances, on the FP64 vector ALUs for diagonal
    # ones), and the two FP64 peaks are equal
    if full:
        F = float(N) * G * (2 * D * (D + 1) + 4 * D)
        work = "full-covariance GMM D=32 G=64 N=2e6 (Sigma = A A^T + 0.1 I, A_de ~ N(0, 0.3))"
        kernel = ("k_estep_full: exact FP64 log-densities Z = X W^T - W mu and the map step as "
                  "an FP64 rank update, both on the matrix cores")
    else:
        F = em_flops(N, D, G)
        work = "diag GMM D=64 G=512 N=8e6 (means N(0,1), variances log-U[0.05,5])"
        kernel = ("k_estep_diag (more than 128 components): exact FP64 log-densities of the "
                  "expanded form on the matrix cores, FP64 map step on the vector ALUs")
    achieved = F / (em_ms / 1e3) / 1e12
    out = {
        "metric": "EM iter/s", "value": round(1e3 / em_ms, 3), "unit": "EM iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(float(np.mean(np.array(kms) + np.array(ems))), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": work + "; step = global stats + 10 Mahalanobis k-means + 10 EM",
                   "N": N, "D": D, "G": G, "em_prec": args.prec,
                   "kernel": kernel},
        "em_iter_ms": round(em_ms, 3), "km_iter_ms": round(float(np.mean(kms)) / KM_ITERS, 3),
        "em_iter_ms_fp32_form": round(em_fp32 / EM_ITERS, 3),
        "final_loglik": lls[-1], "final_loglik_fp32_form": ll32, "wall_s": round(wall, 3),
        "dev_status": int(tr.status.item()),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TF,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TF, 4),
                     "traffic": None},
    }
    print(json.dumps(out))


def cpu_baseline(X, hefts, means, dcovs):
    """One EM iteration of the FP64 oracle over the full data set on the host."""
    from oracle import oracle
    ncpu = os.cpu_count() or 1
    threads = min(16, ncpu)
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    oracle.em_iter(X, hefts, means, dcovs, VAR_FLOOR)
    dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 5), "unit": "EM iter/s", "cores": threads, "kind": "oracle",
            "sample": f"1 EM iteration on the full {X.shape[0]}x{X.shape[1]} data set, G={len(hefts)}"
                      f" ({dt:.2f} s, FP64, OpenMP {threads} threads)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the path runs on one GPU (one rank); --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1707_09094_amd import gmm, synth
    from paper_1707_09094_amd.train import Model, Trainer

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.workload != "d100":
        other_workload(args, gmm, synth, torch, np)
        return
    X, _ = synth.config2(N=args.N)
    N, D = X.shape
    G = G_
    Xd = torch.as_tensor(X).to(dev)
    seed_means = torch.as_tensor(synth.static_subset(X, G)).to(dev)
    head = gmm.PREC_BF16X3 if args.prec == "bf16x3" else gmm.PREC_FP32
    tr = Trainer(Xd, G, gmm.COV_DIAG, head)
    torch.cuda.synchronize()

    last_handoff = [None]

    def fit(em_prec, record=False, keep_handoff=False):
        means = seed_means.clone()
        dcovs = torch.ones(G, D, device=dev)
        hefts = torch.full((G,), 1.0 / G, device=dev)
        tr.global_stats()
        for _ in range(KM_ITERS):
            tr.kmeans_iter(means, dcovs, hefts, gmm.DIST_MAHA, VAR_FLOOR, prec=head)
        ev_km = torch.cuda.Event(enable_timing=True)
        ev_km.record()
        if keep_handoff:
            last_handoff[0] = (hefts.cpu().numpy(), means.cpu().numpy(), dcovs.cpu().numpy())
        model = Model(hefts, means, dcovs, gmm.COV_DIAG)
        lls = []
        for _ in range(EM_ITERS):
            tr.em_iter(model, VAR_FLOOR, prec=em_prec)
            if record:
                lls.append(tr.scal[1].clone())
        ev_em = torch.cuda.Event(enable_timing=True)
        ev_em.record()
        return ev_km, ev_em, model, lls

    for _ in range(args.warmup):
        fit(head)
    torch.cuda.synchronize()

    gmm.gmm_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    marks = []
    for _ in range(args.steps):
        start = torch.cuda.Event(enable_timing=True)
        start.record()
        ev_km, ev_em, model, _ = fit(head)
        marks.append((start, ev_km, ev_em))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    em_ms_tot, em_launches = gmm.gmm_profile_read(gmm.PROF_EM)
    km_ms_tot, km_launches = gmm.gmm_profile_read(gmm.PROF_KM_ASSIGN)
    gmm.gmm_profile_enable(False)
    step_ms = [s.elapsed_time(e) for s, _, e in marks]
    em_phase_ms = [k.elapsed_time(e) for _, k, e in marks]
    if args.profile_only:
        # calibration for HBM byte counters: one plain device copy of 256 MiB
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_only": True, "ms_per_step": float(np.mean(step_ms)),
                          "copy_bytes_each_way": src.numel() * 4}))
        return

    em_iter_s = EM_ITERS * len(em_phase_ms) / (sum(em_phase_ms) / 1e3)
    ms_per_step = float(np.mean(step_ms))
    status = int(tr.status.item())

    # the two arithmetic forms from the same k-means output
    forms = {}
    handoff = None
    for name, pr in (("fp32", gmm.PREC_FP32), ("bf16x3", gmm.PREC_BF16X3)):
        _, _, m, lls = fit(pr, record=True, keep_handoff=handoff is None)
        if handoff is None:
            handoff = last_handoff[0]
        torch.cuda.synchronize()
        ev_a = torch.cuda.Event(enable_timing=True)
        ev_b = torch.cuda.Event(enable_timing=True)
        # time EM_ITERS iterations of this form from a copy of the hand-off
        mm = Model(m.hefts.clone(), m.means.clone(), m.covs.clone(), gmm.COV_DIAG)
        ev_a.record()
        for _ in range(EM_ITERS):
            tr.em_iter(mm, VAR_FLOOR, prec=pr)
        ev_b.record()
        torch.cuda.synchronize()
        forms[name] = {"em_iter_s": EM_ITERS / (ev_a.elapsed_time(ev_b) / 1e3),
                       "final_loglik": float(lls[-1].item()),
                       "em_recomputed": int(tr.i64[1].item())}
    dl = abs(forms["bf16x3"]["final_loglik"] - forms["fp32"]["final_loglik"]) / abs(
        forms["fp32"]["final_loglik"])

    F = em_flops(N, D, G)
    em_kernel_ms = em_ms_tot / max(em_launches, 1)
    achieved_tf = F / (em_kernel_ms / 1e3) / 1e12
    if head == gmm.PREC_BF16X3:
        # E-step contraction on the BF16 matrix cores (algorithmic 4NGD at the
        # dense BF16 peak) + M-step map on FP32 vector ALUs (4NGD at the FP32
        # peak): the shortest possible time of the algorithmic work.
        t_min = 4.0 * N * G * D / (BF16_MFMA_PEAK_TF * 1e12) + 4.0 * N * G * D / (FP32_VALU_PEAK_TF * 1e12)
        peak = F / t_min / 1e12
        bound = "mfma"
    else:
        peak = FP32_VALU_PEAK_TF
        bound = "alu"
    traffic = measured_traffic("paper_1707_09094_amd/csrc/gmm_em_fast.hip") if N == N_ else None
    roof = {"bound": bound, "achieved": round(achieved_tf, 3), "peak": round(peak, 2),
            "unit": "TFLOP/s", "frac": round(achieved_tf / peak, 4),
            "traffic": None if traffic is None else round(traffic),
            "kernel": "k_em2 (fused E-step + M-step map, sample-major BF16x3 MFMA)"
                      if head == gmm.PREC_BF16X3 else "k_em_fast (fused E-step + M-step map, FP32)",
            "kernel_ms": round(em_kernel_ms, 4), "launches": em_launches}

    out = {
        "metric": "EM iter/s & GFLOP/s at D=100 N_G=100 N=1e6; BF16-MFMA vs FP32 at equal loglik",
        "value": round(em_iter_s, 3),
        "unit": "EM iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f32" if head == gmm.PREC_BF16X3 else "f32",
        "data": "synthetic",
        "config": {"workload": "diag GMM D=100 G=100 N=1e6 FP32 samples (means N(0,4), variances "
                               "log-U[0.1,10], Dirichlet(1) weights); step = global stats + 10 "
                               "Mahalanobis k-means + 10 EM iterations",
                   "N": N, "D": D, "G": G, "em_prec": args.prec},
        "gflops": round(F * em_iter_s / 1e9, 1),
        "em_iter_s_fp32": round(forms["fp32"]["em_iter_s"], 3),
        "em_iter_s_bf16x3": round(forms["bf16x3"]["em_iter_s"], 3),
        "bf16x3_speedup": round(forms["bf16x3"]["em_iter_s"] / forms["fp32"]["em_iter_s"], 3),
        "final_loglik_fp32": forms["fp32"]["final_loglik"],
        "final_loglik_rel_delta": dl,
        "em_recomputed_bf16x3": forms["bf16x3"]["em_recomputed"],
        "km_assign_ms": round(km_ms_tot / max(km_launches, 1), 4),
        "wall_s": round(wall, 3),
        "dev_status": status,
        "roofline": roof,
    }
    if not args.no_batched:
        del Xd, tr
        torch.cuda.empty_cache()
        out["batched"] = batched_workload(gmm, synth, torch, dev)
    if not args.no_cpu_baseline:
        # the CPU oracle runs one EM iteration from the GPU's k-means hand-off
        out["cpu_baseline"] = cpu_baseline(X, *handoff)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
