#!/usr/bin/env python3
"""Benchmark: Kernel K-means on one MI355X, n=200000, d=1024, k=64.

Workload: a 64-component Gaussian mixture in R^1024 (means N(0,1), sigma 0.5),
Gaussian kernel gamma = 1/1024, random initial labels.

Plain FP32 legs (the timed steps).  One step = one complete run of the method
on the resident input: the Gram kernel K = kappa(X X^T) (FP32 MFMA, K stored
FP32) followed by 30 reassignment steps (V in CSR form, the sweep of K,
centroid norms, fused distance/argmin/histogram) and the FP64 objective of the
final labels: the paper's protocol of exactly 30 iterations.  Two layouts of
the same FP32 K: the strip-packed upper triangle (81 GB; each stored entry
read once per step and fed to both sides of the sum; the headline) and the
dense n x ldk matrix (160 GB; the SpMM row sweep).
`value` = iterations per second = 1 / the median time of one reassignment step
on the strip-packed K over iterations 2..30 of the timed runs (HIP events on
the launching stream; the Gram excluded); the rate with the Gram included and
the dense-K figures are their own fields.

Also reported:
* time-to-converge of the plain FP32 form from the random labels (packed and
  dense K);
* the mixed + learned form: BF16 Gram with K stored BF16 (strip-packed, 40.7 GB), a feature
  network trained beforehand on 10^7 kernel-value pairs of the same mixture
  (training time reported separately), the warm start (k-means++ and Lloyd in
  feature space, kkm_warm_start), then exact refinement to convergence; the
  same BF16 form from the random labels as a control; speedups with and
  without the training time;
* the metric form against the FP64 oracle on the first 20000 points: every
  precision pair refined from the same warm labels and compared with the
  oracle converged from them (ARI, objective gap, iterations), and one step's
  error report (max distance error, objective error, label flips);
* the MNIST-shaped workload (n=60000, d=784, polynomial kernel, 30 iterations)
  and the rings workload (n=1000): Gram and sweep rooflines, time per step;
* roofline positions of the packed sweep (HBM; its algorithmic bytes are the
  packed entries plus the row-part sums it writes), the dense sweep and the
  Gram (MFMA) from HIP-event timings of those launches, and HBM traffic from
  the recorded counters;
* the matrix-free step (no stored K) beside the stored-K step at n=100000,
  k=32, d in {32, 64, 128, 256}, BF16 product;
* the FP64 oracle timed on the host on the first 20000 points (K build and
  loop apart, all host threads and one thread, median of 3), beside the GPU
  on the same points.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--rows N]
       [--no-cpu-baseline] [--no-converge] [--no-learned] [--no-batched]
       [--cpu-full] [--copy-calibration] [--gram-shapes] [--learned-only]
       [--batched-only] [--matfree-only] [--no-matfree] [--profile-kernels]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "iters/s & time-to-converge at n=200k,k=64: plain FP32 vs mixed+learned @ARI≥.99"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFS = 157.3
BF16_MFMA_PEAK_TFS = 2500.0

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of
# this benchmark at n=200000 (KiB per dispatch), with the scale factors a plain
# 1 GiB copy gave for the same counters (FETCH_SIZE read 524303 of 1048576 KiB,
# WRITE_SIZE all of them).  Valid only while the kernel's sources hash to the
# recorded value; otherwise the traffic is reported as null.
TRAFFIC = {
    "packed_sweep": {"sources": ["csrc/packed.hip", "csrc/iterate.h", "csrc/kkm_common.h"],
                     "sha256": "66383f026b912c68650d64dd811367e16957e8509415de7ca5317ccb281e23c9",
                     "n": 200000, "fetch_kib": 39621828.6, "write_kib": 4963045.4,
                     "fetch_scale": 1.9999, "write_scale": 1.0},
    "spmm_row_sweep": {"sources": ["csrc/iterate.hip", "csrc/iterate.h", "csrc/kkm_common.h"],
                       "sha256": "c637e03921a67e79aae60f3292840e1306a0850dc58cef5bad95c3d92e7f3e0d",
                       "n": 200000, "fetch_kib": 78172500.0, "write_kib": 89559.1,
                       "fetch_scale": 1.9999, "write_scale": 1.0},
    "gram_f32_mfma": {"sources": ["csrc/gram.hip", "csrc/gram_f32.hip", "csrc/gram_tile.h",
                                  "csrc/kkm_common.h"],
                      "sha256": "1920afcb061279bf55ae100518467f6a630c38de26a57e6a3ac2651cdb6d8c45",
                      "n": 200000, "fetch_kib": 150314010.6, "write_kib": 156250877.6,
                      "fetch_scale": 1.9999, "write_scale": 1.0},
}



# feature network and its training (learned warm start)
H1, H2, OUT = 512, 512, 256
TRAIN_BATCH, TRAIN_STEPS, TRAIN_LR = 64, 2442, 1e-3  # 2442 * 64^2 = 1.0e7 kernel values
WARM_RESTARTS, WARM_MAX_ITER = 8, 60
WARM_STREAMS = 4  # restarts run concurrently on this many streams


def sources_sha(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, "paper_2501_05587_amd", p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes(kernel, n):
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    if t["n"] != n or sources_sha(t["sources"]) != t["sha256"]:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def copy_calibration():
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: 5 copies of %d bytes" % (4 * n))


def ari(a, b):
    """Adjusted Rand index (Hubert and Arabie) of two labellings, host numpy."""
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    n = a.size
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    t = np.zeros((ai.max() + 1, bi.max() + 1), np.int64)
    np.add.at(t, (ai, bi), 1)

    def comb(x):
        return float((x.astype(np.float64) * (x - 1) / 2).sum())

    sij, sa, sb = comb(t), comb(t.sum(1)), comb(t.sum(0))
    exp = sa * sb / (n * (n - 1) / 2)
    mx = 0.5 * (sa + sb)
    return 1.0 if mx == exp else (sij - exp) / (mx - exp)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, rows, iters, full=False):
    """The FP64 oracle as it stands on the first `rows` points, no scaling: the
    K build (from the definition) and the loop (`iters` fixed steps) timed
    apart, each the median of 3 runs, with all the host threads OpenMP uses and
    with one thread.  With one thread the loop runs 3 steps per run (the rate
    per step is what is compared) and the K build is timed only when `full`.
    Returns (record, K)."""
    import numpy as np

    import oracle
    X, _ = w.points(rows=rows)
    l0 = w.labels0(rows=rows)
    nthr = oracle.threads()

    def timed(fn, reps=3):
        ts, out = [], None
        for _ in range(reps):
            t = time.perf_counter()
            out = fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), out

    kb, K = timed(lambda: oracle.kernel_matrix(X, w.kernel, w.gamma, w.coef0, w.degree))
    loop, _ = timed(lambda: oracle.fit(K, w.k, l0, iters, check_convergence=False))
    it1 = iters if full else 3
    rec1 = {}
    oracle.set_threads(1)
    try:
        loop1, _ = timed(lambda: oracle.fit(K, w.k, l0, it1, check_convergence=False))
        rec1["loop_ms_per_iter"] = loop1 / it1 * 1e3
        rec1["loop_iters_per_run"] = it1
        if full:
            kb1, _ = timed(lambda: oracle.kernel_matrix(X, w.kernel, w.gamma, w.coef0, w.degree))
            rec1["k_build_s"] = kb1
    finally:
        oracle.set_threads(nthr)
    rec = {"value": iters / loop, "unit": "iters/s", "cores": nthr, "kind": "oracle",
           "sample": "first %d of the %d points, %d fixed iterations (no scaling): K build %.2f s, "
                     "loop %.3f s per iteration, medians of 3, %d threads" % (
                         rows, w.n, iters, kb, loop / iters, nthr),
           "rows": rows, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
           "all_threads": {"threads": nthr, "k_build_s": kb, "loop_ms_per_iter": loop / iters * 1e3},
           "one_thread": rec1}
    log("oracle on %d points: K %.2f s, %.2f ms per iteration (%d threads), %.1f ms per iteration "
        "(1 thread)" % (rows, kb, loop / iters * 1e3, nthr, rec1["loop_ms_per_iter"]))
    return rec, K


def rowpart_bytes(n, k, W):
    """Bytes of the row-part sums a packed sweep writes: k floats for every
    row and every strip right of the row's own."""
    ns = (n + W - 1) // W
    return float(sum(min(W, n - s * W) * (ns - s - 1) for s in range(ns))) * k * 4


def iter_spans(kkm, runs, per_run):
    """Per-step durations (ms) of the recorded iterate launches: `runs` fixed-length
    runs of `per_run` launches each (the steps, then the final objective pass),
    iterations 2.. of every run."""
    import numpy as np
    sp = kkm.kkm_timing_spans("iterate")
    if sp.size != runs * per_run:
        raise RuntimeError("expected %d iterate launches, recorded %d" % (runs * per_run, sp.size))
    return sp.reshape(runs, per_run)[:, 1:per_run - 1].ravel() if per_run > 2 else sp


def gpu_same_prefix(kkm, torch, dev, w, rows, iters, reps=3):
    """The plain FP32 form on the same first `rows` points as the oracle: per-step
    median (iterations 2..30) and the Gram."""
    import numpy as np
    X, _ = w.points(rows=rows)
    Xd = torch.from_numpy(X).to(dev)
    ld = torch.from_numpy(w.labels0(rows=rows)).to(dev)
    K = kkm.alloc_kernel_matrix(rows, kkm.F32, dev)

    def run():
        return kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, w.coef0, w.degree, max_iter=iters,
                              check_convergence=False, K_ws=K)

    run()
    torch.cuda.synchronize()
    kkm.kkm_timing_enable(True)
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    its = iter_spans(kkm, reps, iters + 1)
    gram = kkm.kkm_timing_spans("gram")
    kkm.kkm_timing_enable(False)
    del K
    med = float(np.median(its))
    return {"rows": rows, "iter_ms": med, "iters_per_s": 1e3 / med, "gram_ms": float(np.median(gram))}


def train_feature_map(kkm, torch, w, dev):
    """Train phi_theta on 10^7 kernel values of fresh draws of the same mixture:
    TRAIN_STEPS batches of TRAIN_BATCH new points, each batch's kernel values
    computed by the Gram kernel.  Returns (params, report)."""
    import datagen
    m = TRAIN_STEPS * TRAIN_BATCH
    train_seed = w.data_seed + 30000 if w.train_seed is None else w.train_seed
    init_seed = w.data_seed + 30002 if w.init_seed is None else w.init_seed
    Xtr, _ = datagen.gmm(m, w.d, w.k, 0.5, train_seed, means=w.means())
    params = torch.from_numpy(datagen.mlp_init_params(w.d, H1, H2, OUT, init_seed)).to(dev)
    mo, vo = torch.zeros_like(params), torch.zeros_like(params)
    Xd = torch.from_numpy(Xtr).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = kkm.kkm_mlp_train_fresh(params, mo, vo, Xd, TRAIN_BATCH, w.kernel, w.gamma, lr=TRAIN_LR)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    lh = losses.cpu().numpy()
    rep = {"train_points": m, "kernel_values": TRAIN_STEPS * TRAIN_BATCH ** 2, "batch": TRAIN_BATCH,
           "steps": TRAIN_STEPS, "seconds": secs, "loss_first10": float(lh[:10].mean()),
           "loss_last10": float(lh[-10:].mean()), "params": int(params.numel()),
           "net": "%d-%d-%d-%d GELU" % (w.d, H1, H2, OUT)}
    log("feature map trained in %.2f s: loss %.4g -> %.4g" % (secs, rep["loss_first10"], rep["loss_last10"]))
    return params, rep


def warm_uniforms(k, seed):
    """The uniforms of the WARM_RESTARTS seedings: restart r draws with seed + r."""
    import numpy as np

    import datagen
    return np.stack([datagen.uniforms(k, seed + r) for r in range(WARM_RESTARTS)])


def warm_labels(kkm, w, params, Xd, seed, streams=WARM_STREAMS):
    """The learned warm start (kkm_warm_start): phi_theta(X), WARM_RESTARTS
    k-means++ seedings each followed by Lloyd in feature space on `streams`
    internal streams, the lowest feature-space objective kept.  Returns (labels,
    cheap iterations summed over restarts)."""
    r = kkm.kkm_warm_start(params, Xd, w.k, warm_uniforms(w.k, seed), max_iter=WARM_MAX_ITER,
                           streams=streams, h1=H1, h2=H2, out=OUT)
    return r["labels"], r["cheap_iters"]


def timed_runs(torch, fn, reps=3):
    """One untimed call, then `reps` timed ones; (median seconds, last result)."""
    import numpy as np
    fn()
    out, ts = None, []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts)), out


def speedups(plain_s, control_s, learned_s, train_s):
    """Time-to-converge ratios of the learned form against plain FP32 and
    against the same precision from random labels, without and with the
    feature network's training time."""
    return {"vs_plain_fp32": plain_s / learned_s, "vs_bf16_random_start": control_s / learned_s,
            "vs_plain_fp32_incl_training": plain_s / (learned_s + train_s),
            "vs_bf16_random_start_incl_training": control_s / (learned_s + train_s)}


def learned_c5_leg(kkm, torch, dev):
    """The learned warm start on its own workload: phi_theta trained on 10^7
    kernel values of the 32-component mixture in R^128, then fresh n=100000
    draws, k=32, all to convergence: plain FP32 from random labels, the BF16
    form from the same random labels (the control), the BF16 form from the
    learned warm start, and the FP32 form from the warm start (the reference
    for the result, ARI; and the exact iterations at equal precision); every
    run on the strip-packed K."""
    import datagen
    w = datagen.WORKLOADS["learned100k"]
    X, truth = w.points()
    Xd = torch.from_numpy(X).to(dev)
    ld = torch.from_numpy(w.labels0()).to(dev)
    n = w.n
    params, train_rep = train_feature_map(kkm, torch, w, dev)
    K = kkm.alloc_packed_kernel_matrix(n, kkm.F32, dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    useed = w.label_seed + 30003

    plain_s, rp = timed_runs(torch, lambda: kkm.kkm_fit_packed(
        Xd, w.k, ld, w.kernel, w.gamma, max_iter=w.max_iter, check_convergence=True, K_ws=K,
        labels_out=lab))
    plain_labels = lab.cpu().numpy()
    warm, _ = warm_labels(kkm, w, params, Xd, useed)
    ref = kkm.kkm_fit_packed(Xd, w.k, warm, w.kernel, w.gamma, max_iter=w.max_iter,
                             check_convergence=True, K_ws=K, labels_out=lab)
    ref_labels = lab.cpu().numpy()
    del K
    torch.cuda.empty_cache()
    K16 = kkm.alloc_packed_kernel_matrix(n, kkm.BF16, dev)
    lab16 = torch.empty(n, dtype=torch.int32, device=dev)
    control_s, rc = timed_runs(torch, lambda: kkm.kkm_fit_packed(
        Xd, w.k, ld, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16, max_iter=w.max_iter,
        check_convergence=True, K_ws=K16, labels_out=lab16))
    control_labels = lab16.cpu().numpy()

    def learned_run():
        ta = time.perf_counter()
        wl, ch = warm_labels(kkm, w, params, Xd, useed)
        tb = time.perf_counter()
        r = kkm.kkm_fit_packed(Xd, w.k, wl, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                               max_iter=w.max_iter, check_convergence=True, K_ws=K16, labels_out=lab16)
        return tb - ta, ch, r

    secs, (ws_s, ch, r) = timed_runs(torch, learned_run)
    ml = lab16.cpu().numpy()
    del K16
    torch.cuda.empty_cache()
    rec = {
        "workload": "learned100k: fresh draws n=%d of the 32-component mixture in R^%d (sigma 0.5; "
                    "means seed 5000, training draws 5001, points 5002, labels 5003), k=%d, "
                    "gaussian gamma=1/%d" % (n, w.d, w.k, w.d),
        "k_layout": "strip-packed upper triangle (every run)",
        "training": train_rep,
        "plain_fp32": {"seconds": plain_s, "iters": rp["iters"], "objective": rp["objective"],
                       "gram_ms": rp["times_ms"][0], "ari_vs_truth": ari(plain_labels, truth)},
        "bf16_random_start": {"seconds": control_s, "iters": rc["iters"], "objective": rc["objective"],
                              "gram_ms": rc["times_ms"][0], "ari_vs_truth": ari(control_labels, truth)},
        "mixed_learned": {"seconds": secs, "warm_start_seconds": ws_s,
                          "cheap_iters": ch, "exact_iters": r["iters"], "objective": r["objective"],
                          "gram_ms": r["times_ms"][0], "ari_vs_truth": ari(ml, truth),
                          "ari_vs_fp32_from_same_warm_start": ari(ml, ref_labels)},
        "fp32_from_warm_start": {"iters": ref["iters"], "objective": ref["objective"]},
        "exact_iters_saved_fp32": rp["iters"] - ref["iters"],
        "exact_iters_saved_bf16": rc["iters"] - r["iters"],
        "objective_rel_gap_vs_plain": (r["objective"] - rp["objective"]) / abs(rp["objective"]),
        "speedup_time_to_converge": speedups(plain_s, control_s, secs, train_rep["seconds"]),
    }
    log("learned100k: plain %.3f s (%d iters, J %.2f), bf16 random start %.3f s (%d iters), "
        "mixed+learned %.3f s (%d cheap + %d exact, J %.2f), ARI vs FP32 from same start %.4f" % (
            plain_s, rp["iters"], rp["objective"], control_s, rc["iters"], secs, ch, r["iters"],
            r["objective"], rec["mixed_learned"]["ari_vs_fp32_from_same_warm_start"]))
    return rec


def fixed_iteration_leg(kkm, torch, dev, w, reps=3):
    """The plain FP32 form on workload w with its fixed iteration count: Gram
    and sweep rooflines and the per-step time (iterations 2.. of each run)."""
    import numpy as np
    X, truth = w.points()
    n = w.n
    Xd = torch.from_numpy(X).to(dev)
    ld = torch.from_numpy(w.labels0()).to(dev)
    K = kkm.alloc_kernel_matrix(n, kkm.F32, dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)

    def run():
        return kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, w.coef0, w.degree, max_iter=w.max_iter,
                              check_convergence=False, K_ws=K, labels_out=lab)

    run()
    torch.cuda.synchronize()
    kkm.kkm_timing_enable(True)
    for _ in range(reps):
        r = run()
    torch.cuda.synchronize()
    its = iter_spans(kkm, reps, w.max_iter + 1)
    gram = float(np.median(kkm.kkm_timing_spans("gram")))
    sweep = float(np.median(kkm.kkm_timing_spans("sweep")))
    kkm.kkm_timing_enable(False)
    labels = lab.cpu().numpy()
    del K
    torch.cuda.empty_cache()
    flops = float(n) * (n + 1) * w.d
    kbytes = float(n) * n * 4
    med = float(np.median(its))
    return {"n": n, "d": w.d, "k": w.k, "iterations": w.max_iter, "objective": r["objective"],
            "ari_vs_truth": ari(labels, truth),
            "iter_ms": med, "iters_per_s": 1e3 / med,
            "gram": {"kernel": "gram_f32_mfma", "avg_ms": gram, "algorithmic_flops": flops,
                     "achieved_tflops": flops / (gram * 1e-3) / 1e12,
                     "frac": flops / (gram * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFS},
            "sweep": {"kernel": "spmm_row_sweep", "avg_ms": sweep, "algorithmic_bytes": kbytes,
                      "achieved_gbs": kbytes / (sweep * 1e-3) / 1e9,
                      "frac": kbytes / (sweep * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def mnist_leg(kkm, torch, dev):
    """The MNIST-shaped stand-in: n=60000, d=784, k=10, polynomial (x.y+1)^2,
    30 fixed iterations, FP32 Gram and K (14.4 GB)."""
    import datagen
    w = datagen.WORKLOADS["mnist_like"]
    rec = fixed_iteration_leg(kkm, torch, dev, w)
    rec["workload"] = ("mnist_like: 10 means U[0,1]^784, points clipped to [0,1], 80% of entries "
                       "zeroed; polynomial (x.y+1)^2")
    rec["targets"] = {"gram_ms_at_0.6_mfma": float(w.n) * (w.n + 1) * w.d / (0.6 * FP32_MFMA_PEAK_TFS * 1e12) * 1e3,
                      "sweep_ms_at_0.7_hbm": float(w.n) * w.n * 4 / (0.7 * HBM_PEAK_GBS * 1e9) * 1e3}
    log("mnist_like: gram %.2f ms (%.3f of FP32 MFMA), sweep %.3f ms (%.3f of HBM), %.3f ms per step" % (
        rec["gram"]["avg_ms"], rec["gram"]["frac"], rec["sweep"]["avg_ms"], rec["sweep"]["frac"],
        rec["iter_ms"]))
    return rec


def rings_leg(kkm, torch, dev, reps=5):
    """The rings workload (n=1000, k=4, Gaussian gamma=1): to convergence, the
    time per step in microseconds (K is 4 MB: launch and latency bound)."""
    import numpy as np

    import datagen
    w = datagen.WORKLOADS["rings"]
    X, truth = w.points()
    Xd = torch.from_numpy(X).to(dev)
    ld = torch.from_numpy(w.labels0()).to(dev)

    def run():
        return kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, max_iter=w.max_iter,
                              check_convergence=True)

    secs, r = timed_runs(torch, run, reps)
    kkm.kkm_timing_enable(True)
    run()
    torch.cuda.synchronize()
    its = kkm.kkm_timing_spans("iterate")
    kkm.kkm_timing_enable(False)
    med = float(np.median(its[1:]))
    return {"workload": "rings: n=1000, d=16, four rings, k=4, gaussian gamma=1",
            "iters": r["iters"], "objective": r["objective"],
            "ari_vs_truth": ari(r["labels"].cpu().numpy(), truth),
            "us_per_iter": med * 1e3, "seconds_to_converge": secs}


def matfree_leg(kkm, torch, dev, iters=30, ds=(32, 64, 128, 256)):
    """The matrix-free step (kernel values recomputed on the MFMA every step,
    no stored K) beside the stored-K step, BF16 product, n=100000, k=32: at
    d=128 on the learned warm-start workload's points, at the other d on a
    32-component mixture of the same recipe.  Per d: the median time of one
    step (iterations 2..30 of a fixed 30-iteration run), the matrix-free
    sweep's flop rate (2 n^2 d per step, the products it recomputes) against
    the BF16 MFMA peak, and the stored-K sweep's HBM rate (n^2 bfloat16
    entries read per step); at d=128 also both forms to convergence from the
    random labels."""
    import numpy as np

    import datagen
    w = datagen.WORKLOADS["learned100k"]
    n, k = w.n, w.k
    out = {"n": n, "k": k, "gram": "bf16 mfma", "iterations": iters, "by_d": []}
    for d in ds:
        if d == w.d:
            X, _ = w.points()
            l0 = w.labels0()
        else:
            X, _ = datagen.gmm(n, d, k, 0.5, 7000 + d)
            l0 = datagen.uniform_labels(n, k, 7100 + d)
        gamma = 1.0 / d
        Xd = torch.from_numpy(X).to(dev)
        ld = torch.from_numpy(l0).to(dev)
        K16 = kkm.alloc_kernel_matrix(n, kkm.BF16, dev)
        lab = torch.empty(n, dtype=torch.int32, device=dev)

        def stored(max_iter=iters, conv=False):
            return kkm.kkm_fit_ex(Xd, k, ld, kkm.GAUSS, gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                                  max_iter=max_iter, check_convergence=conv, K_ws=K16, labels_out=lab)

        def matfree(max_iter=iters, conv=False):
            return kkm.kkm_fit_matfree(Xd, k, ld, kkm.GAUSS, gamma, gram_prec=kkm.BF16,
                                       max_iter=max_iter, check_convergence=conv, labels_out=lab)

        rec = {"d": d}
        for name, fn in (("stored_k", stored), ("matfree", matfree)):
            fn(3)
            torch.cuda.synchronize()
            kkm.kkm_timing_enable(True)
            r = fn()
            torch.cuda.synchronize()
            its = iter_spans(kkm, 1, iters + 1)
            sw = float(np.median(kkm.kkm_timing_spans("sweep")))
            kkm.kkm_timing_enable(False)
            med = float(np.median(its))
            rr = {"iter_ms": med, "sweep_ms": sw, "objective_30": r["objective"]}
            if name == "stored_k":
                rr["sweep_hbm_gbs"] = float(n) * n * 2 / (sw * 1e-3) / 1e9
                rr["sweep_frac_hbm"] = rr["sweep_hbm_gbs"] / HBM_PEAK_GBS
            else:
                fl = 2.0 * n * n * d
                rr["sweep_tflops"] = fl / (sw * 1e-3) / 1e12
                rr["sweep_frac_bf16_mfma"] = rr["sweep_tflops"] / BF16_MFMA_PEAK_TFS
            rec[name] = rr
        rec["matfree_over_stored_step_time"] = rec["matfree"]["iter_ms"] / rec["stored_k"]["iter_ms"]
        if d == w.d:
            cs, rc = timed_runs(torch, lambda: stored(300, True), reps=2)
            lc = lab.cpu().numpy()
            ms, rm = timed_runs(torch, lambda: matfree(300, True), reps=2)
            lm = lab.cpu().numpy()
            rec["to_convergence"] = {
                "stored_k": {"seconds": cs, "iters": rc["iters"], "objective": rc["objective"]},
                "matfree": {"seconds": ms, "iters": rm["iters"], "objective": rm["objective"]},
                "ari_matfree_vs_stored": ari(lm, lc)}
        log("matfree d=%d: step %.3f ms (sweep %.3f ms, %.0f TF/s = %.3f of BF16 MFMA) vs stored-K "
            "step %.3f ms (sweep %.3f ms, %.3f of HBM)" % (
                d, rec["matfree"]["iter_ms"], rec["matfree"]["sweep_ms"],
                rec["matfree"]["sweep_tflops"], rec["matfree"]["sweep_frac_bf16_mfma"],
                rec["stored_k"]["iter_ms"], rec["stored_k"]["sweep_ms"],
                rec["stored_k"]["sweep_frac_hbm"]))
        out["by_d"].append(rec)
        del K16, Xd
        torch.cuda.empty_cache()
    return out


def packed_leg(kkm, torch, dev, iters=30, reps=2):
    """The strip-packed symmetric K (upper triangle in strips, each stored
    entry read once per step) beside the dense K on the benchmark workload
    (n=200000, d=1024, k=64): FP32 and bfloat16 storage, 30 fixed iterations
    from the random labels.  Per form: the median step (iterations 2..30), the
    packed sweep kernel (both parts) against the bytes it must move (the packed
    entries, about n^2/2 s_K, plus the row-part sums it writes), the fold of
    the row part, and the Gram writing
    the packed K; and to convergence from the random labels (FP32) and from
    nothing else."""
    import numpy as np

    import datagen
    w = datagen.WORKLOADS["gmm200k"]
    n = w.n
    X, _ = w.points()
    Xd = torch.from_numpy(X).to(dev)
    del X
    ld = torch.from_numpy(w.labels0()).to(dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    out = {"n": n, "d": w.d, "k": w.k, "iterations": iters}
    for name, ks in (("f32", kkm.F32), ("bf16", kkm.BF16)):
        Kp = kkm.alloc_packed_kernel_matrix(n, ks, dev)
        eb = 4 if ks == kkm.F32 else 2

        def run(max_iter=iters, conv=False):
            return kkm.kkm_fit_packed(Xd, w.k, ld, w.kernel, w.gamma, gram_prec=ks, k_store=ks,
                                      max_iter=max_iter, check_convergence=conv, K_ws=Kp,
                                      labels_out=lab)

        run(2)
        torch.cuda.synchronize()
        kkm.kkm_timing_enable(True)
        for _ in range(reps):
            r = run()
        torch.cuda.synchronize()
        its = iter_spans(kkm, reps, iters + 1)
        sw = float(np.median(kkm.kkm_timing_spans("sweep")))
        fold = float(np.median(kkm.kkm_timing_spans("fold")))
        gram = float(np.median(kkm.kkm_timing_spans("gram")))
        kkm.kkm_timing_enable(False)
        pbytes = float(kkm.packed_elements(n, ks)) * eb
        rpb = rowpart_bytes(n, w.k, 1024)
        med = float(np.median(its))
        rec = {"k_store": name, "packed_bytes": pbytes, "rowpart_bytes": rpb,
               "dense_bytes": float(n) * n * eb, "iter_ms": med, "iters_per_s": 1e3 / med,
               "sweep_ms": sw, "fold_ms": fold,
               "sweep_gbs": (pbytes + rpb) / (sw * 1e-3) / 1e9,
               "sweep_frac_hbm": (pbytes + rpb) / (sw * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "gram_ms": gram, "objective_30": r["objective"]}
        if ks == kkm.F32:
            cs, rc = timed_runs(torch, lambda: run(300, True), reps=1)
            rec["to_convergence"] = {"seconds": cs, "iters": rc["iters"], "objective": rc["objective"]}
        log("packed %s: step %.3f ms (%.1f iters/s), sweep %.3f ms = %.0f GB/s on %.1f GB (%.3f of HBM), "
            "fold %.3f ms, gram %.1f ms" % (name, med, 1e3 / med, sw, rec["sweep_gbs"],
                                            (pbytes + rpb) / 1e9, rec["sweep_frac_hbm"], fold, gram))
        out[name] = rec
        del Kp
        torch.cuda.empty_cache()
    return out


def profile_kernels(kkm, torch, dev):
    """One launch of each product kernel at its benchmark size, for counter
    collection under rocprofv3: the FP32 and the BF16 Gram at n=200000,
    d=1024 (K stored FP32 / bfloat16) with two steps on each K, the packed
    Gram and two packed steps for both element types, the BF16 Gram at
    n=100000, d=128, and two matrix-free steps there (BF16 product)."""
    import datagen
    out = {}
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points()
    Xd = torch.from_numpy(X).to(dev)
    del X
    ld = torch.from_numpy(w.labels0()).to(dev)
    for name, gp, ks in (("gram_f32_gmm200k", kkm.F32, kkm.F32), ("gram_bf16_gmm200k", kkm.BF16, kkm.BF16)):
        K = kkm.alloc_kernel_matrix(w.n, ks, dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        K, dg = kkm.kkm_gram(Xd, w.kernel, w.gamma, gram_prec=gp, k_store=ks, K=K)
        torch.cuda.synchronize()
        out[name] = time.perf_counter() - t
        for _ in range(2):  # two steps of the dense sweep on this K
            kkm.kkm_iterate(K, dg, ld, w.k)
        torch.cuda.synchronize()
        log("profile: %s %.3f s, two steps" % (name, out[name]))
        del K
        torch.cuda.empty_cache()
    for name, ks in (("packed_f32_gmm200k", kkm.F32), ("packed_bf16_gmm200k", kkm.BF16)):
        Kp, dg = kkm.kkm_gram_packed(Xd, w.kernel, w.gamma, gram_prec=ks, k_store=ks)
        for _ in range(2):
            kkm.kkm_iterate_packed(Kp, dg, ld, w.k)
        torch.cuda.synchronize()
        log("profile: %s, two steps" % name)
        del Kp
        torch.cuda.empty_cache()
    del Xd
    w = datagen.WORKLOADS["learned100k"]
    X, _ = w.points()
    Xd = torch.from_numpy(X).to(dev)
    ld = torch.from_numpy(w.labels0()).to(dev)
    K = kkm.alloc_kernel_matrix(w.n, kkm.BF16, dev)
    kkm.kkm_gram(Xd, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16, K=K)
    torch.cuda.synchronize()
    del K
    torch.cuda.empty_cache()
    log("profile: gram_bf16_learned100k done")
    for _ in range(2):
        kkm.kkm_iterate_matfree(Xd, ld, w.k, w.kernel, w.gamma, gram_prec=kkm.BF16)
    torch.cuda.synchronize()
    log("profile: matfree steps done")
    return out


def error_report(K_or, k, labels_in, orc, D, J):
    """One step's error against the oracle's step from the same labels: the
    largest distance error over the condition scale sigma_i = |K_ii| +
    max_c (2|E_ic| + |C_c|), the relative objective error and the fraction of
    labels that differ."""
    import numpy as np
    n = K_or.shape[0]
    V = np.zeros((n, k))
    V[np.arange(n), labels_in] = 1.0
    cnt = V.sum(0)
    S = K_or @ V
    live = cnt > 0
    E = np.where(live, S / np.maximum(cnt, 1), 0.0)
    C = np.where(live, (V * S).sum(0) / np.maximum(cnt, 1) ** 2, 0.0)
    sig = np.abs(np.diag(K_or)) + (2 * np.abs(E[:, live]) + np.abs(C[live])).max(axis=1)
    fin = np.isfinite(orc["D"])
    err = np.where(fin, np.abs(D.astype(np.float64) - np.where(fin, orc["D"], 0.0)), 0.0)
    return {"max_dist_err_over_sigma": float((err / sig[:, None]).max()),
            "objective_rel_err": abs(J - orc["J_in"]) / abs(orc["J_in"])}


def metric_check_20k(kkm, torch, dev, w, rows, params, K_or, seed):
    """The metric form against the FP64 oracle on the first `rows` points: the
    learned warm start of these points, every precision pair refined from it to
    convergence and compared with the oracle converged from the same labels,
    and one step from the warm labels against the oracle's step."""
    import oracle
    X, truth = w.points(rows=rows)
    Xd = torch.from_numpy(X).to(dev)
    warm, _ = warm_labels(kkm, w, params, Xd, seed)
    warm_h = warm.cpu().numpy()
    t = time.perf_counter()
    ref = oracle.fit(K_or, w.k, warm_h, 300)
    orc = oracle.step(K_or, w.k, warm_h, want_gap=False)
    log("oracle from warm labels on %d points: %d iterations, J %.6f (%.1f s)" % (
        rows, ref["iters"], ref["objective"], time.perf_counter() - t))
    pairs = (("f32/f32", kkm.F32, kkm.F32), ("bf16/f32", kkm.BF16, kkm.F32),
             ("bf16/bf16", kkm.BF16, kkm.BF16), ("fp8/f32", kkm.FP8_ROWSCALED, kkm.F32),
             ("fp8/bf16", kkm.FP8_ROWSCALED, kkm.BF16))
    forms = {}
    for name, gp, ks in pairs:
        r = kkm.kkm_fit_ex(Xd, w.k, warm, w.kernel, w.gamma, gram_prec=gp, k_store=ks, max_iter=300,
                           check_convergence=True)
        lab = r["labels"].cpu().numpy()
        J_or_of_gpu = oracle.objective(K_or, w.k, lab)
        K, dg = kkm.kkm_gram(Xd, w.kernel, w.gamma, gram_prec=gp, k_store=ks)
        lo, _, _, Jin, D, _ = kkm.kkm_iterate(K, dg, warm, w.k, D_out=True)
        torch.cuda.synchronize()
        rep = error_report(K_or, w.k, warm_h, orc, D.cpu().numpy(), float(Jin.item()))
        rep["step_label_flip_frac"] = float((lo.cpu().numpy() != orc["labels"]).mean())
        del K, D
        rep.update({"ari_vs_oracle_from_same_warm_start": ari(lab, ref["labels"]),
                    "exact_iters": r["iters"], "oracle_iters": ref["iters"],
                    "objective_gap_rel": (J_or_of_gpu - ref["objective"]) / abs(ref["objective"]),
                    "ari_vs_truth": ari(lab, truth)})
        forms[name] = rep
        log("  %s: ARI vs oracle %.4f, %d vs %d iterations, J gap %.2e, step: max dD/sigma %.2e, "
            "dJ/J %.2e, flips %.4f" % (name, rep["ari_vs_oracle_from_same_warm_start"], r["iters"],
                                      ref["iters"], rep["objective_gap_rel"],
                                      rep["max_dist_err_over_sigma"], rep["objective_rel_err"],
                                      rep["step_label_flip_frac"]))
    torch.cuda.empty_cache()
    return {"rows": rows, "oracle_iters": ref["iters"], "oracle_objective": ref["objective"],
            "oracle_ari_vs_truth": ari(ref["labels"], truth), "forms": forms}


def batched_leg(kkm, torch, dev, iters):
    """The batched form: 512 uneven Gaussian-mixture problems, BF16 Gram, FP32 K."""
    import numpy as np

    import datagen
    from paper_2501_05587_amd import autotune

    specs = datagen.batched_instances(512)
    t = time.perf_counter()
    probs, labs = [], []
    for s in specs:
        X, _ = datagen.gmm(s["n"], s["d"], s["k"], s["sigma"], s["seed"])
        probs.append(dict(X=torch.from_numpy(X).to(dev), k=s["k"], kernel=kkm.GAUSS,
                          gamma=s["gamma"]))
        labs.append(datagen.uniform_labels(s["n"], s["k"], s["label_seed"]))
    l0 = torch.from_numpy(np.concatenate(labs)).to(dev)
    nn = np.array([s["n"] for s in specs], dtype=np.float64)
    dd = np.array([s["d"] for s in specs], dtype=np.float64)
    k_bytes = float((nn * nn).sum() * 4)           # every K read once per step
    gram_flops = float((nn * (nn + 1) * dd).sum())  # upper triangles, 2 flops per term
    log("batched: %d problems, sum n %d, sum K %.1f GB, generated in %.1f s" % (
        len(specs), int(nn.sum()), k_bytes / 1e9, time.perf_counter() - t))
    table = autotune.load(torch=torch)
    tuned = autotune.apply(probs, table, 0)
    ws_bytes = max(kkm.kkm_fit_batched_workspace_bytes(ps, kkm.BF16, kkm.F32)
                   for ps in (tuned, probs))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    lab = torch.empty_like(l0)

    def run(ps, graph=True, max_iter=iters, conv=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = kkm.kkm_fit_batched(ps, l0, gram_prec=kkm.BF16, k_store=kkm.F32, max_iter=max_iter,
                                check_convergence=conv, use_graph=graph, labels_out=lab, ws=ws)
        torch.cuda.synchronize()
        r["wall_s"] = time.perf_counter() - t0
        return r

    run(tuned)  # warm-up
    kkm.kkm_timing_enable(True)
    r_tuned = run(tuned)
    tim = kkm.kkm_timing_read()
    kkm.kkm_timing_enable(False)
    r_default = run(probs)
    kkm.kkm_timing_enable(True)
    r_eager = run(tuned, graph=False)
    tim_e = kkm.kkm_timing_read()
    kkm.kkm_timing_enable(False)
    r_conv = run(tuned, max_iter=300, conv=True)
    per_step = r_tuned["times_ms"][1] / iters
    gram_ms = tim["gram"][0] / max(tim["gram"][1], 1)
    sweep_ms = tim_e["sweep"][0] / max(tim_e["sweep"][1], 1)
    out = {
        "workload": "512 problems: n U{256..16384}, d in {32,64,128,256}, k U{2..64}, "
                    "k-component mixtures sigma 0.3, gaussian gamma=1/d",
        "problems": len(specs), "sum_n": int(nn.sum()), "sum_K_bytes": k_bytes,
        "gram": "bf16 mfma, persistent tile queue", "k_store": "f32",
        "iterations": iters, "graph": True,
        "tuned_table": bool(table), "tuned_chunk_rows": sorted(set(p["chunk_rows"] for p in tuned)),
        "gram_ms": gram_ms,
        "gram_achieved_tflops": gram_flops / (gram_ms * 1e-3) / 1e12,
        "gram_frac_bf16_mfma": gram_flops / (gram_ms * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFS,
        "gram_write_gbs": k_bytes / (gram_ms * 1e-3) / 1e9,
        "gram_write_frac_hbm": k_bytes / (gram_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_ms": per_step,
        "aggregate_gbs": k_bytes / (per_step * 1e-3) / 1e9,
        "frac_hbm": k_bytes / (per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_ms_default_chunk_rows": r_default["times_ms"][1] / iters,
        "step_ms_eager": r_eager["times_ms"][1] / iters,
        "sweep_ms": sweep_ms,
        "sweep_frac_hbm": k_bytes / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "iters_per_s": iters / (r_tuned["times_ms"][1] * 1e-3),
        "to_convergence": {"seconds": r_conv["wall_s"], "gram_ms": r_conv["times_ms"][0],
                           "loop_ms": r_conv["times_ms"][1],
                           "iters_max": int(r_conv["iters"].max()),
                           "iters_median": float(np.median(r_conv["iters"])),
                           "iters_min": int(r_conv["iters"].min())},
    }
    del ws
    torch.cuda.empty_cache()
    log("batched: gram %.1f ms, %.2f ms/step (%.0f GB/s, %.3f of HBM), default chunks %.2f ms, "
        "eager %.2f ms; converged in %.3f s (max %d steps)" % (
            gram_ms, per_step, out["aggregate_gbs"], out["frac_hbm"],
            out["step_ms_default_chunk_rows"], out["step_ms_eager"], r_conv["wall_s"],
            out["to_convergence"]["iters_max"]))
    return out


def gram_shapes(kkm, torch, dev):
    """Triangle (SYRK work, mirrored stores) against full (GEMM work) tile shapes
    of the FP32 Gram over n and d, the paper's architecture-dependent switch
    (it switches to GEMM above n/d = 100 on its GPU).  Returns a list of rows."""
    rows = []
    for n in (20000, 60000, 100000):
        K = kkm.alloc_kernel_matrix(n, kkm.F32, dev)
        diag = torch.empty(n, dtype=torch.float32, device=dev)
        for d in (16, 64, 256, 1024):
            g = torch.Generator(device=dev)
            g.manual_seed(n + d)
            X = torch.randn(n, d, generator=g, device=dev)
            row = {"n": n, "d": d, "n_over_d": n / d}
            for name, shape in (("triangle_ms", kkm.GRAM_TRIANGLE), ("full_ms", kkm.GRAM_FULL)):
                best = float("inf")
                for _ in range(3):
                    kkm.kkm_timing_enable(True)
                    kkm.kkm_gram(X, kkm.GAUSS, 1.0 / d, K=K, diagK=diag, shape=shape)
                    torch.cuda.synchronize()
                    best = min(best, kkm.kkm_timing_read()["gram"][0])
                    kkm.kkm_timing_enable(False)
                row[name] = best
            row["full_over_triangle"] = row["full_ms"] / row["triangle_ms"]
            rows.append(row)
            log("gram shapes n=%d d=%d: triangle %.2f ms, full %.2f ms" % (
                n, d, row["triangle_ms"], row["full_ms"]))
        del K
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows", type=int, default=0, help="use only the first N points (0 = all)")
    ap.add_argument("--iters", type=int, default=0, help="override the 30 fixed iterations")
    ap.add_argument("--cpu-rows", type=int, default=20000)
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle's K build and every loop iteration at one thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the MNIST-shaped and rings legs")
    ap.add_argument("--learned-only", action="store_true",
                    help="run only the learned warm start on its n=100000, k=32 workload")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched form and print its record")
    ap.add_argument("--matfree-only", action="store_true",
                    help="run only the matrix-free step beside the stored-K step (n=100000, k=32)")
    ap.add_argument("--no-matfree", action="store_true")
    ap.add_argument("--packed-only", action="store_true",
                    help="run only the strip-packed K beside the dense K (n=200000, FP32 and BF16)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="one launch of each product kernel at its benchmark size (for rocprofv3)")
    ap.add_argument("--gram-shapes", action="store_true",
                    help="time the triangle and full tile shapes of the Gram over n and d")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_2501_05587_amd as kkm

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gram_shapes:
        print(json.dumps({"gram_shapes": gram_shapes(kkm, torch, dev)}), flush=True)
        return
    if args.matfree_only:
        print(json.dumps({"matfree": matfree_leg(kkm, torch, dev)}), flush=True)
        return
    if args.packed_only:
        print(json.dumps({"packed": packed_leg(kkm, torch, dev)}), flush=True)
        return
    if args.profile_kernels:
        print(json.dumps({"profile_kernels": profile_kernels(kkm, torch, dev)}), flush=True)
        return
    if args.learned_only:
        print(json.dumps(learned_c5_leg(kkm, torch, dev)), flush=True)
        return
    if args.batched_only:
        print(json.dumps(batched_leg(kkm, torch, dev, args.iters or 30)), flush=True)
        return

    w = datagen.WORKLOADS["gmm200k"]
    n = args.rows or w.n
    iters = args.iters or w.max_iter
    log("workload %s: n=%d d=%d k=%d gamma=%g, %d iterations" % (w.name, n, w.d, w.k, w.gamma, iters))
    t = time.perf_counter()
    X, truth = w.points(rows=n)
    l0 = w.labels0(rows=n)
    log("data generated in %.1f s" % (time.perf_counter() - t))

    Xd = torch.from_numpy(X).to(dev)
    ld = torch.from_numpy(l0).to(dev)
    K = kkm.alloc_kernel_matrix(n, kkm.F32, dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    del X
    torch.cuda.synchronize()

    # ------------------------------------------------------------ plain FP32, fixed 30 iterations
    def step():
        return kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, w.coef0, w.degree,
                              max_iter=iters, check_convergence=False, K_ws=K, labels_out=lab)

    for i in range(args.warmup):
        r = step()
        log("warmup %d: gram %.1f ms, steps %.1f ms, J=%.6f" % (i, r["times_ms"][0], r["times_ms"][1],
                                                              r["objective"]))
    torch.cuda.synchronize()
    kkm.kkm_timing_enable(True)
    t0 = time.perf_counter()
    rs = []
    for i in range(args.steps):
        rs.append(step())
        log("step %d done: gram %.1f ms, %d steps %.1f ms" % (i, rs[-1]["times_ms"][0],
                                                           rs[-1]["iters"], rs[-1]["times_ms"][1]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = kkm.kkm_timing_read()
    step_spans = iter_spans(kkm, args.steps, iters + 1)
    kkm.kkm_timing_enable(False)
    wall = t1 - t0
    total_iters = sum(r["iters"] for r in rs)
    gram_ms = float(np.mean([r["times_ms"][0] for r in rs]))
    iter_ms = float(np.median(step_spans))

    sweep_ms = tim["sweep"][0] / max(tim["sweep"][1], 1)
    sweep_bytes = float(n) * n * 4  # K read once per sweep
    gram_launch_ms = tim["gram"][0] / max(tim["gram"][1], 1)
    gram_flops = float(n) * (n + 1) * w.d  # n(n+1)/2 dot products of length d, 2 flops each
    roof = {"bound": "hbm", "kernel": "spmm_row_sweep", "achieved": sweep_bytes / (sweep_ms * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic_bytes("spmm_row_sweep", n),
            "algorithmic_bytes": sweep_bytes, "avg_ms": sweep_ms, "launches": tim["sweep"][1]}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof_g = {"bound": "mfma", "kernel": "gram_f32_mfma",
              "achieved": gram_flops / (gram_launch_ms * 1e-3) / 1e12, "peak": FP32_MFMA_PEAK_TFS,
              "unit": "TFLOP/s", "traffic": traffic_bytes("gram_f32_mfma", n),
              "algorithmic_flops": gram_flops, "avg_ms": gram_launch_ms, "launches": tim["gram"][1]}
    roof_g["frac"] = roof_g["achieved"] / roof_g["peak"]
    dense = {"iter_ms": iter_ms, "iters_per_s": 1e3 / iter_ms, "gram_ms": gram_ms,
             "ms_per_step": wall / args.steps * 1e3, "iters_per_s_incl_gram": total_iters / wall,
             "k_store": "f32 [n, ldk] row-major, both triangles", "roofline": roof}

    # ------------------------------------------------------------ plain FP32, strip-packed K (headline)
    # K's upper triangle stored once in strips of 1024 columns; each stored
    # entry is read once per step and feeds both sides of the sum
    Kp = kkm.alloc_packed_kernel_matrix(n, kkm.F32, dev)

    def pstep(max_iter=iters, conv=False):
        return kkm.kkm_fit_packed(Xd, w.k, ld, w.kernel, w.gamma, gram_prec=kkm.F32, k_store=kkm.F32,
                                  max_iter=max_iter, check_convergence=conv, K_ws=Kp, labels_out=lab)

    for i in range(args.warmup):
        pstep()
    torch.cuda.synchronize()
    kkm.kkm_timing_enable(True)
    t0 = time.perf_counter()
    prs = []
    for i in range(args.steps):
        prs.append(pstep())
        log("packed step %d done: gram %.1f ms, %d steps %.1f ms" % (i, prs[-1]["times_ms"][0],
                                                                  prs[-1]["iters"], prs[-1]["times_ms"][1]))
    torch.cuda.synchronize()
    pwall = time.perf_counter() - t0
    p_iter_ms = float(np.median(iter_spans(kkm, args.steps, iters + 1)))
    p_sweep = kkm.kkm_timing_spans("sweep")
    p_fold = kkm.kkm_timing_spans("fold")
    p_gram = kkm.kkm_timing_spans("gram")
    kkm.kkm_timing_enable(False)
    p_sweep_ms = float(np.mean(p_sweep))
    pbytes = float(kkm.packed_elements(n, kkm.F32)) * 4
    rp_bytes = rowpart_bytes(n, w.k, 1024)
    roof = {"bound": "hbm", "kernel": "packed_sweep<float>",
            "achieved": (pbytes + rp_bytes) / (p_sweep_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "traffic": traffic_bytes("packed_sweep", n),
            "algorithmic_bytes": pbytes + rp_bytes, "packed_k_bytes": pbytes, "rowpart_bytes": rp_bytes,
            "avg_ms": p_sweep_ms, "launches": int(p_sweep.size)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    packed = {"iter_ms": p_iter_ms, "iters_per_s": 1e3 / p_iter_ms,
              "gram_ms": float(np.mean(p_gram)), "sweep_ms": p_sweep_ms,
              "fold_ms": float(np.mean(p_fold)), "ms_per_step": pwall / args.steps * 1e3,
              "iters_per_s_incl_gram": sum(r["iters"] for r in prs) / pwall,
              "objective_30": prs[-1]["objective"]}
    log("packed FP32: %.3f ms per iteration (sweep %.3f ms = %.0f GB/s, fold %.3f ms), gram %.1f ms"
        % (p_iter_ms, p_sweep_ms, roof["achieved"], packed["fold_ms"], packed["gram_ms"]))
    plain = None
    if not args.no_converge:
        torch.cuda.synchronize()
        tc = time.perf_counter()
        rc = pstep(300, True)
        torch.cuda.synchronize()
        labs = lab.cpu().numpy()
        plain = {"k_store": "f32 strip-packed", "seconds": time.perf_counter() - tc, "iters": rc["iters"],
                 "objective": rc["objective"], "gram_ms": rc["times_ms"][0],
                 "iter_ms": rc["times_ms"][1] / max(rc["iters"], 1), "ari_vs_truth": ari(labs, truth),
                 "empty_clusters": int((np.bincount(labs, minlength=w.k) == 0).sum())}
        log("plain (packed K) converged: %d iterations in %.3f s, J=%.6f" % (rc["iters"], plain["seconds"],
                                                                            rc["objective"]))
    del Kp
    torch.cuda.empty_cache()

    # ------------------------------------------------------------ plain FP32 to convergence, dense K
    plain_dense = None
    if not args.no_converge:
        torch.cuda.synchronize()
        tc = time.perf_counter()
        rc = kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, w.coef0, w.degree, max_iter=300,
                            check_convergence=True, K_ws=K, labels_out=lab)
        torch.cuda.synchronize()
        labs = lab.cpu().numpy()
        plain_dense = {"k_store": "f32 dense", "seconds": time.perf_counter() - tc, "iters": rc["iters"],
                       "objective": rc["objective"], "gram_ms": rc["times_ms"][0],
                       "iter_ms": rc["times_ms"][1] / max(rc["iters"], 1), "ari_vs_truth": ari(labs, truth),
                       "empty_clusters": int((np.bincount(labs, minlength=w.k) == 0).sum())}
        log("plain (dense K) converged: %d iterations in %.3f s, J=%.6f" % (rc["iters"], plain_dense["seconds"],
                                                                            rc["objective"]))

    # ------------------------------------------------------------ mixed + learned
    learned = None
    params = None
    useed = w.label_seed + 30003
    if not args.no_learned and not args.no_converge:
        params, train_rep = train_feature_map(kkm, torch, w, dev)
        # reference: the plain FP32 form converged from the same warm labels
        warm, cheap = warm_labels(kkm, w, params, Xd, useed)
        ref = kkm.kkm_fit_ex(Xd, w.k, warm, w.kernel, w.gamma, max_iter=300, check_convergence=True,
                             K_ws=K, labels_out=lab)
        ref_labels = lab.cpu().numpy()
        log("reference from warm labels: %d iterations, J=%.6f" % (ref["iters"], ref["objective"]))
        del K
        torch.cuda.empty_cache()
        K16 = kkm.alloc_kernel_matrix(n, kkm.BF16, dev)  # dense: k-means++ on K reads it
        Kp16 = kkm.alloc_packed_kernel_matrix(n, kkm.BF16, dev)  # the refinement's K
        lab16 = torch.empty(n, dtype=torch.int32, device=dev)

        def mixed_learned():
            ta = time.perf_counter()
            wl, ch = warm_labels(kkm, w, params, Xd, useed)
            tb = time.perf_counter()
            r = kkm.kkm_fit_packed(Xd, w.k, wl, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                                   max_iter=300, check_convergence=True, K_ws=Kp16, labels_out=lab16)
            return tb - ta, ch, r

        def control():
            # the same precision and layout from the random labels
            return kkm.kkm_fit_packed(Xd, w.k, ld, w.kernel, w.gamma, gram_prec=kkm.BF16,
                                      k_store=kkm.BF16, max_iter=300, check_convergence=True,
                                      K_ws=Kp16, labels_out=lab16)

        def kernel_seeded():
            # the non-learned warm start: k-means++ on the exact kernel matrix
            ta = time.perf_counter()
            Kg, dg = kkm.kkm_gram(Xd, w.kernel, w.gamma, w.coef0, w.degree, gram_prec=kkm.BF16,
                                  k_store=kkm.BF16, K=K16)
            _, lab0 = kkm.kkm_kernel_kmeanspp(Kg, dg, w.k, datagen.uniforms(w.k, useed))
            torch.cuda.synchronize()
            tb = time.perf_counter()
            r = kkm.kkm_refine(Kg, dg, w.k, lab0, max_iter=300, labels_out=lab16)
            return tb - ta, r

        control_s, rcn = timed_runs(torch, control)
        control_labels = lab16.cpu().numpy()
        ks_secs, (ks_seed_s, kr) = timed_runs(torch, kernel_seeded)
        ks_labels = lab16.cpu().numpy()
        kseeded = {"seconds": ks_secs, "gram_and_seeding_seconds": ks_seed_s,
                   "exact_iters": kr["iters"], "objective": kr["objective"],
                   "ari_vs_truth": ari(ks_labels, truth),
                   "empty_clusters": int((np.bincount(ks_labels, minlength=w.k) == 0).sum())}
        log("kernel k-means++ + exact: %.3f s (Gram + seeding %.3f s, %d exact iterations), J=%.3f" % (
            ks_secs, ks_seed_s, kr["iters"], kr["objective"]))

        secs, (ws_s, ch, r) = timed_runs(torch, mixed_learned)
        ml_labels = lab16.cpu().numpy()
        # per-iteration rate of the mixed form: 30 fixed iterations on the packed BF16 K,
        # and on the dense BF16 K for comparison
        kkm.kkm_timing_enable(True)
        kkm.kkm_fit_packed(Xd, w.k, ld, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                           max_iter=iters, check_convergence=False, K_ws=Kp16, labels_out=lab16)
        torch.cuda.synchronize()
        tim16 = kkm.kkm_timing_read()
        it16 = float(np.median(iter_spans(kkm, 1, iters + 1)))
        kkm.kkm_timing_enable(False)
        sw16 = tim16["sweep"][0] / max(tim16["sweep"][1], 1)
        fold16 = tim16["fold"][0] / max(tim16["fold"][1], 1)
        gp16 = tim16["gram"][0] / max(tim16["gram"][1], 1)
        b16 = float(kkm.packed_elements(n, kkm.BF16)) * 2 + rowpart_bytes(n, w.k, 1024)
        kkm.kkm_timing_enable(True)
        kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                       max_iter=iters, check_convergence=False, K_ws=K16, labels_out=lab16)
        torch.cuda.synchronize()
        timd = kkm.kkm_timing_read()
        itd16 = float(np.median(iter_spans(kkm, 1, iters + 1)))
        kkm.kkm_timing_enable(False)
        swd16 = timd["sweep"][0] / max(timd["sweep"][1], 1)
        g16 = timd["gram"][0] / max(timd["gram"][1], 1)
        learned = {
            "seconds": secs, "warm_start_seconds": ws_s,
            "cheap_iters": ch, "exact_iters": r["iters"], "objective": r["objective"],
            "gram": "bf16 mfma", "k_store": "bf16 strip-packed", "gram_ms": r["times_ms"][0],
            "iter_ms": it16, "iters_per_s": 1e3 / it16,
            "ari_vs_fp32_from_same_warm_start": ari(ml_labels, ref_labels),
            "ari_vs_truth": ari(ml_labels, truth),
            "empty_clusters": int((np.bincount(ml_labels, minlength=w.k) == 0).sum()),
            "fp32_from_warm_start": {"iters": ref["iters"], "objective": ref["objective"]},
            "bf16_random_start": {"seconds": control_s, "iters": rcn["iters"],
                                  "objective": rcn["objective"],
                                  "ari_vs_truth": ari(control_labels, truth)},
            # the reference ran on the dense K, so the iterations saved are taken against
            # the plain run on the same dense K
            "exact_iters_saved_fp32": (plain_dense["iters"] - ref["iters"]) if plain_dense else None,
            "exact_iters_saved_bf16": rcn["iters"] - r["iters"],
            "sweep_bf16": {"kernel": "packed_sweep<unsigned short>", "avg_ms": sw16,
                           "algorithmic_bytes": b16, "achieved_gbs": b16 / (sw16 * 1e-3) / 1e9,
                           "frac_hbm": b16 / (sw16 * 1e-3) / 1e9 / HBM_PEAK_GBS, "fold_ms": fold16},
            "gram_bf16_packed_ms": gp16,
            "dense_bf16": {"iter_ms": itd16, "sweep_ms": swd16,
                           "sweep_frac_hbm": float(n) * n * 2 / (swd16 * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "gram_bf16": {"avg_ms": g16, "achieved_tflops": gram_flops / (g16 * 1e-3) / 1e12,
                          "frac_mfma": gram_flops / (g16 * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFS},
            "training": train_rep,
            "kernel_kmeanspp_warm_start": kseeded,
        }
        if plain:
            # against the faster plain FP32 run (strip-packed K); the dense-K run beside it
            learned["speedup_time_to_converge"] = speedups(plain["seconds"], control_s, secs,
                                                           train_rep["seconds"])
        if plain_dense:
            learned["speedup_vs_plain_fp32_dense_k"] = plain_dense["seconds"] / secs
        log("mixed+learned: %.3f s (warm start %.3f s, %d cheap + %d exact iterations), ARI vs FP32 "
            "from same start %.4f; bf16 from random labels %.3f s (%d iterations)" % (
                secs, ws_s, ch, r["iters"], learned["ari_vs_fp32_from_same_warm_start"], control_s,
                rcn["iters"]))
        del K16, Kp16
    else:
        del K
    torch.cuda.empty_cache()
    small = None
    if not args.no_small:
        small = {"mnist_like": mnist_leg(kkm, torch, dev), "rings": rings_leg(kkm, torch, dev)}
    batched = None if args.no_batched else batched_leg(kkm, torch, dev, iters)
    learned_c5 = None if (args.no_learned or args.no_converge) else learned_c5_leg(kkm, torch, dev)
    matfree = None if args.no_matfree else matfree_leg(kkm, torch, dev)

    cpu = None
    same_prefix = None
    metric_20k = None
    if not args.no_cpu_baseline:
        rows = min(args.cpu_rows, n)
        cpu, K_or = cpu_baseline(w, rows, iters, full=args.cpu_full)
        same_prefix = gpu_same_prefix(kkm, torch, dev, w, rows, iters)
        cpu["gpu_same_rows"] = same_prefix
        if params is not None:
            metric_20k = metric_check_20k(kkm, torch, dev, w, rows, params, K_or, useed)
        del K_or

    out = {
        "metric": METRIC,
        "value": 1e3 / p_iter_ms,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": pwall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gmm200k: %d-component Gaussian mixture, sigma 0.5" % w.k,
                   "n": n, "d": w.d, "k": w.k, "kernel": "gaussian gamma=1/%d" % w.d,
                   "iterations_per_step": iters, "gram": "f32 mfma",
                   "k_store": "f32, strip-packed upper triangle (strips of 1024 columns)",
                   "parallelism": "single gpu"},
        "value_definition": "1 / median time of one reassignment step on the strip-packed FP32 K, "
                            "iterations 2..%d of the timed runs, Gram excluded" % iters,
        "iters_per_s_incl_gram": packed["iters_per_s_incl_gram"],
        "gram_ms": packed["gram_ms"],
        "iter_ms": p_iter_ms,
        "packed_fp32": packed,
        "dense_fp32": dense,
        "plain_fp32_to_convergence": plain,
        "plain_fp32_dense_to_convergence": plain_dense,
        "mixed_learned_to_convergence": learned,
        "metric_form_vs_oracle_20k": metric_20k,
        "mnist_like_60k": small and small["mnist_like"],
        "rings_1k": small and small["rings"],
        "batched": batched,
        "learned_warm_start_100k": learned_c5,
        "matfree_vs_stored_k_100k": matfree,
        "roofline": roof,
        "roofline_gram": roof_g,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
