#!/usr/bin/env python3
"""Benchmark: Kernel K-means on one MI355X, n=200000, d=1024, k=64.

Workload: a 64-component Gaussian mixture in R^1024 (means N(0,1), sigma 0.5),
Gaussian kernel gamma = 1/1024, random initial labels.

Plain FP32 leg (the timed steps behind `value`).  One step = one complete run
of the method on the resident input: the Gram kernel K = kappa(X X^T) (FP32
MFMA, K stored FP32, 160 GB) followed by 30 reassignment steps (V in CSR form,
SpMM row sweep of K, centroid norms, fused distance/argmin/histogram) and the
FP64 objective of the final labels: the paper's protocol of exactly 30
iterations.  `value` = iterations executed / timed wall time, Gram included.

Also reported:
* time-to-converge of the plain FP32 form from the random labels;
* the mixed + learned form: BF16 Gram with K stored BF16 (80 GB), a feature
  network trained beforehand on 10^7 kernel-value pairs of the same mixture
  (training time reported separately), k-means++ and Lloyd in feature space,
  then exact refinement to convergence; its time-to-converge and the ARI of its
  labels against the plain FP32 form converged from the same warm labels;
* roofline positions of the sweep (HBM) and the Gram (MFMA) from HIP-event
  timings of those launches, and HBM traffic from the recorded counters;
* the FP64 oracle timed on the host on a bounded prefix of the workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--rows N]
       [--no-cpu-baseline] [--no-converge] [--no-learned] [--copy-calibration]
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
    "spmm_row_sweep": {"sources": ["csrc/iterate.hip", "csrc/iterate.h", "csrc/kkm_common.h"],
                       "sha256": "5dfa764ff32bcad8404bb7b0d925b865fc7dfd0af7fedd260eee0ae69eda4208",
                       "n": 200000, "fetch_kib": 78169660.7, "write_kib": 85552.3,
                       "fetch_scale": 1.9999, "write_scale": 1.0},
    "gram_f32_mfma": {"sources": ["csrc/gram.hip", "csrc/gram_f32.hip", "csrc/gram_tile.h", "csrc/kkm_common.h"],
                      "sha256": "50f85bd9f32aa068be140202f556027e826462f5f6b4933083f3e8d392393e86",
                      "n": 200000, "fetch_kib": 160830564.2, "write_kib": 156250900.2,
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
    t = TRAFFIC[kernel]
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


def cpu_baseline(w, rows, iters):
    """The FP64 oracle on the first `rows` points: K from the definition and
    `iters` fixed steps; time scaled to the full n by (n/rows)^2 (both parts
    are O(n^2) at fixed d)."""
    import oracle
    X, _ = w.points(rows=rows)
    l0 = w.labels0(rows=rows)
    t0 = time.perf_counter()
    K = oracle.kernel_matrix(X, w.kernel, w.gamma, w.coef0, w.degree)
    t1 = time.perf_counter()
    oracle.fit(K, w.k, l0, iters, check_convergence=False)
    t2 = time.perf_counter()
    scale = (w.n / rows) ** 2
    full_s = (t2 - t0) * scale
    return {"value": iters / full_s, "unit": "iters/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "first %d of the %d points, %d fixed iterations: K %.2f s + loop %.2f s; "
                      "scaled by (n/%d)^2 = %.0f to the full workload" % (
                          rows, w.n, iters, t1 - t0, t2 - t1, rows, scale)}


def train_feature_map(kkm, torch, w, dev):
    """Train phi_theta on 10^7 kernel values of fresh draws of the same mixture:
    TRAIN_STEPS batches of TRAIN_BATCH new points, each batch's kernel values
    computed by the Gram kernel.  Returns (params, report)."""
    import datagen
    m = TRAIN_STEPS * TRAIN_BATCH
    means = datagen.gmm_means(w.d, w.k, w.data_seed)
    Xtr, _ = datagen.gmm(m, w.d, w.k, 0.5, w.data_seed + 30000, means=means)
    params = torch.from_numpy(datagen.mlp_init_params(w.d, H1, H2, OUT, w.data_seed + 30002)).to(dev)
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


def warm_labels(kkm, w, params, Xd, seed, streams=WARM_STREAMS):
    """phi_theta(X), then WARM_RESTARTS k-means++ seedings each followed by
    Lloyd in feature space; keeps the labelling with the lowest feature-space
    objective (the lowest restart index on ties).  Returns (labels, cheap
    iterations summed over restarts).  The restarts are independent; they run
    on `streams` HIP streams of default priority, one host thread each (the
    library calls release the interpreter lock), and each restart computes
    exactly what it computes alone."""
    import threading

    import torch

    import datagen
    F = kkm.kkm_mlp_forward(params, Xd, H1, H2, OUT)
    main = torch.cuda.current_stream()
    ready = torch.cuda.Event()
    ready.record(main)
    out = [None] * WARM_RESTARTS
    side = [torch.cuda.Stream() for _ in range(max(1, streams))]
    errors = []

    def worker(t):
        try:
            st = side[t]
            with torch.cuda.stream(st):
                st.wait_event(ready)
                for r in range(t, WARM_RESTARTS, len(side)):
                    _, seeded = kkm.kkm_feature_kmeanspp(F, w.k, datagen.uniforms(w.k, seed + r))
                    lab, it, _, obj = kkm.kkm_feature_lloyd(F, w.k, seeded, max_iter=WARM_MAX_ITER,
                                                            return_objective=True)
                    out[r] = (obj, it, lab)
        except Exception as e:  # re-raised on the calling thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(len(side))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    if errors:
        raise errors[0]
    for st in side:
        main.wait_stream(st)
    best = min(range(WARM_RESTARTS), key=lambda r: (out[r][0], r))
    lab = out[best][2]
    lab.record_stream(main)
    return lab, sum(o[1] for o in out)


def learned_c5_leg(kkm, torch, dev):
    """The learned warm start on its own workload: phi_theta trained on 10^7
    kernel values of the 32-component mixture in R^128, then fresh n=100000
    draws, k=32: plain FP32 from random labels against the BF16 form from the
    learned warm start, both to convergence, and the FP32 form converged from
    the same warm labels as the reference for the result (ARI)."""
    import numpy as np

    import datagen
    w = datagen.WORKLOADS["learned100k"]
    X, truth = w.points()
    Xd = torch.from_numpy(X).to(dev)
    ld = torch.from_numpy(w.labels0()).to(dev)
    n = w.n
    params, train_rep = train_feature_map(kkm, torch, w, dev)
    K = kkm.alloc_kernel_matrix(n, kkm.F32, dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)

    def plain_run():
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, max_iter=w.max_iter, check_convergence=True,
                           K_ws=K, labels_out=lab)
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    plain_run()
    pr = [plain_run() for _ in range(3)]
    plain_s = float(np.median([x[0] for x in pr]))
    rp = pr[-1][1]
    plain_labels = lab.cpu().numpy()
    useed = w.label_seed + 30003
    warm, _ = warm_labels(kkm, w, params, Xd, useed)
    ref = kkm.kkm_fit_ex(Xd, w.k, warm, w.kernel, w.gamma, max_iter=w.max_iter, check_convergence=True,
                         K_ws=K, labels_out=lab)
    ref_labels = lab.cpu().numpy()
    del K
    torch.cuda.empty_cache()
    K16 = kkm.alloc_kernel_matrix(n, kkm.BF16, dev)
    lab16 = torch.empty(n, dtype=torch.int32, device=dev)

    def learned_run():
        torch.cuda.synchronize()
        ta = time.perf_counter()
        wl, ch = warm_labels(kkm, w, params, Xd, useed)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        r = kkm.kkm_fit_ex(Xd, w.k, wl, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                           max_iter=w.max_iter, check_convergence=True, K_ws=K16, labels_out=lab16)
        torch.cuda.synchronize()
        return time.perf_counter() - ta, tb - ta, ch, r

    learned_run()
    lr = [learned_run() for _ in range(3)]
    secs = float(np.median([x[0] for x in lr]))
    _, _, ch, r = lr[-1]
    ml = lab16.cpu().numpy()
    del K16
    torch.cuda.empty_cache()
    rec = {
        "workload": "learned100k: fresh draws n=%d of the 32-component mixture in R^%d (sigma 0.5), "
                    "k=%d, gaussian gamma=1/%d" % (n, w.d, w.k, w.d),
        "training": train_rep,
        "plain_fp32": {"seconds": plain_s, "iters": rp["iters"], "objective": rp["objective"],
                       "gram_ms": rp["times_ms"][0], "ari_vs_truth": ari(plain_labels, truth)},
        "mixed_learned": {"seconds": secs, "warm_start_seconds": float(np.median([x[1] for x in lr])),
                          "cheap_iters": ch, "exact_iters": r["iters"], "objective": r["objective"],
                          "gram_ms": r["times_ms"][0], "ari_vs_truth": ari(ml, truth),
                          "ari_vs_fp32_from_same_warm_start": ari(ml, ref_labels)},
        "fp32_from_warm_start": {"iters": ref["iters"], "objective": ref["objective"]},
        "exact_iters_saved": rp["iters"] - r["iters"],
        "objective_rel_gap_vs_plain": (r["objective"] - rp["objective"]) / abs(rp["objective"]),
        "speedup_time_to_converge_vs_plain": plain_s / secs,
    }
    log("learned100k: plain %.3f s (%d iters, J %.2f), mixed+learned %.3f s (%d cheap + %d exact, J %.2f), "
        "ARI vs FP32 from same start %.4f" % (plain_s, rp["iters"], rp["objective"], secs, ch, r["iters"],
                                              r["objective"], rec["mixed_learned"]["ari_vs_fp32_from_same_warm_start"]))
    return rec


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
    ap.add_argument("--cpu-rows", type=int, default=24000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--learned-only", action="store_true",
                    help="run only the learned warm start on its n=100000, k=32 workload")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched form and print its record")
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

    if args.copy_calibration:
        copy_calibration()
        return
    if args.gram_shapes:
        print(json.dumps({"gram_shapes": gram_shapes(kkm, torch, torch.device("cuda:0"))}),
              flush=True)
        return
    if args.learned_only:
        print(json.dumps(learned_c5_leg(kkm, torch, torch.device("cuda:0"))), flush=True)
        return
    if args.batched_only:
        print(json.dumps(batched_leg(kkm, torch, torch.device("cuda:0"), args.iters or 30)),
              flush=True)
        return

    w = datagen.WORKLOADS["gmm200k"]
    n = args.rows or w.n
    iters = args.iters or w.max_iter
    log("workload %s: n=%d d=%d k=%d gamma=%g, %d iterations" % (w.name, n, w.d, w.k, w.gamma, iters))
    t = time.perf_counter()
    X, truth = w.points(rows=n)
    l0 = w.labels0(rows=n)
    log("data generated in %.1f s" % (time.perf_counter() - t))

    dev = torch.device("cuda:0")
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
    kkm.kkm_timing_enable(False)
    wall = t1 - t0
    total_iters = sum(r["iters"] for r in rs)
    gram_ms = float(np.mean([r["times_ms"][0] for r in rs]))
    iter_ms = float(np.mean([r["times_ms"][1] / max(r["iters"], 1) for r in rs]))

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

    # ------------------------------------------------------------ plain FP32 to convergence
    plain = None
    if not args.no_converge:
        torch.cuda.synchronize()
        tc = time.perf_counter()
        rc = kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, w.coef0, w.degree, max_iter=300,
                            check_convergence=True, K_ws=K, labels_out=lab)
        torch.cuda.synchronize()
        labs = lab.cpu().numpy()
        plain = {"seconds": time.perf_counter() - tc, "iters": rc["iters"], "objective": rc["objective"],
                 "gram_ms": rc["times_ms"][0], "iter_ms": rc["times_ms"][1] / max(rc["iters"], 1),
                 "ari_vs_truth": ari(labs, truth),
                 "empty_clusters": int((np.bincount(labs, minlength=w.k) == 0).sum())}
        log("plain converged: %d iterations in %.3f s, J=%.6f" % (rc["iters"], plain["seconds"],
                                                                  rc["objective"]))

    # ------------------------------------------------------------ mixed + learned
    learned = None
    if not args.no_learned and not args.no_converge:
        params, train_rep = train_feature_map(kkm, torch, w, dev)
        useed = w.label_seed + 30003
        # reference: the plain FP32 form converged from the same warm labels
        warm, cheap = warm_labels(kkm, w, params, Xd, useed)
        ref = kkm.kkm_fit_ex(Xd, w.k, warm, w.kernel, w.gamma, max_iter=300, check_convergence=True,
                             K_ws=K, labels_out=lab)
        ref_labels = lab.cpu().numpy()
        log("reference from warm labels: %d iterations, J=%.6f" % (ref["iters"], ref["objective"]))
        del K
        torch.cuda.empty_cache()
        K16 = kkm.alloc_kernel_matrix(n, kkm.BF16, dev)
        lab16 = torch.empty(n, dtype=torch.int32, device=dev)

        def mixed_learned():
            torch.cuda.synchronize()
            ta = time.perf_counter()
            wl, ch = warm_labels(kkm, w, params, Xd, useed)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            r = kkm.kkm_fit_ex(Xd, w.k, wl, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                               max_iter=300, check_convergence=True, K_ws=K16, labels_out=lab16)
            torch.cuda.synchronize()
            return time.perf_counter() - ta, tb - ta, ch, r

        def kernel_seeded():
            # the non-learned warm start: k-means++ on the exact kernel matrix
            torch.cuda.synchronize()
            ta = time.perf_counter()
            Kg, dg = kkm.kkm_gram(Xd, w.kernel, w.gamma, w.coef0, w.degree, gram_prec=kkm.BF16,
                                  k_store=kkm.BF16, K=K16)
            _, lab0 = kkm.kkm_kernel_kmeanspp(Kg, dg, w.k, datagen.uniforms(w.k, useed))
            torch.cuda.synchronize()
            tb = time.perf_counter()
            r = kkm.kkm_refine(Kg, dg, w.k, lab0, max_iter=300, labels_out=lab16)
            torch.cuda.synchronize()
            return time.perf_counter() - ta, tb - ta, r

        kernel_seeded()
        kruns = [kernel_seeded() for _ in range(3)]
        ks_secs = float(np.median([x[0] for x in kruns]))
        _, _, kr = kruns[-1]
        ks_labels = lab16.cpu().numpy()
        kseeded = {"seconds": ks_secs, "gram_and_seeding_seconds": float(np.median([x[1] for x in kruns])),
                   "exact_iters": kr["iters"], "objective": kr["objective"],
                   "ari_vs_truth": ari(ks_labels, truth),
                   "empty_clusters": int((np.bincount(ks_labels, minlength=w.k) == 0).sum())}
        log("kernel k-means++ + exact: %.3f s (Gram + seeding %.3f s, %d exact iterations), J=%.3f" % (
            ks_secs, kseeded["gram_and_seeding_seconds"], kr["iters"], kr["objective"]))

        mixed_learned()  # warm-up of the whole leg
        runs = [mixed_learned() for _ in range(3)]
        secs = float(np.median([x[0] for x in runs]))
        _, _, ch, r = runs[-1]
        ml_labels = lab16.cpu().numpy()
        # per-iteration rate of the mixed form: 30 fixed iterations on the BF16 K
        kkm.kkm_timing_enable(True)
        rf = kkm.kkm_fit_ex(Xd, w.k, ld, w.kernel, w.gamma, gram_prec=kkm.BF16, k_store=kkm.BF16,
                            max_iter=iters, check_convergence=False, K_ws=K16, labels_out=lab16)
        torch.cuda.synchronize()
        tim16 = kkm.kkm_timing_read()
        kkm.kkm_timing_enable(False)
        sw16 = tim16["sweep"][0] / max(tim16["sweep"][1], 1)
        g16 = tim16["gram"][0] / max(tim16["gram"][1], 1)
        learned = {
            "seconds": secs, "warm_start_seconds": float(np.median([x[1] for x in runs])),
            "cheap_iters": ch, "exact_iters": r["iters"], "objective": r["objective"],
            "gram": "bf16 mfma", "k_store": "bf16", "gram_ms": r["times_ms"][0],
            "iter_ms": rf["times_ms"][1] / max(rf["iters"], 1),
            "iters_per_s": rf["iters"] / (rf["times_ms"][1] * 1e-3),
            "ari_vs_fp32_from_same_warm_start": ari(ml_labels, ref_labels),
            "ari_vs_truth": ari(ml_labels, truth),
            "empty_clusters": int((np.bincount(ml_labels, minlength=w.k) == 0).sum()),
            "fp32_from_warm_start": {"iters": ref["iters"], "objective": ref["objective"]},
            "sweep_bf16": {"avg_ms": sw16, "achieved_gbs": float(n) * n * 2 / (sw16 * 1e-3) / 1e9,
                           "frac_hbm": float(n) * n * 2 / (sw16 * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "gram_bf16": {"avg_ms": g16, "achieved_tflops": gram_flops / (g16 * 1e-3) / 1e12,
                          "frac_mfma": gram_flops / (g16 * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFS},
            "training": train_rep,
            "kernel_kmeanspp_warm_start": kseeded,
        }
        if plain:
            learned["speedup_time_to_converge_vs_plain"] = plain["seconds"] / secs
        log("mixed+learned: %.3f s (warm start %.3f s, %d cheap + %d exact iterations), ARI vs FP32 "
            "from same start %.4f" % (secs, learned["warm_start_seconds"], ch, r["iters"],
                                       learned["ari_vs_fp32_from_same_warm_start"]))
        del K16
    else:
        del K
    torch.cuda.empty_cache()
    batched = None if args.no_batched else batched_leg(kkm, torch, dev, iters)
    learned_c5 = None if (args.no_learned or args.no_converge) else learned_c5_leg(kkm, torch, dev)

    out = {
        "metric": METRIC,
        "value": total_iters / wall,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gmm200k: %d-component Gaussian mixture, sigma 0.5" % w.k,
                   "n": n, "d": w.d, "k": w.k, "kernel": "gaussian gamma=1/%d" % w.d,
                   "iterations_per_step": iters, "gram": "f32 mfma", "k_store": "f32",
                   "parallelism": "single gpu"},
        "gram_ms": gram_ms,
        "iter_ms": iter_ms,
        "plain_fp32_to_convergence": plain,
        "mixed_learned_to_convergence": learned,
        "batched": batched,
        "learned_warm_start_100k": learned_c5,
        "roofline": roof,
        "roofline_gram": roof_g,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, min(args.cpu_rows, n), iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
