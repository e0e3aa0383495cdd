"""Autotuner for the batched form: the sweep tile height of each problem.

Each sweep work item of a step covers chunk_rows consecutive rows of V's CSR
order (rows of K) by 1024 FP32 (2048 BF16) columns.  Short items give more
parallelism but write more partial sums (one row of n floats per cluster
segment of each item) and re-read them in the fused assignment; long items
write fewer partials but leave fewer items to spread over the GPU.  The best
height depends on n and k and on the element type of K, so it is measured:
for every (n, k) bucket a batch of equal synthetic problems is run through
kkm_fit_batched with each candidate height and the fastest per-step time
wins.

The table is keyed by the GPU's architecture name, the element type of K and
the bucket ("n<=2^a,k<=4^b"), and stored as JSON.  ``apply`` fills each
problem's chunk_rows from it (0, the library default, where no entry
exists).  Tuning changes only the summation order of the sweep, never the
method.

    python -m paper_2501_05587_amd.autotune --out table.json   # on the GPU
"""
import argparse
import json
import math
import os
import time

CANDIDATES = (16, 32, 64, 128, 256, 512, 1024, 2048, 4096)
TABLE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")


def arch(torch):
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def bucket(n: int, k: int):
    """(a, b) with 2^(a-1) < n <= 2^a (a >= 8) and 4^(b-1) < k <= 4^b (b >= 1)."""
    a = max(8, int(math.ceil(math.log2(max(n, 1)))))
    b = max(1, int(math.ceil(math.log(max(k, 1), 4) - 1e-12)))
    return a, b


def key(n: int, k: int) -> str:
    a, b = bucket(n, k)
    return "n<=2^%d,k<=4^%d" % (a, b)


def default_path(arch_name: str) -> str:
    return os.path.join(TABLE_DIR, "%s.json" % arch_name)


def load(path=None, torch=None):
    """The tuned table for this GPU ({} if there is none)."""
    if path is None:
        if torch is None:
            import torch
        path = default_path(arch(torch))
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def apply(problems, table, k_store=0):
    """Copies of the problem dicts with chunk_rows taken from the table."""
    sub = table.get("bf16" if k_store == 1 else "f32", {})
    out = []
    for p in problems:
        n, k = int(p["X"].shape[0]), int(p["k"])
        out.append(dict(p, chunk_rows=int(sub.get(key(n, k), {}).get("chunk_rows", 0))))
    return out


def _trial(kkm, torch, n, k, L, k_store, count, iters, gen):
    d = 32
    probs = []
    for _ in range(count):
        X = torch.randn(n, d, generator=gen, device="cuda", dtype=torch.float32)
        probs.append(dict(X=X, k=k, kernel=kkm.GAUSS, gamma=1.0 / d, chunk_rows=L))
    l0 = torch.randint(0, k, (n * count,), generator=gen, device="cuda", dtype=torch.int32)
    best = float("inf")
    for _ in range(2):
        r = kkm.kkm_fit_batched(probs, l0, gram_prec=kkm.BF16, k_store=k_store, max_iter=iters,
                                check_convergence=False, use_graph=True)
        best = min(best, r["times_ms"][1] / iters)
    return best


def tune_bucket(kkm, torch, a, b, k_store=0, iters=6, budget_bytes=6e9, seed=0):
    """Per-step milliseconds of every candidate for bucket (a, b) and the best
    chunk_rows.  The trial batch holds equal problems of n = 2^a points and
    k = min(4^b, n) clusters, enough of them to stream about budget_bytes of
    K per step."""
    n = 2 ** a
    k = min(4 ** b, n, 1024)
    es = 2 if k_store == 1 else 4
    count = int(max(1, min(512, budget_bytes // (n * n * es))))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed * 7919 + a * 31 + b)
    times = {}
    for L in CANDIDATES:
        if L > max(n, CANDIDATES[0]):
            break
        times[L] = _trial(kkm, torch, n, k, L, k_store, count, iters, gen)
    best = min(times, key=times.get)
    return {"chunk_rows": best, "ms_per_step": times[best], "problems": count, "n": n, "k": k,
            "candidates_ms": {str(L): t for L, t in times.items()}}


def tune(kkm, torch, buckets, k_store=0, log=print):
    sub = {}
    for a, b in sorted(set(buckets)):
        t = time.perf_counter()
        r = tune_bucket(kkm, torch, a, b, k_store)
        sub["n<=2^%d,k<=4^%d" % (a, b)] = r
        log("bucket n<=2^%d k<=4^%d: chunk_rows %d (%.3f ms/step, %d problems) in %.1f s" %
            (a, b, r["chunk_rows"], r["ms_per_step"], r["problems"], time.perf_counter() - t))
    return sub


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None, help="table path (default: tuned/<arch>.json)")
    ap.add_argument("--n-max", type=int, default=14, help="largest n bucket exponent")
    ap.add_argument("--k-max", type=int, default=3, help="largest k bucket exponent (4^b)")
    ap.add_argument("--k-store", default="f32", choices=("f32", "bf16"))
    args = ap.parse_args()
    import torch

    import paper_2501_05587_amd as kkm
    name = arch(torch)
    path = args.out or default_path(name)
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    ks = 1 if args.k_store == "bf16" else 0
    buckets = [(a, b) for a in range(8, args.n_max + 1) for b in range(1, args.k_max + 1)]
    table[args.k_store] = tune(kkm, torch, buckets, ks, log=lambda *x: print(*x, flush=True))
    table["arch"] = name
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
