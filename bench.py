#!/usr/bin/env python3
"""ProHD vs exact Hausdorff distance on one MI355X: set-pairs per second.

Workload (default ``heavy2m``): A and B each 2 000 000 x 256 float32, a
128-cluster Gaussian mixture with 0.1 % Student-t(3) outliers per set
(seeded, synthetic), ProHD at the paper's defaults alpha = 0.01 and
m = floor(sqrt(256)) = 16 (k = 20 000 per end on the centroid axis, 1 250 per
end on each principal component).

One step = the whole ProHD path on the device: prohd_project (sums + float64
Gram + eigensolve + projections), prohd_select (per-direction extremes,
union) and prohd_hd (candidate distance, pruned search with refinement),
inputs resident in HBM.  ``value`` is ProHD set-pairs/s over the timed
steps (eager launches; the same step captured once as a HIP graph and
replayed is timed and checked beside it, as is the step with the unpruned
search), and the exact distance (exact_hd) of the same pair is timed after
it (``exact``).
``roofline`` is for the kernel with the most time per step, timed with HIP
events on the stream it runs on; ``path_roofline`` in the detail file rates
the step's other kernels.  ``cpu_baseline`` times the FP64 oracle on a
bounded sample of the same workload and scales it to the full pair.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HD set-pairs/sec at 2M×2M D=256 (ProHD vs exact); rel. err vs FP64 oracle"
PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0        # GB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _source_block(src, start):
    """Text from the line holding `start` (and its template line) to the
    closing brace of that function."""
    i = src.index(start)
    i = src.rfind("\ntemplate", 0, i) if src.rfind("\ntemplate", 0, i) > src.rfind("\n}\n", 0, i) else src.rfind("\n", 0, i)
    j = src.index("\n}\n", i) + 3
    return src[i:j]


# source blocks (file, first line) of each measured kernel and of the host
# code that picks its launch shape
KERNEL_SOURCES = {
    "hd_tile": ("k_hd.hip", ("void dist_seg(", "int64_t tile_split(", "void tile_schedule(",
                             "void dist_tile(", "int64_t tile_grid(", "prohd_status launch_tile_k(",
                             "prohd_status launch_tile(")),
    "stats_gram": ("k_stats.hip", ("void g256_mul(", "void g256_slice(", "void gram_partial256(",
                                   "StatsLayout stats_layout(", "prohd_status stats_dp(")),
}


def kernel_source_hash(kernel="hd_tile"):
    """Hash of a kernel's source and of the host code that picks its launch
    shape: a counter summary is valid while this is unchanged."""
    fname, starts = KERNEL_SOURCES[kernel]
    with open(os.path.join(ROOT, "paper_2511_18207_amd", "csrc", fname)) as fh:
        src = fh.read()
    h = hashlib.sha256()
    for start in starts:
        h.update(_source_block(src, start).encode())
    return h.hexdigest()[:16]


def load_traffic(name, kernel):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or
    None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash(kernel):
        return None
    return d.get("bytes_per_launch")


def attainable_peaks(dev):
    """Rates this GPU reaches on plain library work, as a yardstick beside the
    datasheet peaks: square float32 and float64 products through torch
    (hipBLASLt / rocBLAS), a 4 GiB read-only reduction and a 2 GiB copy."""
    import torch

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    for name, dt, n in (("gemm_fp32_tflops", torch.float32, 8192), ("gemm_fp64_tflops", torch.float64, 8192)):
        a = torch.randn(n, n, device=dev, dtype=dt)
        b = torch.randn(n, n, device=dev, dtype=dt)
        ms = timed(lambda: torch.matmul(a, b), 5)
        out[name] = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
        del a, b
    x = torch.ones(1 << 30, device=dev, dtype=torch.float32)
    ms = timed(lambda: x.sum(), 10)
    out["hbm_read_gbs"] = 4.0 * (1 << 30) / (ms * 1e-3) / 1e9
    y = torch.empty(1 << 29, device=dev, dtype=torch.float32)
    ms = timed(lambda: y.copy_(x[: 1 << 29]), 10)
    out["hbm_copy_gbs"] = 2 * 4.0 * (1 << 29) / (ms * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return out


def cpu_baseline(A, B, m, alpha, n_sample):
    """FP64 oracle on the first n_sample rows of each set, phases timed; the
    linear phases scale with n, the candidate distance with n^2."""
    import numpy as np

    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
    a, b = A[:n_sample], B[:n_sample]
    t0 = time.perf_counter()
    u0 = oracle.centroid_direction(a, b)
    P, _ = oracle.principal_directions(a, b, m)
    U = np.vstack([u0[None, :], P])
    pa = U @ a.astype(np.float64).T
    pb = U @ b.astype(np.float64).T
    kA = [oracle.k_rule(alpha, a.shape[0])] + [oracle.k_rule(alpha / m, a.shape[0])] * m
    kB = [oracle.k_rule(alpha, b.shape[0])] + [oracle.k_rule(alpha / m, b.shape[0])] * m
    IA, IB = oracle.select(pa, pb, kA, kB)
    t1 = time.perf_counter()
    oracle.subset_hd(a, b, IA, IB)
    t2 = time.perf_counter()
    f = A.shape[0] / n_sample
    est = (t1 - t0) * f + (t2 - t1) * f * f
    return {
        "value": 1.0 / est, "unit": "set-pairs/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"first {n_sample} rows of each set of the same workload, FP64 oracle ProHD "
                   f"(alpha={alpha}, m={m}); directions+projection+selection took "
                   f"{t1 - t0:.2f} s (scaled x{f:g}), candidate distance {t2 - t1:.2f} s "
                   f"(|I|={IA.size}/{IB.size}, scaled x{f * f:g}); estimated {est:.1f} s per full pair"),
    }


LEARNED_LAW = {"K": 128, "centre_seed": 77, "D": 256}


def learned_form(args, dev, nu):
    """Learned proposal: train the scorer on pairs of one Student-t mixture
    (fixed centres, new samples per pair), then compare ProHD + top-scored
    points with plain ProHD at an equal candidate budget on held-out pairs,
    exact HD as judge."""
    import numpy as np
    import torch

    import paper_2511_18207_amd as ph
    import synth
    from paper_2511_18207_amd import learned as LN

    n, D = args.learned_n, LEARNED_LAW["D"]

    def draw(seed):
        A, B = synth.t_mixture(n, n, D, seed, K=LEARNED_LAW["K"], nu=nu,
                               centre_seed=LEARNED_LAW["centre_seed"])
        return torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)

    ws = ph.Workspace(dev)
    t0 = time.perf_counter()
    pairs = []
    label_ms = 0.0
    for i in range(args.learned_pairs):
        dA, dB = draw(10_000 + i)
        torch.cuda.synchronize()
        l0 = time.perf_counter()
        pairs.append(LN.TrainPair(dA, dB, ws=ws))
        torch.cuda.synchronize()
        label_ms += 1e3 * (time.perf_counter() - l0)
    log(f"learned[nu={nu:g}]: {len(pairs)} training pairs {n}x{n} labelled in {label_ms:.0f} ms "
        f"(total {time.perf_counter() - t0:.1f}s)")
    sc = LN.Scorer(D, seed=1)
    batch = 16384
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = LN.train(sc, pairs, args.learned_steps, batch=batch, lr=2e-3, lr_final=1e-4,
                      pos_share=0.5, seed=0, ws=ws)
    torch.cuda.synchronize()
    train_ms = 1e3 * (time.perf_counter() - t1)
    # training step FLOPs: forward 2 n (2D*256 + 256*128 + 128), backward about twice that
    fwd_flops = 2.0 * (2 * D * 256 + 256 * 128 + 128)
    log(f"learned[nu={nu:g}]: {args.learned_steps} steps in {train_ms:.0f} ms, loss {losses[:50].mean():.4f} -> "
        f"{losses[-100:].mean():.4f}")
    del pairs
    torch.cuda.empty_cache()

    evals = []
    e = torch.cuda.Event
    for i in range(args.learned_eval):
        dA, dB = draw(20_000 + i)
        H = ph.decode_result(ph.exact_hd(dA, dB, ws=ws))["H"]
        rep = LN.equal_budget(dA, dB, sc, alpha=0.01, H=H, ws=ws)
        # time plain ProHD and the learned form (score both sets, merge, hd)
        base = ph.prohd(dA, dB, alpha=0.01, inner_full=False, ws=ws)
        e0, e1, e2 = e(enable_timing=True), e(enable_timing=True), e(enable_timing=True)
        e0.record()
        ph.prohd(dA, dB, alpha=0.01, ws=ws)
        e1.record()
        LN.proposal(dA, dB, sc, alpha=0.01, ws=ws, base=base)
        e2.record()
        torch.cuda.synchronize()
        rep["prohd_ms"] = e0.elapsed_time(e1)
        rep["learned_extra_ms"] = e1.elapsed_time(e2)
        evals.append(rep)
        log(f"learned[nu={nu:g}] eval {i}: H={H:.5f} full err prohd {rep['full']['prohd_err']:.3e} learned "
            f"{rep['full']['learned_err']:.3e} plain {rep['full']['plain_err']:.3e} | candidates "
            f"prohd {rep['candidates']['prohd_err']:.3e} learned {rep['candidates']['learned_err']:.3e} "
            f"plain {rep['candidates']['plain_err']:.3e}")
    # scoring throughput on one set
    X = dA
    cB = ph.centroid(dB, ws=ws)
    sc.score(X, cB, ws=ws)
    e0, e1 = e(enable_timing=True), e(enable_timing=True)
    e0.record()
    for _ in range(5):
        sc.score(X, cB, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    score_ms = e0.elapsed_time(e1) / 5

    def mean(mode, key):
        return float(np.mean([r[mode][key] for r in evals]))

    return {
        "law": f"Student-t({nu:g}) mixture, {LEARNED_LAW['K']} clusters, D={D}, "
               "centres N(0,4I) fixed across pairs, B centres + N(0,0.25I)",
        "train": {"pairs": args.learned_pairs, "n_per_set": n, "points": 2 * n * args.learned_pairs,
                  "label_frac": LN.LABEL_FRAC, "label_ms": label_ms, "steps": args.learned_steps,
                  "batch": batch, "train_ms": train_ms,
                  "ms_per_step": train_ms / args.learned_steps,
                  "loss_first": float(losses[:50].mean()), "loss_last": float(losses[-100:].mean())},
        "score": {"rows": int(X.shape[0]), "ms": score_ms,
                  "tflops": X.shape[0] * fwd_flops / (score_ms * 1e-3) / 1e12},
        "eval": evals,
        "mean_rel_err": {mode: {k: mean(mode, k + "_err") for k in ("prohd", "learned", "plain")}
                         for mode in ("candidates", "full")},
    }


def batched_form(args, dev):
    """Many uneven pairs: batch_sizes(P, 0) (log-uniform 256..65 536 per set,
    D in {64, 128, 256}), each pair the gauss_outliers law; ProHD (alpha 0.01,
    m = floor(sqrt D)) and the exact distance per pair, each one graph launch
    of persistent kernels with tuned work shapes."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import oracle
    import paper_2511_18207_amd as ph
    import synth

    P = args.batched_pairs
    nA, nB, D = synth.batch_sizes(P, 0)
    plan = ph.BatchPlan(nA, nB, D, alpha=0.01)
    t0 = time.perf_counter()
    hA = np.empty(int(plan.offA[-1]), dtype=np.float32)
    hB = np.empty(int(plan.offB[-1]), dtype=np.float32)

    def gen(i):
        a, b = synth.batch_pair(0, i, nA[i], nB[i], D[i])
        hA[plan.offA[i]:plan.offA[i + 1]] = a.ravel()
        hB[plan.offB[i]:plan.offB[i + 1]] = b.ravel()

    with ThreadPoolExecutor(16) as ex:
        list(ex.map(gen, range(P)))
    dA = torch.from_numpy(hA).to(dev)
    dB = torch.from_numpy(hB).to(dev)
    torch.cuda.synchronize()
    log(f"batched: {P} pairs, {(hA.size + hB.size) * 4 / 1e9:.1f} GB generated and copied in "
        f"{time.perf_counter() - t0:.1f}s")
    ws = ph.Workspace(dev)
    out = torch.zeros((P, ph.RESULT_BYTES), dtype=torch.uint8, device=dev)
    res = {}
    ev = torch.cuda.Event
    for mode, reps in (("prohd", 5), ("exact", 2)):
        t1 = time.perf_counter()
        plan.tune(dA, dB, mode=mode, out=out, ws=ws)
        tune_s = time.perf_counter() - t1
        plan.run(dA, dB, mode=mode, out=out, ws=ws)   # builds tables, captures the graph
        torch.cuda.synchronize()
        e0, e1 = ev(enable_timing=True), ev(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.run(dA, dB, mode=mode, out=out, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        results = plan.results(out)
        # kernel breakdown of one eager run
        ph.profile_reset()
        ph.profile_enable(True)
        plan.run(dA, dB, mode=mode, out=out, ws=ws, eager=True)
        torch.cuda.synchronize()
        ph.profile_enable(False)
        kern = {}
        for name in ("batch_gram", "batch_gram_reduce", "batch_eig", "batch_project",
                     "batch_select", "batch_compact", "batch_prep", "batch_tile", "batch_refine",
                     "batch_finalize", "batch_fill"):
            n, tot = ph.profile_read(name)
            if n:
                kern[name] = {"launches": n, "ms": tot}
        ph.profile_reset()
        res[mode] = {"ms": ms, "pairs_per_s": P * 1e3 / ms, "tune_s": tune_s, "kernels": kern,
                     "status_nonzero": int(sum(r["status"] != 0 for r in results)),
                     "H_sum": float(sum(r["H"] for r in results)), "_results": results}
        log(f"batched {mode}: {ms:.2f} ms per batch of {P} ({P * 1e3 / ms:.0f} pairs/s), tuned in {tune_s:.1f}s")
    # rooflines: covariance (FP64 matrix), distance tile (FP32 matrix), projection (HBM)
    rows = (nA + nB).astype(np.float64)
    Df = D.astype(np.float64)
    gram_flops = float((rows * Df * (Df + 1)).sum())   # the symmetric half, as the single pair
    # exact mode: pairs with both sets >= 16384 rows take the pruned
    # single-pair search; the batched tile searches the others in full
    pruned = np.array([ph.prune_levels(int(a), int(b)) > 0 for a, b in zip(nA, nB)])
    tile_flops = float((2.0 * nA * nB * Df)[~pruned].sum())
    proj_bytes = float((rows * Df * 4 + rows * (np.floor(np.sqrt(Df)) + 1) * 4).sum())
    kp, kx = res["prohd"]["kernels"], res["exact"]["kernels"]
    roof = {}
    if "batch_gram" in kp:
        a = gram_flops / (kp["batch_gram"]["ms"] * 1e-3) / 1e12
        roof["batch_gram"] = {"bound": "mfma", "achieved": a, "peak": 78.6, "unit": "TFLOP/s", "frac": a / 78.6}
    if "batch_project" in kp:
        a = proj_bytes / (kp["batch_project"]["ms"] * 1e-3) / 1e9
        roof["batch_project"] = {"bound": "hbm", "achieved": a, "peak": 8000.0, "unit": "GB/s", "frac": a / 8000.0}
    if "batch_tile" in kx:
        a = tile_flops / (kx["batch_tile"]["ms"] * 1e-3) / 1e12
        roof["batch_tile_exact"] = {"bound": "mfma", "achieved": a, "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
                                    "frac": a / PEAK_FP32_MFMA}
    # sampled parity: a few pairs against the oracle
    rp, rx = res["prohd"].pop("_results"), res["exact"].pop("_results")
    work = nA.astype(np.int64) * nB * D
    order = np.argsort(work)
    # the smallest pairs, two from the middle, and the pair with the most work
    sample = [int(i) for i in order[[0, 1, P // 4, P // 2, P - 1]]]
    checks = []
    for i in sample:
        a = hA[plan.offA[i]:plan.offA[i + 1]].reshape(int(nA[i]), int(D[i]))
        b = hB[plan.offB[i]:plan.offB[i + 1]].reshape(int(nB[i]), int(D[i]))
        m = int(np.floor(np.sqrt(D[i]) + 1e-9))
        wp = oracle.prohd(a, b, alpha=0.01, m=m)["H"]
        we = oracle.exact_hd(a, b, one_pass=True)["H"]
        checks.append({"pair": i, "nA": int(nA[i]), "nB": int(nB[i]), "D": int(D[i]),
                       "prohd_rel_err": abs(rp[i]["H"] - wp) / wp, "exact_rel_err": abs(rx[i]["H"] - we) / we})
    errs = np.array([abs(p_["H"] - x_["H"]) / x_["H"] for p_, x_ in zip(rp, rx) if x_["H"] > 0])
    plan.close()
    return {
        "workload": f"{P} pairs, sizes log-uniform 256..65536 per set, D in (64, 128, 256), "
                    "gauss_outliers law per pair, alpha 0.01, m = floor(sqrt D)",
        "points": int((nA + nB).sum()), "gbytes": (hA.size + hB.size) * 4 / 1e9,
        "prohd": res["prohd"], "exact": res["exact"], "roofline": roof,
        "algorithmic": {"gram_flops": gram_flops, "tile_flops_exact": tile_flops, "project_bytes": proj_bytes,
                        "exact_pairs_pruned_search": int(pruned.sum())},
        "prohd_vs_exact_rel_err": {"mean": float(errs.mean()), "max": float(errs.max()),
                                   "median": float(np.median(errs))},
        "sampled_oracle_check": checks,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--exact-steps", type=int, default=3)
    ap.add_argument("--workload", default="heavy2m")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exact", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-pairs", type=int, default=10)
    ap.add_argument("--learned-eval", type=int, default=4)
    ap.add_argument("--learned-n", type=int, default=500_000)
    ap.add_argument("--learned-steps", type=int, default=3000)
    ap.add_argument("--learned-nu", type=float, nargs="+", default=[30.0, 3.0])
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--batched-pairs", type=int, default=4096)
    ap.add_argument("--detail-out", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file for the full results (empty: stderr only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy first (HBM-counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU sharding is a design, not built", file=sys.stderr, flush=True)
        return 2

    import numpy as np
    import torch

    import paper_2511_18207_amd as ph
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ph.lib()

    t0 = time.perf_counter()
    A, B, params = synth.workload(args.workload, seed=args.seed)
    log(f"generated {args.workload} {A.shape} {B.shape} in {time.perf_counter() - t0:.1f}s")
    nA, D = A.shape
    nB = B.shape[0]
    m = params["m"]
    if "k" in params:
        kA = kB = [params["k"]] * (m + 1)
        alpha = None
    else:
        alpha = params["alpha"]
        kA = ph.alpha_k(alpha, nA, m)
        kB = ph.alpha_k(alpha, nB, m)
    dA = torch.from_numpy(A).to(dev)
    dB = torch.from_numpy(B).to(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    capA = int(min(nA, 2 * sum(min(k, nA) for k in kA)))
    capB = int(min(nB, 2 * sum(min(k, nB) for k in kB)))
    ws = ph.Workspace(dev)
    ws.get(ph.workspace_size(nA, nB, D, m + 1, capA, capB))
    out = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)

    def step(prune=True):
        _, pA, pB, _, _ = ph.prohd_project(dA, dB, m, ws=ws, evals=False)
        iA, cA, iB, cB = ph.prohd_select(pA, pB, kA, kB, capA=capA, capB=capB, ws=ws)
        ph.prohd_hd(dA, dB, iA, cA, iB, cB, capA=capA, capB=capB, ws=ws, out=out, prune=prune)
        return iA, cA, iB, cB

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    def timed(fn, reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, (time.perf_counter() - t0) / reps, r

    # eager launches (the headline), then the same steps with per-launch HIP
    # events (the per-kernel times of the rooflines), then the step captured
    # once as a HIP graph and replayed (reported beside it: the host keeps
    # ahead of the GPU, so the graph removes no gaps here)
    eager_ms, eager_wall, (iA, cA, iB, cB) = timed(step, args.steps)
    res = ph.decode_result(out)
    ph.profile_reset()
    ph.profile_enable(True)
    prof_ms, _, _ = timed(step, args.steps)
    ph.profile_enable(False)
    graph_ms = None
    graph_same = None
    try:
        gout = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)
        out_keep, out = out, gout
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        out = out_keep
        for _ in range(args.warmup):
            g.replay()
        graph_ms, graph_wall, _ = timed(g.replay, args.steps)
        gres = ph.decode_result(gout)
        graph_same = all(gres[k] == res[k] for k in ("H", "hAB", "hBA", "ab_a", "ab_b", "ba_b", "ba_a",
                                                     "nA_sel", "nB_sel", "status"))
    except Exception as exc:   # capture refused: report the eager figure
        out = out_keep
        log(f"graph capture failed: {exc}")
    use_graph = False
    ms_step = eager_ms
    wall = eager_wall
    log(f"step: eager {eager_ms:.3f} ms, with per-launch events {prof_ms:.3f} ms, graph replay "
        f"{graph_ms if graph_ms is None else round(graph_ms, 3)} ms (same result: {graph_same})")
    kernels = {}
    for name in ("stats_gram", "stats_reduce", "eig", "project_mfma", "select_", "compact_",
                 "hd_prep", "hd_subset", "hd_gather", "hd_tile", "hd_tile_rows", "hd_tile_gx", "hd_keys",
                 "hd_refine", "hd_dyn_refine", "hd_uncertain", "hd_finalize"):
        n, tot = ph.profile_read(name)
        if n:
            kernels[name] = {"launches_per_step": n / args.steps, "ms_per_step": tot / args.steps}
    ph.profile_reset()
    log(f"ProHD {ms_step:.3f} ms/step (wall {1e3 * wall:.3f}), H={res['H']:.6f} "
        f"|I|={res['nA_sel']}/{res['nB_sel']}")

    # the same step with the unpruned distance search (same result), for
    # comparison
    uout = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)
    out_keep, out = out, uout
    step(prune=False)
    torch.cuda.synchronize()
    u0, u1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    u0.record()
    for _ in range(3):
        step(prune=False)
    u1.record()
    torch.cuda.synchronize()
    out = out_keep
    ures = ph.decode_result(uout)
    unpruned = {"ms_per_step": u0.elapsed_time(u1) / 3, "H": ures["H"],
                "same_result": all(ures[k] == res[k] for k in ("H", "hAB", "hBA", "ab_a", "ab_b",
                                                               "ba_b", "ba_a"))}
    log(f"unpruned step {unpruned['ms_per_step']:.3f} ms, same result: {unpruned['same_result']}")

    # sampled parity at full size: the witness pair and 32 random candidate
    # rows re-measured in float64 on the host against all of B_sel
    IA = iA[: int(cA.item())].cpu().numpy()
    IB = iB[: int(cB.item())].cpu().numpy()
    Bs = B[IB].astype(np.float64)
    g = np.random.default_rng(1)
    sample = np.concatenate([[res["ab_a"]], g.choice(IA, size=min(32, IA.size), replace=False)])
    nn = np.array([np.sqrt(((Bs - A[i].astype(np.float64)) ** 2).sum(1)).min() for i in sample])
    check = {
        "witness_nn_rel_err": float(abs(nn[0] - res["hAB"]) / res["hAB"]),
        "sampled_rows_within_hAB": bool(np.all(nn <= res["hAB"] * (1 + 1e-6))),
        "sampled_rows": int(sample.size),
    }

    # per-kernel rooflines of the step: algorithmic work per launch (stated
    # per kernel) over the launch's average time from the HIP events; the
    # kernel with the most time per step is the headline roofline
    def per_step(name):
        k = kernels.get(name)
        return k["ms_per_step"] if k else None

    def avg_ms(name):
        k = kernels[name]
        return k["ms_per_step"] / k["launches_per_step"]

    def entry(kernel, bound, work, ms, peak, unit, launches):
        scale = 1e12 if unit == "TFLOP/s" else 1e9
        ach = work / (ms * 1e-3) / scale
        key = "algorithmic_flops" if unit == "TFLOP/s" else "algorithmic_bytes"
        return {"kernel": kernel, "bound": bound, "achieved": ach, "peak": peak, "unit": unit,
                "frac": ach / peak, "avg_ms": ms, key: work, "launches_per_step": launches}

    nAs, nBs = res["nA_sel"], res["nB_sel"]
    lev = ph.prune_levels(nA, nB, capA, capB)
    path_roof = {}
    if "stats_gram" in kernels:
        # the symmetric half of the union Gram: (nA + nB) D (D + 1) FP64 flops
        path_roof["stats_gram"] = entry(
            "gram_partial256 (covariance of the union, float64 v_mfma_f64_16x16x4f64)", "mfma",
            float(nA + nB) * D * (D + 1), avg_ms("stats_gram"), 78.6, "TFLOP/s", 1)
    if lev and "hd_tile_rows" in kernels:
        # first pruning level: every candidate row against every F-th row of
        # the other list, 2 D flops per pair, both directions (one launch,
        # or one per direction)
        F = 16 ** lev
        nl = kernels["hd_tile_rows"]["launches_per_step"]
        tf = 2.0 * D * (nAs * math.ceil(nBs / F) + nBs * math.ceil(nAs / F)) / nl
        path_roof["hd_tile"] = entry(
            f"dist_tile, first pruning level (F = {F}, float32 v_mfma_f32_32x32x2f32)", "mfma", tf,
            avg_ms("hd_tile_rows"), PEAK_FP32_MFMA, "TFLOP/s", nl)
    elif not lev and "hd_tile" in kernels:
        path_roof["hd_tile"] = entry(
            "dist_tile (candidate distance, float32 v_mfma_f32_32x32x2f32)", "mfma",
            2.0 * nAs * nBs * D, avg_ms("hd_tile"), PEAK_FP32_MFMA, "TFLOP/s", 1)
    if "project_mfma" in kernels:
        # one read of both sets plus the projection writes
        path_roof["project"] = entry("project_mfma", "hbm", float(nA + nB) * 4 * (D + m + 1),
                                     avg_ms("project_mfma"), PEAK_HBM, "GB/s", 1)
    if "select_" in kernels:
        sb = float(nA + nB) * 4 * (m + 1)
        path_roof["select"] = entry("selection passes (whole chain)", "hbm", sb, per_step("select_"),
                                    PEAK_HBM, "GB/s", kernels["select_"]["launches_per_step"])
    if "hd_refine" in kernels:
        # 256 rows per direction against the other list, 2 D FP64 flops per pair
        rf = 2.0 * D * 256 * (nAs + nBs) / 2
        path_roof["refine"] = entry("refine_rows (first pass, float64 v_mfma_f64_16x16x4f64)", "mfma",
                                    rf, avg_ms("hd_refine"), 78.6, "TFLOP/s", 2)
    dom = max(path_roof, key=lambda k: path_roof[k]["avg_ms"] * path_roof[k]["launches_per_step"])
    roof = dict(path_roof[dom])
    roof["name"] = dom
    roof["traffic"] = load_traffic(f"{dom}_{args.workload}_counters", dom) \
        if dom in KERNEL_SOURCES else None
    roof["share_of_step"] = roof["avg_ms"] * roof["launches_per_step"] / ms_step
    peaks = None
    if not args.no_peaks:
        peaks = attainable_peaks(dev)
        log("attainable: " + ", ".join(f"{k} {v:.1f}" for k, v in peaks.items()))
        att = {"stats_gram": peaks["gemm_fp64_tflops"], "refine": peaks["gemm_fp64_tflops"],
               "hd_tile": peaks["gemm_fp32_tflops"],
               "project": max(peaks["hbm_read_gbs"], peaks["hbm_copy_gbs"]),
               "select": max(peaks["hbm_read_gbs"], peaks["hbm_copy_gbs"])}
        for k, v in path_roof.items():
            v["frac_of_attainable"] = v["achieved"] / att[k]
        roof["frac_of_attainable"] = roof["achieved"] / att[dom]

    # error certificate (Sec. II-E bounds) of this step's directions and
    # projections, with the inner-minimum-over-the-full-set value as the
    # lower bound
    dirs_c, pA_c, pB_c, _, _ = ph.prohd_project(dA, dB, m, ws=ws, evals=False)
    iA_c, cA_c, iB_c, cB_c = ph.prohd_select(pA_c, pB_c, kA, kB, capA=capA, capB=capB, ws=ws)
    full_out = ph.prohd_hd(dA, dB, iA_c, cA_c, iB_c, cB_c, capA=capA, capB=capB, ws=ws, inner_full=True)
    cws = ph.Workspace(dev)
    ph.certificate(dA, dB, dirs_c, pA_c, pB_c, lower=full_out, ws=cws)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    cert = ph.certificate(dA, dB, dirs_c, pA_c, pB_c, lower=full_out, ws=cws)
    c1.record()
    torch.cuda.synchronize()
    cert["ms"] = c0.elapsed_time(c1)
    ph.profile_reset()
    ph.profile_enable(True)
    ph.certificate(dA, dB, dirs_c, pA_c, pB_c, lower=full_out, ws=cws)
    torch.cuda.synchronize()
    ph.profile_enable(False)
    cert["kernels_ms"] = {k: ph.profile_read(k)[1] for k in ("cert_rows", "cert_bins", "cert_scan",
                                                              "cert_query", "centroid", "cert_init")}
    ph.profile_reset()
    cert["inner_full_H"] = ph.decode_result(full_out)["H"]
    del cws
    log(f"certificate [{cert['lb']:.6f}, {cert['ub']:.6f}] in {cert['ms']:.3f} ms")

    def time_prohd(prec, kA_, kB_, reps, full=False):
        capA_ = int(min(nA, 2 * sum(min(k, nA) for k in kA_)))
        capB_ = int(min(nB, 2 * sum(min(k, nB) for k in kB_)))
        o = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)

        def run():
            _, pA, pB, _, _ = ph.prohd_project(dA, dB, m, ws=ws, evals=False)
            iA_, cA_, iB_, cB_ = ph.prohd_select(pA, pB, kA_, kB_, capA=capA_, capB=capB_, ws=ws)
            ph.prohd_hd(dA, dB, iA_, cA_, iB_, cB_, capA=capA_, capB=capB_, ws=ws, out=o, prec=prec,
                        inner_full=full)
        run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, ph.decode_result(o)

    exact = None
    if not args.no_exact:
        exact = {}
        Bd = B.astype(np.float64)
        for prec in ("fp32", "bf16", "fp8"):
            ph.profile_reset()
            ph.profile_enable(True)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            eout = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)
            reps = max(1, args.exact_steps)
            e0.record()
            for _ in range(reps):
                ph.exact_hd(dA, dB, ws=ws, out=eout, prec=prec)
            e1.record()
            torch.cuda.synchronize()
            ph.profile_enable(False)
            ems = e0.elapsed_time(e1) / reps
            er = ph.decode_result(eout)
            ek = {}
            for name in ("hd_prep", "hd_quant", "hd_subset", "hd_gather", "hd_tile_rows", "hd_tile_gx", "hd_tile",
                         "hd_keys", "hd_refine", "hd_dyn_refine", "hd_uncertain", "hd_finalize"):
                n_, t_ = ph.profile_read(name)
                if n_:
                    ek[name] = {"launches": n_ / reps, "ms": t_ / reps}
            ph.profile_reset()
            peak = {"fp32": PEAK_FP32_MFMA, "bf16": 2500.0, "fp8": 5000.0}[prec]
            # first pruning level: every row of each set against every F-th
            # row of the other, 2 D flops per pair
            elev = ph.prune_levels(nA, nB)
            first = None
            if elev and "hd_tile_rows" in ek:
                F = 16 ** elev
                ff = 2.0 * D * (nA * math.ceil(nB / F) + nB * math.ceil(nA / F))
                fms = ek["hd_tile_rows"]["ms"]
                first = {"F": F, "algorithmic_flops": ff, "ms": fms,
                         "tflops": ff / (fms * 1e-3) / 1e12, "frac": ff / (fms * 1e-3) / 1e12 / peak}
            # sampled parity: the witness row's NN over all of B in float64
            wnn = np.sqrt(((Bd - A[er["ab_a"]].astype(np.float64)) ** 2).sum(1)).min()
            exact[prec] = {"ms": ems, "pairs_per_s": 1e3 / ems, "H": er["H"], "hAB": er["hAB"],
                           "hBA": er["hBA"], "refined": er["refined"], "prune_levels": elev,
                           "first_level": first, "kernels": ek,
                           "witness_nn_rel_err": float(abs(wnn - er["hAB"]) / er["hAB"])}
            log(f"exact[{prec}] {ems:.1f} ms, H={er['H']:.6f}, levels {elev}, refined {er['refined']}, "
                f"kernels " + ", ".join(f"{k} {v['ms']:.2f}" for k, v in ek.items()))
        del Bd
        Hx = exact["fp32"]["H"]
        for prec in ("bf16", "fp8"):
            exact[prec]["rel_err_vs_fp32_exact"] = abs(exact[prec]["H"] - Hx) / Hx
        exact["prohd_fp32_rel_err_vs_exact"] = abs(res["H"] - Hx) / Hx
        exact["certificate_contains_exact"] = bool(cert["lb"] <= Hx <= cert["ub"])
        # precision form: ProHD with low-precision tiles against the float32
        # path, in candidate mode (Alg. 3's value) and in inner-full mode
        # (inner minimum over the whole other set, where the tiles carry the
        # n x |I| search), at the paper's alpha and at 4x alpha
        forms = []
        for full in (False, True):
            for mult in (1, 4):
                for prec in ("fp32", "bf16", "fp8"):
                    if not full and mult == 1 and prec == "fp32":
                        continue   # the headline step itself
                    if alpha is None:
                        kA_, kB_ = [k * mult for k in kA], [k * mult for k in kB]
                    else:
                        a_ = alpha * mult
                        kA_ = ph.alpha_k(a_, nA, m)
                        kB_ = ph.alpha_k(a_, nB, m)
                    ms_, r_ = time_prohd(prec, kA_, kB_, 3, full=full)
                    forms.append({"prec": prec, "mode": "inner_full" if full else "candidates",
                                  "alpha": None if alpha is None else alpha * mult, "ms": ms_,
                                  "H": r_["H"], "nA_sel": r_["nA_sel"], "nB_sel": r_["nB_sel"],
                                  "refined": r_["refined"], "rel_err_vs_exact": abs(r_["H"] - Hx) / Hx})
                    log(f"prohd[{prec}, {forms[-1]['mode']}, alpha x{mult}] {ms_:.2f} ms "
                        f"H={r_['H']:.6f} err={forms[-1]['rel_err_vs_exact']:.2e} refined={r_['refined']}")
        exact["precision_form"] = forms

    # sampling baselines at ProHD's budget and an alpha sweep on random clouds
    base = None
    if not args.no_baselines:
        from paper_2511_18207_amd import evaluate as EV
        base = {}
        for name in ("gauss5k", "mix200k"):
            A2, B2, p2 = synth.workload(name, seed=args.seed)
            a2, b2 = torch.from_numpy(A2).to(dev), torch.from_numpy(B2).to(dev)
            H2 = ph.decode_result(ph.exact_hd(a2, b2, ws=ws))["H"]
            base[name] = EV.baselines(a2, b2, H2, m=p2["m"], k=p2["k"], ws=ws)
            del a2, b2
        if exact is not None:
            base["heavy2m"] = EV.baselines(dA, dB, exact["fp32"]["H"], alpha=alpha, m=m, ws=ws,
                                           seeds=(0,))
        for name, b_ in base.items():
            c_ = b_["candidates"]
            log(f"baselines {name}: prohd {c_['prohd_err']:.3e} random {c_['random_err_mean']:.3e} "
                f"systematic {c_['systematic_err_mean']:.3e} (budget {c_['budget']})")
        sweep = EV.alpha_sweep(lambda D_: synth.uniform_clouds(100_000, 100_000, D_, seed=7),
                               (2, 4, 8, 16, 32, 64, 128), (0.001, 0.005, 0.01, 0.02, 0.05, 0.1), ws=ws)
        base["alpha_sweep_uniform_clouds"] = sweep
        log(f"alpha sweep: {len(sweep)} points")
        # adaptive alpha (prohd_adaptive) at a 1e-3 budget on the random
        # clouds and on this workload (e4m3 search tiles there)
        adapt = []
        kw = dict(alpha0=0.005, growth=2.0, alpha_max=0.32, tol=1e-3)
        for D_ in (4, 16, 64):
            A2, B2 = synth.uniform_clouds(100_000, 100_000, D_, seed=7)
            a2, b2 = torch.from_numpy(A2).to(dev), torch.from_numpy(B2).to(dev)
            H2 = ph.decode_result(ph.exact_hd(a2, b2, ws=ws))["H"]
            t0 = time.perf_counter()
            r_ = ph.adaptive(a2, b2, ws=ws, **kw)
            adapt.append({"workload": f"uniform clouds 100k x 100k D={D_}", "H": H2,
                          "ms": 1e3 * (time.perf_counter() - t0),
                          "rel_err": abs(r_["H"] - H2) / H2,
                          **{k: r_[k] for k in ("alpha", "H", "lb", "ub", "steps", "reason",
                                                "nA_sel", "nB_sel")}})
            del a2, b2
        if exact is not None:
            t0 = time.perf_counter()
            r_ = ph.adaptive(dA, dB, ws=ws, prec="fp8", **kw)
            Hx = exact["fp32"]["H"]
            adapt.append({"workload": f"{args.workload} (e4m3 tiles)", "H_exact": Hx,
                          "ms": 1e3 * (time.perf_counter() - t0), "rel_err": abs(r_["H"] - Hx) / Hx,
                          **{k: r_[k] for k in ("alpha", "H", "lb", "ub", "steps", "reason",
                                                "nA_sel", "nB_sel")}})
        for a_ in adapt:
            log(f"adaptive {a_['workload']}: alpha {a_['alpha']} after {a_['steps']} steps "
                f"(reason {a_['reason']}), err {a_['rel_err']:.2e}, {a_['ms']:.1f} ms")
        base["adaptive_alpha"] = adapt

    learned = None
    if not args.no_learned:
        del ws
        torch.cuda.empty_cache()
        # both tail laws of the learned form's workload: nu = 30 (the one it
        # is built for) and nu = 3 (every cluster heavy-tailed)
        learned = {f"nu{nu:g}": learned_form(args, dev, nu) for nu in args.learned_nu}
        ws = None

    batched = None
    if not args.no_batched:
        if ws is not None:
            del ws
            ws = None
        torch.cuda.empty_cache()
        batched = batched_form(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(A, B, m, alpha if alpha is not None else 0.01, min(args.cpu_sample, nA))
        log(f"cpu baseline {time.perf_counter() - t0:.1f}s: {cpu['value']:.4g} pairs/s")

    # stored FP64 oracle values for this workload and seed (written by
    # tests/golden/make_golden.py from oracle/ alone), when present
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{args.workload}_seed{args.seed}.json")
    if os.path.exists(gpath):
        with open(gpath) as fh:
            golden = json.load(fh)
    vs_oracle = {}
    if golden is not None:
        Ho = golden["prohd"]["H"]
        vs_oracle["prohd_H_oracle"] = Ho
        vs_oracle["prohd_rel_err"] = abs(res["H"] - Ho) / Ho
        if "exact" in golden and exact is not None:
            Hx_o = golden["exact"]["H"]
            vs_oracle["exact_H_oracle"] = Hx_o
            for prec in ("fp32", "bf16", "fp8"):
                vs_oracle[f"exact_{prec}_rel_err"] = abs(exact[prec]["H"] - Hx_o) / Hx_o
        if cpu is not None and "seconds_prohd" in golden:
            cpu["full_pair_recorded_s"] = golden["seconds_prohd"]

    detail = {
        "result": {"H": res["H"], "hAB": res["hAB"], "hBA": res["hBA"], "nA_sel": res["nA_sel"],
                   "nB_sel": res["nB_sel"], "status": res["status"], "refined": res.get("refined")},
        "vs_oracle": vs_oracle,
        "check": check,
        "unpruned_step": unpruned,
        "step_timing": {"eager_ms": eager_ms, "with_launch_events_ms": prof_ms, "graph_ms": graph_ms,
                        "graph_same_result": graph_same, "headline": "graph" if use_graph else "eager"},
        "certificate": cert,
        "roofline": roof,
        "path_roofline": path_roof,
        "attainable": peaks,
        "exact": exact,
        "kernels": kernels,
        "baselines": base,
        "learned": learned,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    dpath = args.detail_out
    if dpath:
        os.makedirs(os.path.dirname(os.path.abspath(dpath)), exist_ok=True)
        with open(dpath, "w") as fh:
            json.dump(detail, fh, indent=1)
        log(f"details written to {dpath}")
    log("detail " + json.dumps(detail))

    # the one stdout line: headline, roofline of the dominant kernel, CPU
    # oracle baseline, errors against the FP64 oracle and short summaries of
    # the forms (everything else is in the detail file / stderr line)
    def r4(x):
        return None if x is None else float(f"{x:.4g}")

    head_roof = {k: roof[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic",
                                      "avg_ms", "algorithmic_flops", "algorithmic_bytes",
                                      "share_of_step") if k in roof}
    line = {
        "metric": METRIC,
        "value": 1e3 / ms_step,
        "unit": "set-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "nA": nA, "nB": nB, "D": D, "alpha": alpha, "m": m,
                   "seed": args.seed},
        "result": {"H": res["H"], "nA_sel": res["nA_sel"], "nB_sel": res["nB_sel"],
                   "status": res["status"], "refined": res.get("refined")},
        "rel_err_vs_oracle": {k: r4(v) for k, v in vs_oracle.items() if k.endswith("rel_err")},
        "unpruned_ms_per_step": r4(unpruned["ms_per_step"]),
        "graph_ms_per_step": r4(graph_ms),
        "roofline": head_roof,
        "cpu_baseline": None if cpu is None else {
            k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample", "full_pair_recorded_s")
            if k in cpu},
        "exact": None if exact is None else {
            p_: {"ms": r4(exact[p_]["ms"]), "pairs_per_s": r4(exact[p_]["pairs_per_s"])}
            for p_ in ("fp32", "bf16", "fp8")},
        "forms": {
            "precision": None if exact is None else [
                [f_["prec"], f_["mode"], f_["alpha"], r4(f_["ms"]), r4(f_["rel_err_vs_exact"])]
                for f_ in exact["precision_form"]],
            "adaptive": None if base is None else [
                [a_["workload"], a_["alpha"], a_["steps"], a_["reason"], r4(a_["rel_err"]), r4(a_["ms"])]
                for a_ in base.get("adaptive_alpha", [])],
            "batched_prohd_pairs_per_s": None if batched is None else r4(batched["prohd"]["pairs_per_s"]),
            "batched_exact_pairs_per_s": None if batched is None else r4(batched["exact"]["pairs_per_s"]),
            "learned_mean_rel_err": None if learned is None else {
                law: {m_: {k: r4(v) for k, v in L_["mean_rel_err"][m_].items()}
                      for m_ in ("candidates", "full")} for law, L_ in learned.items()},
            "learned_score_ms": None if learned is None else {
                law: r4(L_["score"]["ms"]) for law, L_ in learned.items()},
        },
        "detail": dpath or "stderr",
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
