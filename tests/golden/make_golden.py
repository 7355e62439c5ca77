"""Write stored oracle results for the full-size workloads.

Every value in the files this script writes comes from ``oracle/`` (FP64
CPU) on inputs from ``synth/``; nothing comes from the HIP path.  The GPU
tests load them so that a full-size parity check does not have to rerun the
slow oracle on the GPU machine.

    python tests/golden/make_golden.py mix200k 0 1 2      # ProHD + exact
    python tests/golden/make_golden.py heavy2m 0 --no-exact
    python tests/golden/make_golden.py heavy2m 0 --exact-only   # adds the exact
        distance to an existing file (one pass over the distance matrix for
        both directions, oracle.exact_hd(one_pass=True))

Output: tests/golden/<workload>_seed<s>.json
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def idx_hash(I):
    return hashlib.sha256(np.asarray(I, dtype=np.int64).tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("seeds", type=int, nargs="+")
    ap.add_argument("--no-exact", action="store_true")
    ap.add_argument("--exact-only", action="store_true")
    args = ap.parse_args()
    for seed in args.seeds:
        A, B, params = synth.workload(args.workload, seed=seed)
        out = os.path.join(HERE, f"{args.workload}_seed{seed}.json")
        if args.exact_only:
            with open(out) as fh:
                rec = json.load(fh)
            t1 = time.perf_counter()
            e = oracle.exact_hd(A, B, one_pass=True)
            rec["exact"] = {k: e[k] for k in ("H", "hAB", "hBA", "ab_a", "ab_b", "ba_b", "ba_a")}
            rec["seconds_exact"] = time.perf_counter() - t1
            rec["exact_host_threads"] = len(os.sched_getaffinity(0))
            with open(out, "w") as fh:
                json.dump(rec, fh, indent=1)
            print(f"wrote {out}: H={rec['exact']['H']:.9g} ({rec['seconds_exact']:.0f} s)", flush=True)
            continue
        m = params["m"]
        kw = {"m": m, "k": params["k"]} if "k" in params else {"m": m, "alpha": params["alpha"]}
        t0 = time.perf_counter()
        p = oracle.prohd(A, B, **kw)
        t1 = time.perf_counter()
        rec = {
            "workload": args.workload, "seed": seed, "params": params,
            "generator": "synth.workload", "source": "oracle.prohd / oracle.exact_hd (FP64)",
            "prohd": {k: p[k] for k in ("H", "hAB", "hBA", "ab_a", "ab_b", "ba_b", "ba_a",
                                         "nA_sel", "nB_sel")},
            "IA_sha256": idx_hash(p["IA"]), "IB_sha256": idx_hash(p["IB"]),
            "kA": p["kA"], "kB": p["kB"],
            "dirs": p["dirs"].tolist(),
            "evals_top": p["evals"][: m + 2].tolist(),
            "seconds_prohd": t1 - t0,
        }
        if not args.no_exact:
            e = oracle.exact_hd(A, B, one_pass=A.shape[0] * B.shape[0] > 1 << 32)
            rec["exact"] = {k: e[k] for k in ("H", "hAB", "hBA", "ab_a", "ab_b", "ba_b", "ba_a")}
            rec["seconds_exact"] = time.perf_counter() - t1
        with open(out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(f"wrote {out}: H_hat={p['H']:.9g} |I|={p['nA_sel']}/{p['nB_sel']}"
              + (f" H={rec['exact']['H']:.9g}" if "exact" in rec else ""), flush=True)


if __name__ == "__main__":
    main()
