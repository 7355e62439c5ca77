"""Evaluation helpers around the library: sampling baselines at ProHD's
candidate budget and alpha sweeps.

The paper compares ProHD with random and systematic sampling of the same
number of points (Sec. III, Table II), and studies the error and time as
alpha grows on random clouds (Sec. III).  Here both run on the device: the
baselines draw index lists (seeded; the random numbers are inputs) and
evaluate the subset distance with ``prohd_hd`` -- the same kernels as
ProHD's own candidate distance -- so the three methods differ only in how
the subsets are chosen.
"""

from __future__ import annotations

import math

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def sample_indices(n, size, kind, seed, device="cuda"):
    """Ascending int32 indices of ``size`` rows out of ``n``.

    ``random``: uniformly without replacement (seeded permutation);
    ``systematic``: the paper's systematic random sampling (Sec. III
    baselines) -- a seeded random permutation of the rows, then every
    (n / size)-th position of it from a seeded random start (the stride that
    gives exactly ``size`` rows, where the paper's floor(1 / alpha) gives
    about alpha n)."""
    torch = _torch()
    size = int(min(max(1, size), n))
    if kind == "random":
        g = torch.Generator(device="cpu")
        g.manual_seed(int(seed))
        idx = torch.randperm(int(n), generator=g)[:size]
        idx, _ = torch.sort(idx)
    elif kind == "systematic":
        g = np.random.default_rng(seed)
        perm = g.permutation(int(n))
        step = n / size
        start = g.uniform(0.0, step)
        pos = np.clip(np.floor(start + step * np.arange(size)).astype(np.int64), 0, n - 1)
        idx = torch.from_numpy(np.sort(perm[pos]))
    else:
        raise ValueError(kind)
    return idx.to(device=device, dtype=torch.int32).contiguous()


def subset_hd(A, B, idxA, idxB, inner_full=False, ws=None):
    """H over the given rows (device index lists), via prohd_hd."""
    torch = _torch()
    cA = torch.tensor([idxA.numel()], dtype=torch.int64, device=A.device)
    cB = torch.tensor([idxB.numel()], dtype=torch.int64, device=A.device)
    return L.decode_result(L.prohd_hd(A, B, idxA, cA, idxB, cB, inner_full=inner_full, ws=ws))


def baselines(A, B, H, alpha=None, m=None, k=None, seeds=(0, 1, 2), ws=None):
    """ProHD against random and systematic sampling with the same |I_A| and
    |I_B|, in both inner modes.  ``H``: the exact distance.  Returns a dict
    of relative errors |x - H| / H (sampling: mean and max over seeds)."""
    nA, nB = A.shape[0], B.shape[0]

    def err(x):
        return abs(x - H) / H if H > 0 else abs(x)

    out = {"H": H}
    for mode, full in (("candidates", False), ("full", True)):
        r = L.prohd(A, B, alpha=0.01 if alpha is None else alpha, m=m, k=k, inner_full=full, ws=ws)
        sA, sB = int(r["nA_sel"]), int(r["nB_sel"])
        row = {"budget": [sA, sB], "prohd": r["H"], "prohd_err": err(r["H"])}
        for kind in ("random", "systematic"):
            vals = []
            for s in seeds:
                iA = sample_indices(nA, sA, kind, 2 * s, A.device)
                iB = sample_indices(nB, sB, kind, 2 * s + 1, A.device)
                vals.append(subset_hd(A, B, iA, iB, inner_full=full, ws=ws)["H"])
            e = [err(v) for v in vals]
            row[kind] = vals
            row[kind + "_err_mean"] = float(np.mean(e))
            row[kind + "_err_max"] = float(np.max(e))
        out[mode] = row
    return out


def alpha_sweep(make_pair, dims, alphas, ws=None, reps=3):
    """ProHD error and time against alpha for pairs ``make_pair(D)`` (host
    float32 arrays), m = floor(sqrt(D)).  Returns one dict per (D, alpha)."""
    torch = _torch()
    rows = []
    for D in dims:
        A, B = make_pair(D)
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        H = L.decode_result(L.exact_hd(dA, dB, ws=ws))["H"]
        m = L.default_m(D)
        for a in alphas:
            L.prohd(dA, dB, alpha=a, m=m, ws=ws)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                r = L.prohd(dA, dB, alpha=a, m=m, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            f = L.prohd(dA, dB, alpha=a, m=m, inner_full=True, ws=ws)
            rows.append({"D": D, "n": A.shape[0], "alpha": a, "m": m, "H": H, "prohd": r["H"],
                         "rel_err": abs(r["H"] - H) / H, "full": f["H"],
                         "full_rel_err": abs(f["H"] - H) / H,
                         "budget": int(r["nA_sel"]) + int(r["nB_sel"]),
                         "ms": e0.elapsed_time(e1) / reps})
        del dA, dB
    return rows
