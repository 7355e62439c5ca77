"""Learned candidate proposal: a scorer network adds likely Hausdorff
witnesses to ProHD's extreme candidates (Alg. 1 / Alg. 2 select extremes
along directions; this form only ever adds points to those sets, so plain
ProHD remains the fallback and the exact distance of Eq. (1) the yardstick).

Every arithmetic step runs in the library's kernels through the C ABI:

* labels -- ``exact_hd`` with per-row nearest-neighbour distances (the exact
  brute-force search); a point is a positive when its NN distance to the
  other set is among the largest ``frac`` of its own set
  (``prohd_select_scored`` picks them, ties to the smaller index);
* features ``[x, x - c_other]`` with ``c_other`` from ``prohd_centroid``;
* training -- ``prohd_mlp_train_step`` (bfloat16 forward and backward on the
  matrix cores, AdamW on float32 master parameters);
* inference -- ``prohd_mlp_score``, then ``prohd_select_scored`` merges the
  top-s points into ProHD's index lists and ``prohd_hd`` evaluates.

torch is used for device buffers, the batch sampler's random indices and
index bookkeeping only.
"""

from __future__ import annotations

import math

import numpy as np

from . import _lib as L

LABEL_FRAC = 0.001


def _torch():
    import torch
    return torch


def witness_labels(A, B, frac=LABEL_FRAC, ws=None, prec="fp32"):
    """(yA, yB, exact) -- float32 0/1 labels per row of A and of B, and the
    decoded exact result.  Positives: the ceil-free ``max(1, floor(frac n))``
    rows with the largest NN distance to the other set."""
    torch = _torch()
    out, nnA, nnB = L.exact_hd(A, B, nn2=True, ws=ws, prec=prec)
    nA, nB = A.shape[0], B.shape[0]
    sA = max(1, int(math.floor(frac * nA)))
    sB = max(1, int(math.floor(frac * nB)))
    idxA = torch.empty(sA, dtype=torch.int32, device=A.device)
    idxB = torch.empty(sB, dtype=torch.int32, device=A.device)
    cnt = torch.zeros(2, dtype=torch.int64, device=A.device)
    L.select_scored(nnA, sA, nnB, sB, idxA, cnt[0:1], idxB, cnt[1:2], ws=ws)
    yA = torch.zeros(nA, dtype=torch.float32, device=A.device)
    yB = torch.zeros(nB, dtype=torch.float32, device=A.device)
    yA[idxA.long()] = 1.0
    yB[idxB.long()] = 1.0
    return yA, yB, L.decode_result(out)


class Scorer:
    """Parameters and optimiser state of the scorer for dimension D."""

    def __init__(self, D, seed=0, device="cuda"):
        torch = _torch()
        self.D = int(D)
        self.params = L.mlp_init(self.D, seed=seed, device=device)
        P = self.params.numel()
        self.m = torch.zeros(P, dtype=torch.float32, device=device)
        self.v = torch.zeros(P, dtype=torch.float32, device=device)
        self.grad = torch.empty(P, dtype=torch.float32, device=device)
        self.loss = torch.empty(1, dtype=torch.float32, device=device)
        self.t = 0

    def train_step(self, X, c_other, labels, idx, lr, pos_weight=1.0, weight_decay=0.01, ws=None):
        self.t += 1
        return L.mlp_train_step(X, c_other, labels, idx, self.params, self.grad, self.m, self.v,
                                self.t, lr, pos_weight=pos_weight, weight_decay=weight_decay,
                                loss=self.loss, ws=ws)

    def score(self, X, c_other, out=None, ws=None):
        return L.mlp_score(X, c_other, self.params, out=out, ws=ws)

    def save(self, path):
        from safetensors.torch import save_file
        save_file({"params": self.params.detach().cpu()}, path,
                  metadata={"D": str(self.D), "H1": "256", "H2": "128", "t": str(self.t)})

    @classmethod
    def load(cls, path, device="cuda"):
        from safetensors import safe_open
        with safe_open(path, framework="pt") as f:
            meta = f.metadata()
            p = f.get_tensor("params")
        if meta.get("H1") != "256" or meta.get("H2") != "128":
            raise ValueError("scorer file has other layer sizes")
        s = cls(int(meta["D"]), device=device)
        if p.numel() != s.params.numel():
            raise ValueError("scorer file has the wrong parameter count")
        s.params.copy_(p.to(device=device, dtype=s.params.dtype))
        s.t = int(meta.get("t", "0"))
        return s


class TrainPair:
    """One training pair resident on the device with its centroids and labels."""

    def __init__(self, A, B, frac=LABEL_FRAC, ws=None):
        self.A, self.B = A, B
        self.cA = L.centroid(A, ws=ws)
        self.cB = L.centroid(B, ws=ws)
        self.yA, self.yB, self.exact = witness_labels(A, B, frac, ws=ws)
        self.posA = self.yA.nonzero().flatten().to(_torch().int32)
        self.posB = self.yB.nonzero().flatten().to(_torch().int32)

    def side(self, s):
        """(X, c_other, labels, positive indices) of side 0 (A) or 1 (B)."""
        if s == 0:
            return self.A, self.cB, self.yA, self.posA
        return self.B, self.cA, self.yB, self.posB


def train(scorer, pairs, steps, batch=16384, lr=1e-3, lr_final=1e-4, pos_share=0.25,
          pos_weight=1.0, weight_decay=0.01, seed=0, ws=None, log_every=0, log=print):
    """Trains ``scorer`` on ``pairs`` (TrainPair list).  Each step takes one
    side of one pair; a ``pos_share`` fraction of the batch is drawn from
    that side's positives (uniformly, with replacement), the rest from all
    its rows.  Learning rate: cosine from ``lr`` to ``lr_final``.  Returns
    the per-step losses (host)."""
    torch = _torch()
    dev = scorer.params.device
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    losses = torch.empty(steps, dtype=torch.float32, device=dev)
    npos = int(round(pos_share * batch))
    for it in range(steps):
        pr = pairs[it % len(pairs)]
        X, c, y, pos = pr.side((it // len(pairs)) % 2)
        n = X.shape[0]
        idx = torch.randint(0, n, (batch,), generator=g, device=dev, dtype=torch.int32)
        if npos and pos.numel():
            j = torch.randint(0, pos.numel(), (npos,), generator=g, device=dev)
            idx[:npos] = pos[j]
        cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * it / max(1, steps - 1)))
        loss = scorer.train_step(X, c, y, idx, cur, pos_weight=pos_weight,
                                 weight_decay=weight_decay, ws=ws)
        losses[it:it + 1].copy_(loss)
        if log_every and (it + 1) % log_every == 0:
            log(f"[train] step {it + 1}/{steps} loss {losses[max(0, it + 1 - log_every):it + 1].mean().item():.4f}")
    return losses.cpu().numpy()


def _alpha_k(alpha, m, n):
    return L.alpha_k(alpha, n, m)


def proposal(A, B, scorer, alpha=0.01, m=None, add_frac=0.1, inner_full=False, ws=None,
             prec="fp32", base=None):
    """ProHD(alpha) with the top-s scored points of each set added
    (s = add_frac x |I| of that set).  With ``scorer=None`` this is plain
    ProHD.  Returns a dict: H (decoded result), the index lists and sizes."""
    torch = _torch()
    if base is None:
        base = L.prohd(A, B, alpha=alpha, m=m, inner_full=inner_full, ws=ws, prec=prec)
    if scorer is None:
        return base
    nA, nB = A.shape[0], B.shape[0]
    n0A, n0B = int(base["nA_sel"]), int(base["nB_sel"])
    sA = int(round(add_frac * n0A))
    sB = int(round(add_frac * n0B))
    capA, capB = min(nA, n0A + sA), min(nB, n0B + sB)
    idxA = torch.empty(capA, dtype=torch.int32, device=A.device)
    idxB = torch.empty(capB, dtype=torch.int32, device=A.device)
    idxA[:n0A] = base["idxA"][:n0A]
    idxB[:n0B] = base["idxB"][:n0B]
    cnt = torch.tensor([n0A, n0B], dtype=torch.int64, device=A.device)
    cA = L.centroid(A, ws=ws)
    cB = L.centroid(B, ws=ws)
    scA = scorer.score(A, cB, ws=ws)
    scB = scorer.score(B, cA, ws=ws)
    L.select_scored(scA, sA, scB, sB, idxA, cnt[0:1], idxB, cnt[1:2], ws=ws)
    out = L.prohd_hd(A, B, idxA, cnt[0:1], idxB, cnt[1:2], inner_full=inner_full, ws=ws,
                     prec=prec)
    res = L.decode_result(out)
    res.update({"idxA": idxA, "idxB": idxB, "nselA": cnt[0:1], "nselB": cnt[1:2], "added": (sA, sB)})
    return res


def plain_at_budget(A, B, target, base, inner_full=False, ws=None, prec="fp32", tol=0.01,
                    iters=40):
    """Plain ProHD on the same directions with every k scaled by one factor
    f, f chosen (bisection) so that |I_A| + |I_B| is within ``tol`` of
    ``target``.  Returns the decoded result with the chosen factor."""
    torch = _torch()
    pA, pB = base["projA"], base["projB"]
    kA0, kB0 = base["kA"], base["kB"]
    nA, nB = A.shape[0], B.shape[0]

    def run(f):
        kA = [min(nA, max(1, int(math.floor(k * f)))) for k in kA0]
        kB = [min(nB, max(1, int(math.floor(k * f)))) for k in kB0]
        iA, cA, iB, cB = L.prohd_select(pA, pB, kA, kB, ws=ws)
        tot = int(cA.item()) + int(cB.item())
        return tot, (iA, cA, iB, cB)

    lo, hi = 1.0, 2.0
    tot, sel = run(hi)
    while tot < target and hi < 1e4:
        lo, hi = hi, hi * 2
        tot, sel = run(hi)
    best = None
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        tot, sel = run(mid)
        if best is None or abs(tot - target) < abs(best[0] - target):
            best = (tot, sel, mid)
        if abs(tot - target) <= tol * target:
            break
        if tot < target:
            lo = mid
        else:
            hi = mid
    tot, (iA, cA, iB, cB), f = best
    out = L.prohd_hd(A, B, iA, cA, iB, cB, inner_full=inner_full, ws=ws, prec=prec)
    res = L.decode_result(out)
    res.update({"factor": f, "budget": tot})
    return res


def equal_budget(A, B, scorer, alpha=0.01, m=None, add_frac=0.1, H=None, ws=None, prec="fp32"):
    """Learned proposal vs plain ProHD at the same total candidate count, in
    both inner modes.  ``H``: the exact distance (computed when None).
    Returns a dict of values and relative errors |x - H| / H."""
    if H is None:
        H = L.decode_result(L.exact_hd(A, B, ws=ws, prec=prec))["H"]
    rep = {"H": H}
    for mode, full in (("candidates", False), ("full", True)):
        base = L.prohd(A, B, alpha=alpha, m=m, inner_full=full, ws=ws, prec=prec)
        learned = proposal(A, B, scorer, alpha=alpha, m=m, add_frac=add_frac, inner_full=full,
                           ws=ws, prec=prec, base=base)
        budget = int(learned["nA_sel"]) + int(learned["nB_sel"])
        plain = plain_at_budget(A, B, budget, base, inner_full=full, ws=ws, prec=prec)

        def err(x):
            return abs(x - H) / H if H > 0 else abs(x)

        rep[mode] = {
            "prohd": base["H"], "prohd_err": err(base["H"]),
            "prohd_budget": int(base["nA_sel"]) + int(base["nB_sel"]),
            "learned": learned["H"], "learned_err": err(learned["H"]), "learned_budget": budget,
            "plain": plain["H"], "plain_err": err(plain["H"]), "plain_budget": plain["budget"],
            "plain_factor": plain["factor"],
        }
    return rep
