"""GPU parity of the certified refinement, through the C ABI, against the
FP64 oracle.

The distance search bounds every row's true minimum from both sides (from
the search's worst-case error) and re-measures in float64 every row whose
upper bound reaches the largest lower bound (k_hd.hip, certified
refinement; the batched form re-measures 256 rows first, then every row the
bound cannot rule out).  The case that needs many rows re-measured: a cloud
in [0, 100]^64 against a copy of itself moved by 0.01-0.02 per row, one row
moved by 0.05, so that the expanded form cannot resolve the
nearest-neighbour distances in any of the three search precisions.  Exact
distance (Eq. (1)) and the candidate distance (Alg. 3, both inner modes)
must match the oracle at 1e-4; on ordinary data a handful of rows is
re-measured.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, rel, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def perturbed_copy(n, D, seed):
    g = np.random.default_rng(seed)
    A = g.uniform(0.0, 100.0, size=(n, D)).astype(np.float32)
    v = g.standard_normal((n, D))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    step = g.uniform(0.01, 0.02, size=n)
    j = int(g.integers(n))
    step[j] = 0.05
    B = (A.astype(np.float64) + v * step[:, None]).astype(np.float32)
    return A, B, j


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_exact_near_duplicate(prec):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"exact_hd near-duplicate 8000x64 prec={prec}")
    A, B, j = perturbed_copy(8000, 64, seed=0)
    o = oracle.exact_hd(A, B)
    assert o["ab_a"] == j
    r = ph.decode_result(ph.exact_hd(to_dev(torch, A), to_dev(torch, B), sync=True, prec=prec))
    assert r["status"] == 0
    assert rel(r["H"], o["H"]) <= 1e-4, (r["H"], o["H"])
    assert rel(r["hAB"], o["hAB"]) <= 1e-4 and rel(r["hBA"], o["hBA"]) <= 1e-4
    assert r["ab_a"] == o["ab_a"]
    assert r["refined"] > 256          # the uncertain rows were re-measured


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("inner_full", [False, True])
def test_prohd_hd_near_duplicate(prec, inner_full):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_hd near-duplicate prec={prec} full={inner_full}")
    A, B, j = perturbed_copy(6000, 64, seed=1)
    g = np.random.default_rng(2)
    I = np.union1d(g.choice(6000, 2500, replace=False), [j]).astype(np.int32)
    o = oracle.subset_hd(A, B, I, I, inner="full" if inner_full else "candidates")
    cnt = torch.tensor([I.size, I.size], dtype=torch.int64, device=dev)
    dI = torch.from_numpy(I).cuda()
    out = ph.prohd_hd(to_dev(torch, A), to_dev(torch, B), dI, cnt[0:1], dI.clone(), cnt[1:2],
                      inner_full=inner_full, sync=True, prec=prec)
    r = ph.decode_result(out)
    assert r["status"] == 0
    assert rel(r["H"], o["H"]) <= 1e-4, (r["H"], o["H"])


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_few_rows_refined_on_ordinary_data(prec):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"exact_hd gauss 5000x5000x32 prec={prec} (refined rows)")
    A, B = synth.gauss_outliers(5000, 5000, 32, seed=0)
    o = oracle.exact_hd(A, B)
    r = ph.decode_result(ph.exact_hd(to_dev(torch, A), to_dev(torch, B), sync=True, prec=prec))
    assert r["status"] == 0 and rel(r["H"], o["H"]) <= 1e-5
    print(f"[refine] gauss 5000 {prec}: refined {r['refined']}", flush=True)
    if prec == "fp32":
        assert 1 <= r["refined"] <= 16, r["refined"]
    else:
        assert 1 <= r["refined"] < 5000, r["refined"]


def test_batched_near_duplicate():
    """The batched form (float32 search) on a batch mixing near-duplicate
    pairs with ordinary ones: per-pair exact distance and ProHD against the
    oracle."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("batched near-duplicate pairs, exact + prohd")
    As, Bs = [], []
    for i, (n, D) in enumerate([(3000, 64), (1200, 64), (2500, 128), (900, 256)]):
        if i % 2 == 0:
            a, b, _ = perturbed_copy(n, D, seed=10 + i)
        else:
            a, b = synth.gauss_outliers(n, n + 100, D, seed=10 + i)
        As.append(a)
        Bs.append(b)
    nA = [a.shape[0] for a in As]
    nB = [b.shape[0] for b in Bs]
    D = [a.shape[1] for a in As]
    plan = ph.BatchPlan(nA, nB, D, alpha=0.01)
    dA, dB = plan.pack(As, Bs)
    try:
        rx = plan.results(plan.run(dA, dB, mode="exact", sync=True))
        rp = plan.results(plan.run(dA, dB, mode="prohd", sync=True))
    finally:
        plan.close()
    for i in range(len(As)):
        ox = oracle.exact_hd(As[i], Bs[i])["H"]
        m = int(np.floor(np.sqrt(D[i]) + 1e-9))
        op = oracle.prohd(As[i], Bs[i], alpha=0.01, m=m)["H"]
        assert rx[i]["status"] == 0 and rel(rx[i]["H"], ox) <= 1e-4, (i, rx[i]["H"], ox)
        assert rp[i]["status"] == 0 and rel(rp[i]["H"], op) <= 1e-4, (i, rp[i]["H"], op)
