"""GPU parity of the pruned distance search (PROHD_PRUNE) through the C ABI,
against the FP64 oracle and against the unpruned search.

The pruned search (k_hd.hip, pruned search) bounds every outer row's
minimum from above by its minimum over every F-th inner row, re-measures
the 256 rows with the largest bounds against the whole inner set, drops the
rows whose bound cannot exceed the largest re-measured minimum, and searches
the rest against 16 times finer subsets level by level, the last level
against the whole inner set.  It must return the unpruned search's result
exactly (same witness rows, same float64 values) and the oracle's value of
Eq. (1) / the candidate distance of Alg. 3:

* exact distance on ragged Gaussian sets with outliers, three precisions;
* the near-duplicate case (a set against a slightly moved copy of itself),
  where no row can be dropped and every row goes through every level;
* candidate lists (Alg. 3, both inner modes) of ragged sizes;
* the size rule: below 16384 rows on either side the flag changes nothing.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, rel, to_dev, torch_gpu

pytestmark = pytest.mark.gpu

KEYS = ("H", "hAB", "hBA", "ab_a", "ab_b", "ba_b", "ba_a", "nA_sel", "nB_sel", "status")


def _subset_launches(ph, fn):
    """Result of fn() and the number of subset-gather launches it made."""
    ph.profile_reset()
    ph.profile_enable(True)
    try:
        r = fn()
    finally:
        ph.profile_enable(False)
    n, _ = ph.profile_read("hd_subset")
    return r, n


def _same(a, b):
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])


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


@pytest.fixture(scope="module")
def gauss40k():
    A, B = synth.gauss_outliers(40000, 36017, 64, seed=4)
    return A, B, oracle.exact_hd(A, B, one_pass=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_exact_pruned(gauss40k, prec):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    A, B, o = gauss40k
    banner(f"exact_hd pruned gauss 40000x36017x64 prec={prec}")
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    rp, n = _subset_launches(ph, lambda: ph.decode_result(ph.exact_hd(dA, dB, sync=True, prec=prec)))
    assert n == 2 * 2                                   # pruned, levels of strides 256 and 16
    ru = ph.decode_result(ph.exact_hd(dA, dB, sync=True, prec=prec, prune=False))
    print(f"[prune] exact {prec}: H {rp['H']:.9g} (unpruned {ru['H']:.9g}, oracle {o['H']:.9g}), "
          f"refined {rp['refined']} / {ru['refined']}", flush=True)
    _same(rp, ru)
    assert rel(rp["H"], o["H"]) <= 1e-5
    assert rel(rp["hAB"], o["hAB"]) <= 1e-5 and rel(rp["hBA"], o["hBA"]) <= 1e-5
    assert rp["ab_a"] == o["ab_a"] and rp["ba_b"] == o["ba_b"]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_exact_pruned_near_duplicate(prec):
    """Every row's subset bound exceeds the largest re-measured minimum (the
    nearest row of the copy is almost never in the subset), so the second
    stage searches every row against the whole copy, and the certified
    refinement then re-measures the rows the expansion cannot resolve."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"exact_hd pruned near-duplicate 20000x64 prec={prec}")
    A, B, j = perturbed_copy(20000, 64, seed=3)
    o = oracle.exact_hd(A, B, one_pass=True)
    assert o["ab_a"] == j
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    rp, n = _subset_launches(ph, lambda: ph.decode_result(ph.exact_hd(dA, dB, sync=True, prec=prec)))
    assert n == 2 * 2
    assert rp["status"] == 0
    assert rel(rp["H"], o["H"]) <= 1e-4, (rp["H"], o["H"])
    assert rel(rp["hAB"], o["hAB"]) <= 1e-4 and rel(rp["hBA"], o["hBA"]) <= 1e-4
    assert rp["ab_a"] == j
    assert rp["refined"] > 256
    ru = ph.decode_result(ph.exact_hd(dA, dB, sync=True, prec=prec, prune=False))
    _same(rp, ru)


@pytest.fixture(scope="module")
def tmix60k():
    A, B = synth.t_mixture(60000, 50000, 128, seed=6)
    g = np.random.default_rng(7)
    IA = np.sort(g.choice(60000, 21111, replace=False)).astype(np.int32)
    IB = np.sort(g.choice(50000, 16384, replace=False)).astype(np.int32)
    return A, B, IA, IB, {}


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("inner_full", [False, True])
def test_prohd_hd_pruned_candidates(tmix60k, prec, inner_full):
    """Candidate distance of Alg. 3 (inner minimum over the other candidate
    list, or over the whole other set) on lists of 21 111 and 16 384 rows
    (the smallest pruned size)."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    A, B, IA, IB, memo = tmix60k
    mode = "full" if inner_full else "candidates"
    banner(f"prohd_hd pruned t-mixture 60000x50000x128 lists 21111/16384 prec={prec} inner={mode}")
    if mode not in memo:
        memo[mode] = oracle.subset_hd(A, B, IA, IB, inner=mode)
    o = memo[mode]
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    dIA, dIB = torch.from_numpy(IA).cuda(), torch.from_numpy(IB).cuda()
    cnt = torch.tensor([IA.size, IB.size], dtype=torch.int64, device=dev)

    def run(prune):
        return ph.decode_result(ph.prohd_hd(dA, dB, dIA, cnt[0:1], dIB, cnt[1:2], sync=True,
                                            prec=prec, prune=prune, inner_full=inner_full))

    rp, n = _subset_launches(ph, lambda: run(True))
    assert n == 2 * 2
    ru = run(False)
    print(f"[prune] {mode} {prec}: H {rp['H']:.9g} (oracle {o['H']:.9g}), refined "
          f"{rp['refined']} / {ru['refined']}", flush=True)
    _same(rp, ru)
    assert rel(rp["H"], o["H"]) <= 1e-5
    assert rel(rp["hAB"], o["hAB"]) <= 1e-5 and rel(rp["hBA"], o["hBA"]) <= 1e-5


def test_prune_size_rule():
    """One side below 16384 rows: the flag is ignored (no subset launch) and
    the result is the unpruned one, in both inner modes."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("exact_hd prune size rule 16383 x 30000 x 32")
    A, B = synth.gauss_outliers(16383, 30000, 32, seed=8)
    o = oracle.exact_hd(A, B, one_pass=True)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    rp, n = _subset_launches(ph, lambda: ph.decode_result(ph.exact_hd(dA, dB, sync=True)))
    assert n == 0
    assert rel(rp["H"], o["H"]) <= 1e-5
    I = torch.arange(16383, dtype=torch.int32, device=dev)
    J = torch.arange(30000, dtype=torch.int32, device=dev)
    cnt = torch.tensor([16383, 30000], dtype=torch.int64, device=dev)
    rf, n = _subset_launches(ph, lambda: ph.decode_result(
        ph.prohd_hd(dA, dB, I, cnt[0:1], J, cnt[1:2], inner_full=True, sync=True)))
    assert n == 0
    assert rel(rf["H"], o["H"]) <= 1e-5


def test_prohd_end_to_end_pruned_mix200k():
    """ProHD (alpha mode) on the 200 000 x 200 000, D = 128 mixture: the
    pruned and unpruned searches give the same result."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("prohd pruned vs unpruned mix200k seed 0 (alpha 0.1)")
    A, B, _ = synth.workload("mix200k", seed=0)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    del A, B
    rp, n = _subset_launches(ph, lambda: ph.prohd(dA, dB, alpha=0.1))
    lev = ph.prune_levels(200_000, 200_000, rp["idxA"].numel(), rp["idxB"].numel())
    assert lev >= 2 and n == 2 * lev, (rp["nA_sel"], rp["nB_sel"], lev, n)
    ru = ph.prohd(dA, dB, alpha=0.1, prune=False)
    _same(rp, ru)


def test_exact_pruned_four_levels():
    """Exact distance at 1 200 000 x 1 100 000, D = 16 (strides 65536, 4096,
    256, 16): pruned against unpruned field by field, and the witness rows'
    nearest-neighbour distances re-measured in float64 on the host."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("exact_hd pruned gauss 1200000x1100000x16 (four levels)")
    A, B = synth.gauss_outliers(1_200_000, 1_100_000, 16, seed=9)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    rp, n = _subset_launches(ph, lambda: ph.decode_result(ph.exact_hd(dA, dB, sync=True)))
    assert n == 2 * 4
    ru = ph.decode_result(ph.exact_hd(dA, dB, sync=True, prune=False))
    _same(rp, ru)
    Bd = B.astype(np.float64)
    Ad = A.astype(np.float64)
    nnA = np.sqrt(((Bd - Ad[rp["ab_a"]]) ** 2).sum(1)).min()
    nnB = np.sqrt(((Ad - Bd[rp["ba_b"]]) ** 2).sum(1)).min()
    assert rel(rp["hAB"], nnA) <= 1e-12 and rel(rp["hBA"], nnB) <= 1e-12
