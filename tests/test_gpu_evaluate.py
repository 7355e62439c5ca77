"""GPU: sampling baselines and the alpha sweep (evaluate.py) -- the subset
distance they use is prohd_hd on given indices, checked here against the
oracle's subset distance; the samplers' index lists are checked for their
definitions."""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, rel, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def test_samplers_and_subset_hd():
    torch, dev = torch_gpu()
    from paper_2511_18207_amd import evaluate as EV
    banner("evaluate samplers + subset_hd")
    A, B = synth.gauss_outliers(3000, 2500, 16, seed=4)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    for kind in ("random", "systematic"):
        iA = EV.sample_indices(3000, 137, kind, 1)
        iB = EV.sample_indices(2500, 90, kind, 2)
        a, b = iA.cpu().numpy(), iB.cpu().numpy()
        assert a.size == 137 and b.size == 90
        assert np.all(np.diff(a) > 0) and np.all(np.diff(b) > 0) and a.max() < 3000 and b.max() < 2500
        if kind == "systematic":
            # the same seeded permutation, read at equally spaced positions
            for idx, n, size, seed in ((a, 3000, 137, 1), (b, 2500, 90, 2)):
                g = np.random.default_rng(seed)
                perm = g.permutation(n)
                step = n / size
                pos = np.floor(g.uniform(0.0, step) + step * np.arange(size)).astype(np.int64)
                assert np.ptp(np.diff(pos)) <= 1
                assert np.array_equal(np.sort(perm[pos]), idx)
        for full in (False, True):
            got = EV.subset_hd(dA, dB, iA, iB, inner_full=full)
            want = oracle.subset_hd(A, B, a, b, inner="full" if full else "candidates")
            assert rel(got["H"], want["H"]) <= 1e-5


def test_baselines_and_sweep_shapes():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    from paper_2511_18207_amd import evaluate as EV
    banner("evaluate baselines + alpha sweep")
    A, B = synth.gauss_outliers(5000, 5000, 32, seed=0)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    H = oracle.exact_hd(A, B)["H"]
    rep = EV.baselines(dA, dB, H, m=3, k=100)
    for mode in ("candidates", "full"):
        r = rep[mode]
        assert r["budget"][0] > 0 and len(r["random"]) == 3
        assert r["prohd_err"] >= 0 and r["random_err_max"] >= r["random_err_mean"] >= 0
    # the inner-full value never exceeds H, whatever the subset
    assert all(v <= H * (1 + 1e-6) for v in rep["full"]["random"] + rep["full"]["systematic"])
    rows = EV.alpha_sweep(lambda D: synth.uniform_clouds(4000, 4000, D, seed=1), (2, 8), (0.01, 0.1))
    assert len(rows) == 4
    for D in (2, 8):
        r = [x for x in rows if x["D"] == D]
        assert r[0]["budget"] <= r[1]["budget"]
        assert all(x["full"] <= x["H"] * (1 + 1e-6) for x in r)
