"""GPU parity: prohd_select (through the C ABI) against the oracle's selection.

Both sides get the same float32 projections, so the kept index sets must be
identical (bit-exact index work), ties and -0.0 included.
"""

import numpy as np
import pytest

import oracle
from gpu_common import banner, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def _run(torch, ph, PA, PB, kA, kB):
    idxA, nA, idxB, nB = ph.prohd_select(to_dev(torch, PA), to_dev(torch, PB), kA, kB)
    na, nb = int(nA.item()), int(nB.item())
    return idxA[:na].cpu().numpy(), idxB[:nb].cpu().numpy()


@pytest.mark.parametrize("nA,nB,ndirs,seed", [(1, 1, 1, 0), (7, 5, 2, 1), (4097, 3000, 4, 2),
                                              (50000, 70001, 9, 3)])
def test_select_with_ties(nA, nB, ndirs, seed):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_select ties nA={nA} nB={nB} ndirs={ndirs}")
    g = np.random.default_rng(seed)
    PA = g.integers(-20, 21, size=(ndirs, nA)).astype(np.float32)
    PB = (g.integers(-5, 6, size=(ndirs, nB)) * 0.25).astype(np.float32)
    PA[PA == 0] = -0.0
    kA = g.integers(1, max(2, nA // 3 + 2), size=ndirs)
    kB = g.integers(1, max(2, nB // 3 + 2), size=ndirs)
    kA[0] = nA + 5  # clipped to n
    gotA, gotB = _run(torch, ph, PA, PB, kA, kB)
    wantA, wantB = oracle.select(PA, PB, kA, kB)
    assert np.array_equal(gotA, wantA)
    assert np.array_equal(gotB, wantB)


@pytest.mark.parametrize("n,ndirs,k", [(200_000, 9, 1000), (1_000_003, 3, 20000), (65536, 17, 1)])
def test_select_continuous(n, ndirs, k):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_select continuous n={n} ndirs={ndirs} k={k}")
    g = np.random.default_rng(n + k)
    PA = g.standard_normal((ndirs, n)).astype(np.float32) * 3
    PB = (g.standard_t(3, size=(ndirs, n - 1)) + 0.5).astype(np.float32)
    kk = [k] * ndirs
    gotA, gotB = _run(torch, ph, PA, PB, kk, kk)
    wantA, wantB = oracle.select(PA, PB, kk, kk)
    assert np.array_equal(gotA, wantA)
    assert np.array_equal(gotB, wantB)


def test_select_all_equal_values():
    # every projection equal: both ends take the k smallest indices
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("prohd_select constant projections")
    PA = np.full((2, 10000), 1.5, np.float32)
    PB = np.zeros((2, 333), np.float32)
    gotA, gotB = _run(torch, ph, PA, PB, [17, 3], [5, 200])
    assert list(gotA) == list(range(17))
    assert list(gotB) == list(range(200))


def test_select_rejects_small_capacity():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    P = to_dev(torch, np.zeros((1, 100), np.float32))
    with pytest.raises(ph.ProhdError):
        ph.prohd_select(P, P, [10], [10], capA=19, capB=20)


def _top_input(kind, n, g):
    if kind == "rand":
        return g.standard_normal(n).astype(np.float32)
    if kind == "ties":   # a few distinct values, -0.0 among the zeros
        p = g.integers(-3, 4, size=n).astype(np.float32)
        p[p == 0] = -0.0
        return p
    # row bounds: non-negative squared distances, repeated values, +inf
    p = (g.gamma(2.0, 1.0, size=n) ** 2).astype(np.float32)
    p[g.integers(0, max(n, 1), size=n // 50)] = np.float32(4.0)
    p[g.integers(0, max(n, 1), size=n // 500)] = np.inf
    return p


@pytest.mark.parametrize("n,k,kind,seed", [
    (0, 64, "rand", 0), (1, 64, "rand", 1), (5, 3, "ties", 2), (63, 64, "ties", 3),
    (64, 64, "rand", 4), (65, 64, "ties", 5), (513, 64, "bounds", 6), (1000, 17, "rand", 7),
    (1000, 0, "rand", 8), (78966, 64, "bounds", 9), (300001, 64, "ties", 10),
    (2_000_003, 64, "bounds", 11), (2_000_003, 1, "rand", 12)])
def test_top_keys(n, k, kind, seed):
    """prohd_top_keys (the pruned search's seed step) against the oracle's
    k largest under (value, index): identical index lists."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_top_keys n={n} k={k} kind={kind}")
    g = np.random.default_rng(seed)
    p = _top_input(kind, n, g)
    idx, cnt = ph.top_keys(to_dev(torch, p), k)
    c = int(cnt.item())
    want = oracle.largest_indices(p, k)
    assert c == len(want)
    assert np.array_equal(idx[:c].cpu().numpy(), want)


@pytest.mark.parametrize("n,dn", [(5000, 1234), (5000, 9000), (5000, -3), (700000, 600001)])
def test_top_keys_device_length(n, dn):
    """The length read on the device (clipped to the host bound)."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_top_keys device length n={n} dn={dn}")
    g = np.random.default_rng(n + dn)
    p = _top_input("bounds", n, g)
    dlen = torch.tensor([dn], dtype=torch.int64, device=dev)
    ws = ph.Workspace(dev)
    for _ in range(2):   # the workspace's wave lists are reused
        idx, cnt = ph.top_keys(to_dev(torch, p), 64, dev_n=dlen, ws=ws)
        c = int(cnt.item())
        want = oracle.largest_indices(p[:max(0, min(dn, n))], 64)
        assert c == len(want)
        assert np.array_equal(idx[:c].cpu().numpy(), want)
