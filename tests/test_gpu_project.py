"""GPU parity: prohd_project (directions, eigenvalues, projections) and the
whole ProHD chain, through the C ABI, against the FP64 oracle.

Directions: the centroid axis must match the oracle's (same sign); each
principal component must match up to sign, to within float32 rounding when
its eigenvalue is separated from its neighbours (Davis-Kahan: the float64
covariance error is ~1e-13 of its norm).  Near-degenerate eigenvalues are
compared as subspaces.  Candidate sets are compared with the oracle run on
the GPU's own directions: they may differ only at indices whose projection
lies within 1e-5 relative of that direction end's k-th value.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, rel, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def _dirs_close(got, want, evals):
    """Compare unit rows up to sign; separated eigenvalues elementwise."""
    m = want.shape[0]
    ev = np.asarray(evals, dtype=np.float64)
    scale = max(abs(ev[0]), 1e-300)
    for r in range(m):
        gap = min(abs(ev[r] - ev[r + 1]) if r + 1 < ev.size else np.inf,
                  abs(ev[r] - ev[r - 1]) if r > 0 else np.inf)
        c = abs(float(got[r] @ want[r]))
        if gap > 1e-6 * scale:
            assert c >= 1 - 1e-6, (r, c, gap)
    # subspace of all m: principal angles via SVD of the cross product
    s = np.linalg.svd(got @ want.T, compute_uv=False)
    if m < ev.size and abs(ev[m - 1] - ev[m]) > 1e-6 * scale:
        assert s.min() >= 1 - 1e-6


CASES = [
    ("gauss", 5000, 5000, 32, 3),
    ("mix", 20000, 15000, 128, 8),
    ("heavy", 30000, 30000, 256, 16),
    ("gauss", 700, 300, 7, 2),
    ("mix", 3000, 4000, 64, 8),
    ("gauss", 100, 80, 1, 1),
]


def _data(kind, nA, nB, D, seed):
    if kind == "gauss":
        return synth.gauss_outliers(nA, nB, D, seed=seed)
    if kind == "mix":
        return synth.mixture(nA, nB, D, seed=seed, K=64, normalize=True)
    return synth.mixture(nA, nB, D, seed=seed, K=128, outlier_frac=0.001)


@pytest.mark.parametrize("kind,nA,nB,D,m", CASES)
def test_project_directions_and_projections(kind, nA, nB, D, m):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_project {kind} nA={nA} nB={nB} D={D} m={m}")
    A, B = _data(kind, nA, nB, D, seed=D)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    dirs, pA, pB, ev, st = ph.prohd_project(dA, dB, m, sync=True)
    assert int(st.item()) == 0
    dirs = dirs.cpu().numpy().astype(np.float64)
    u0 = oracle.centroid_direction(A, B)
    U, evals = oracle.principal_directions(A, B, m)
    # centroid axis: same direction and sign
    assert float(dirs[0] @ u0) >= 1 - 1e-6
    assert np.allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-6)
    _dirs_close(dirs[1:], U, evals)
    # eigenvalues of the covariance, descending
    assert np.allclose(ev.cpu().numpy(), evals, rtol=1e-9, atol=1e-12 * abs(evals[0]))
    # canonical sign of the principal rows
    for r in range(1, m + 1):
        assert dirs[r][np.argmax(np.abs(dirs[r]))] > 0
    # projections against float64 products with the GPU's own directions
    for X, P in ((A, pA), (B, pB)):
        want = dirs @ X.astype(np.float64).T
        got = P.cpu().numpy()
        tol = 1e-6 * np.linalg.norm(X.astype(np.float64), axis=1).max() + 1e-30
        assert np.max(np.abs(got - want)) <= tol


def test_project_given_dirs():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("prohd_project given directions")
    A, B = synth.gauss_outliers(3001, 2999, 33, seed=4)   # D % 4 != 0 path
    g = np.random.default_rng(0)
    U = g.standard_normal((5, 33)).astype(np.float32)
    dirs, pA, pB, ev, st = ph.prohd_project(to_dev(torch, A), to_dev(torch, B), 4,
                                            dirs=to_dev(torch, U), sync=True)
    assert np.array_equal(dirs.cpu().numpy(), U)
    for X, P in ((A, pA), (B, pB)):
        want = U.astype(np.float64) @ X.astype(np.float64).T
        assert np.max(np.abs(P.cpu().numpy() - want)) <= 1e-5 * np.abs(want).max()


@pytest.mark.parametrize("D,m", [(64, 15), (256, 16), (256, 23), (64, 32), (256, 40), (50, 32),
                                 (50, 50), (256, 63)])
def test_project_direction_counts(D, m):
    """Every direction-group shape of the projection kernel: 16 or fewer,
    17 (one block and the extra direction), 18-32 (two blocks), 33 (two
    blocks and the extra direction), more than 33 (several launches); D not
    a multiple of 4 takes the scalar-load path.  Row counts leave ragged
    16-row blocks."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_project given directions D={D} ndirs={m + 1}")
    A, B = synth.gauss_outliers(2053, 1011, D, seed=m)
    g = np.random.default_rng(m)
    U = g.standard_normal((m + 1, D)).astype(np.float32)
    dirs, pA, pB, ev, st = ph.prohd_project(to_dev(torch, A), to_dev(torch, B), m,
                                            dirs=to_dev(torch, U), sync=True)
    assert int(st.item()) == 0
    for X, P in ((A, pA), (B, pB)):
        want = U.astype(np.float64) @ X.astype(np.float64).T
        bound = (D + 2) * 2.0 ** -24 * (np.abs(U).astype(np.float64) @ np.abs(X.astype(np.float64)).T)
        assert np.all(np.abs(P.cpu().numpy() - want) <= bound + 1e-30)


def test_project_identical_sets_fallback_axis():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("prohd_project identical sets -> e_1")
    A = synth.mixture(2000, 5, 16, seed=3, K=4)[0]
    d = to_dev(torch, A)
    dirs, _, _, _, st = ph.prohd_project(d, d, 2, sync=True)
    assert np.array_equal(dirs[0].cpu().numpy(), np.eye(16, dtype=np.float32)[0])


@pytest.mark.parametrize("kind,nA,nB,D", [("mix", 60000, 50000, 128), ("heavy", 40000, 30000, 256),
                                          ("gauss", 7000, 9000, 50)])
def test_project_is_reproducible(kind, nA, nB, D):
    """Two calls on the same input give the same bits: eigenvalues,
    directions and projections.  (The covariance reduction used to let two
    threads write the mirrored entries of a diagonal tile, whose matrix-core
    sums can differ in the last bit, so the eigenvalues changed from run to
    run at the 1e-15 level.)"""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_project reproducible {kind} {nA}x{nB}x{D}")
    if kind == "mix":
        A, B = synth.mixture(nA, nB, D, seed=5)
    elif kind == "heavy":
        A, B = synth.t_mixture(nA, nB, D, seed=5, nu=3.0)
    else:
        A, B = synth.gauss_outliers(nA, nB, D, seed=5)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    m = ph.default_m(D)
    runs = [ph.prohd_project(dA, dB, m, sync=True) for _ in range(3)]
    for d, pA, pB, ev, st in runs[1:]:
        assert torch.equal(ev, runs[0][3])
        assert torch.equal(d, runs[0][0])
        assert torch.equal(pA, runs[0][1]) and torch.equal(pB, runs[0][2])


def _check_selection(got, want, P64, ks):
    """Symmetric difference only at near-ties with a direction end's k-th value."""
    diff = np.setxor1d(got, want)
    if diff.size == 0:
        return
    near = np.zeros(diff.size, dtype=bool)
    for d in range(P64.shape[0]):
        p = P64[d]
        k = min(ks[d], p.size)
        srt = np.sort(p)
        for vk in (srt[k - 1], srt[-k]):
            near |= np.abs(p[diff] - vk) <= 1e-5 * max(abs(vk), 1e-30)
    assert near.all(), diff[~near]


@pytest.mark.parametrize("kind,nA,nB,D,m,k,seed", [
    # the 5 000 x 5 000, D = 32 workload on its ten seeds
    *[("gauss", 5000, 5000, 32, 3, 100, s) for s in range(10)],
    ("mix", 40000, 40000, 128, 8, 200, 0),
    ("heavy", 50000, 50000, 256, 16, None, 0),
])
def test_prohd_end_to_end(kind, nA, nB, D, m, k, seed):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd end-to-end {kind} nA={nA} D={D} m={m} k={k} seed={seed}")
    A, B = _data(kind, nA, nB, D, seed)
    kw = {"m": m, "k": k} if k is not None else {"m": m, "alpha": 0.01}
    r = ph.prohd(to_dev(torch, A), to_dev(torch, B), **kw)
    assert r["status"] == 0
    dirs = r["dirs"].cpu().numpy().astype(np.float64)
    # selection against the oracle on the same (GPU) directions
    o_same = oracle.prohd(A, B, dirs=dirs, m=m, **({"k": k} if k is not None else {"alpha": 0.01}))
    IA = r["idxA"][: int(r["nselA"].item())].cpu().numpy()
    IB = r["idxB"][: int(r["nselB"].item())].cpu().numpy()
    assert np.all(np.diff(IA) > 0) and np.all(np.diff(IB) > 0)
    _check_selection(IA, o_same["IA"], dirs @ A.astype(np.float64).T, o_same["kA"])
    _check_selection(IB, o_same["IB"], dirs @ B.astype(np.float64).T, o_same["kB"])
    # the value on the GPU's candidates, and against the oracle's own directions
    o_cand = oracle.subset_hd(A, B, IA, IB)
    assert rel(r["H"], o_cand["H"]) <= 1e-5
    o_own = oracle.prohd(A, B, **kw)
    assert rel(r["H"], o_own["H"]) <= 1e-4
    assert (r["nA_sel"], r["nB_sel"]) == (IA.size, IB.size)


@pytest.mark.parametrize("seed", range(10))
def test_gauss5k_exact_all_seeds(seed):
    """Exact distance (Eq. (1)) of the 5 000 x 5 000, D = 32 workload on its
    ten seeds, against the oracle at 1e-5."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"exact gauss5k seed={seed}")
    A, B = _data("gauss", 5000, 5000, 32, seed)
    o = oracle.exact_hd(A, B)
    r = ph.decode_result(ph.exact_hd(to_dev(torch, A), to_dev(torch, B), sync=True))
    assert r["status"] == 0 and rel(r["H"], o["H"]) <= 1e-5
    assert rel(r["hAB"], o["hAB"]) <= 1e-5 and rel(r["hBA"], o["hBA"]) <= 1e-5
