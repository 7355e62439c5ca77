"""Pins for the FP64 oracle: it is checked against things other than itself.

Each test names what fixes the expected value: brute force on tiny inputs,
an independent library routine, a closed form worked by hand, or a theorem of
the paper (Sec. II-E).  A plausible slip in the oracle -- a dropped term, a
wrong sign, a transposed operand, an off-by-one in ``k``, a wrong end of a sort
-- fails at least one of them.
"""

import math

import numpy as np
import pytest
from scipy.spatial.distance import directed_hausdorff
from sklearn.decomposition import PCA

import oracle
import synth


def _rand(seed, n, D, scale=1.0, shift=0.0):
    g = np.random.default_rng(seed)
    return (scale * g.standard_normal((n, D)) + shift).astype(np.float32)


# ---------------------------------------------------------------- Eq. (1)
@pytest.mark.parametrize("D", [1, 2, 3, 32])
def test_exact_matches_triple_loop_and_scipy(D):
    A = _rand(1 + D, 37, D)
    B = _rand(2 + D, 23, D, shift=0.3)
    r = oracle.exact_hd(A, B)
    vAB, ia, jb = oracle.directed_hd_bruteforce(A, B)
    vBA, ib, ja = oracle.directed_hd_bruteforce(B, A)
    assert abs(r["hAB"] - vAB) <= 1e-12 * vAB
    assert abs(r["hBA"] - vBA) <= 1e-12 * vBA
    assert (r["ab_a"], r["ab_b"], r["ba_b"], r["ba_a"]) == (ia, jb, ib, ja)
    # independent library: SciPy's early-break directed Hausdorff
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    assert abs(r["hAB"] - directed_hausdorff(A64, B64, seed=0)[0]) <= 1e-12 * vAB
    assert abs(r["hBA"] - directed_hausdorff(B64, A64, seed=0)[0]) <= 1e-12 * vBA
    assert r["H"] == max(r["hAB"], r["hBA"])


def test_exact_nn_arrays_match_bruteforce():
    A = _rand(5, 40, 4)
    B = _rand(6, 31, 4, scale=2.0)
    r = oracle.exact_hd(A, B, block_elems=64)  # many tiny blocks
    for i in range(A.shape[0]):
        d = np.sqrt(((A[i].astype(np.float64) - B.astype(np.float64)) ** 2).sum(1))
        assert r["nnA"][i] == pytest.approx(d.min(), rel=1e-13)
        assert r["argA"][i] == int(np.argmin(d))
    for j in range(B.shape[0]):
        d = np.sqrt(((B[j].astype(np.float64) - A.astype(np.float64)) ** 2).sum(1))
        assert r["nnB"][j] == pytest.approx(d.min(), rel=1e-13)


def test_exact_hand_example():
    # A = {0, 10}, B = {1, 2, 3} on a line: h(A,B) = max(1, 7) = 7 (10 -> 3),
    # h(B,A) = max(1, 2, 3) = 3 (3 -> 0); H = 7.
    r = oracle.exact_hd([[0.0], [10.0]], [[1.0], [2.0], [3.0]])
    assert (r["hAB"], r["hBA"], r["H"]) == (7.0, 3.0, 7.0)
    assert (r["ab_a"], r["ab_b"], r["ba_b"], r["ba_a"]) == (1, 2, 2, 0)


def test_identical_and_permuted_sets_give_zero():
    A = _rand(7, 300, 8)
    perm = np.random.default_rng(0).permutation(300)
    for B in (A, A[perm]):
        assert oracle.exact_hd(A, B)["H"] == 0.0
        assert oracle.prohd(A, B, k=5, m=2)["H"] == 0.0


def test_symmetry():
    A = _rand(8, 400, 6)
    B = _rand(9, 350, 6, shift=0.4)
    r1, r2 = oracle.exact_hd(A, B), oracle.exact_hd(B, A)
    assert r1["H"] == r2["H"] and r1["hAB"] == r2["hBA"]
    p1 = oracle.prohd(A, B, k=7, m=2)
    p2 = oracle.prohd(B, A, k=7, m=2)
    assert p1["H"] == p2["H"]
    assert np.array_equal(p1["IA"], p2["IB"]) and np.array_equal(p1["IB"], p2["IA"])


def test_rigid_motion_invariance():
    A = _rand(10, 500, 5, scale=[3.0, 2.0, 1.5, 1.0, 0.5])
    B = _rand(11, 450, 5, scale=[3.0, 2.0, 1.5, 1.0, 0.5], shift=0.7)
    g = np.random.default_rng(3)
    Q, R = np.linalg.qr(g.standard_normal((5, 5)))
    Q = Q * np.sign(np.diag(R))
    t = g.standard_normal(5) * 4.0
    A2 = A.astype(np.float64) @ Q.T + t
    B2 = B.astype(np.float64) @ Q.T + t
    assert oracle.exact_hd(A2, B2)["H"] == pytest.approx(oracle.exact_hd(A, B)["H"], rel=1e-10)
    p1 = oracle.prohd(A, B, k=12, m=2)
    p2 = oracle.prohd(A2, B2, k=12, m=2)
    assert np.array_equal(p1["IA"], p2["IA"]) and np.array_equal(p1["IB"], p2["IB"])
    assert p2["H"] == pytest.approx(p1["H"], rel=1e-10)


# ------------------------------------------------- closed forms and examples
@pytest.mark.parametrize("D", [3, 16, 64])
def test_concentric_shells_closed_form(D):
    # A on the unit sphere, B the same directions at radius 2, permuted:
    # every a has its partner 2a at distance 1 and no point of B is closer
    # (reverse triangle inequality), so H = 1; the selections correspond
    # because B's projections are exactly twice A's, hence H_hat = 1 too.
    # The float32 rows are unit vectors only to within rounding, so the bound
    # is |H - 1| <= 3 * max_i | |a_i| - 1 | (partner distance |a_i|, any other
    # b at least 2|a_j| - |a_i|).
    A, B = synth.shells(2000, D, seed=D, r1=1.0, r2=2.0)
    dev = np.abs(np.linalg.norm(A.astype(np.float64), axis=1) - 1.0).max()
    tol = 3 * dev + 1e-13
    assert abs(oracle.exact_hd(A, B)["H"] - 1.0) <= tol
    p = oracle.prohd(A, B, alpha=0.05)
    assert abs(p["H"] - 1.0) <= tol
    assert p["nA_sel"] == p["nB_sel"]


def test_full_selection_reduces_to_exact():
    A = _rand(12, 101, 4)
    B = _rand(13, 80, 4, shift=0.2)
    p = oracle.prohd(A, B, k=51, m=2)  # k >= ceil(n/2) keeps every row
    assert p["nA_sel"] == 101 and p["nB_sel"] == 80
    assert p["H"] == oracle.exact_hd(A, B)["H"]


def test_counterexample_1d_overestimates():
    # D=1, alpha=0.4: centroids coincide (both 5) -> axis e_1; m = 1, alpha' = 0.4;
    # k = floor(0.4*5) = 2 per end.  A_sel = {0, 4.9, 5.1, 10}, B_sel = {0, 1, 9, 10}.
    # h(A_sel,B_sel) = 3.9 (4.9 -> 1, 5.1 -> 9); h(B_sel,A_sel) = 1; H_hat = 3.9.
    # Exact: h(A,B) = 0.1, h(B,A) = 1 (1 -> 0, 9 -> 10): H = 1.
    A = np.array([[0.0], [4.9], [5.0], [5.1], [10.0]])
    B = np.array([[0.0], [1.0], [5.0], [9.0], [10.0]])
    for X, Y in ((A, B), (B, A)):
        p = oracle.prohd(X, Y, alpha=0.4)
        assert p["H"] == pytest.approx(3.9, abs=1e-12)
        assert (p["nA_sel"], p["nB_sel"]) == (4, 4)
        assert oracle.exact_hd(X, Y)["H"] == pytest.approx(1.0, abs=1e-12)
    p = oracle.prohd(A, B, alpha=0.4)
    assert list(p["IA"]) == [0, 1, 3, 4] and list(p["IB"]) == [0, 1, 3, 4]


def test_composition_2d_hand_example():
    # Centroids (0,0) and (0,1.4): centroid axis (0,1).  PC1 of the union is
    # within 0.01 rad of (1,0) (x variance ~50, xy covariance ~ -0.4).
    # alpha = 0.2, m = 1, k = 1 per end on both directions:
    #   axis (0,1):  A bottom/top = rows 3/1, B bottom/top = rows 3/2;
    #   PC1:         rows 0/4 in both sets.
    # I_A = {0,1,3,4}, I_B = {0,2,3,4}.  Worked distances:
    #   h(A_sel,B_sel) = |(-5,0.2)-(-10,1)| = sqrt(25.64)
    #   h(B_sel,A_sel) = |(0,3)-(-5,0.2)|   = sqrt(32.84)   -> H_hat
    #   exact H = 3 ((0,0) <-> (0,3)).
    A = np.array([[-10, 0], [-5, 0.2], [0, 0], [5, -0.2], [10, 0]])
    B = np.array([[-10, 1], [-5, 1.2], [0, 3], [5, 0.8], [10, 1]])
    p = oracle.prohd(A, B, alpha=0.2)
    assert np.allclose(p["dirs"][0], [0, 1])
    assert abs(p["dirs"][1][0]) > 0.9999
    assert list(p["IA"]) == [0, 1, 3, 4] and list(p["IB"]) == [0, 2, 3, 4]
    assert p["hAB"] == pytest.approx(math.sqrt(25.64), rel=1e-14)
    assert p["hBA"] == pytest.approx(math.sqrt(32.84), rel=1e-14)
    assert (p["ba_b"], p["ba_a"]) == (2, 1)
    assert oracle.exact_hd(A, B)["H"] == pytest.approx(3.0, rel=1e-14)
    full = oracle.prohd(A, B, alpha=0.2, inner="full")
    # outer max over candidates, inner min over all rows: (0,3) -> (0,0) = 3
    assert full["H"] == pytest.approx(3.0, rel=1e-14)


# ------------------------------------------------------------ Alg. 1 pieces
def test_k_rule():
    assert oracle.k_rule(0.01, 2_000_000) == 20_000
    assert oracle.k_rule(0.01 / 16, 2_000_000) == 1_250
    assert oracle.k_rule(0.29, 100) == 29   # 0.29*100 = 28.999... in binary
    assert oracle.k_rule(0.01, 50) == 1     # max(1, .)
    assert oracle.k_rule(0.9, 3) == 2
    assert oracle.k_rule(5.0, 3) == 3       # clipped to n


def test_centroid_direction_closed_form():
    A = _rand(14, 64, 3)
    t = np.array([3.0, -4.0, 0.0])
    u = oracle.centroid_direction(A, A.astype(np.float64) + t)
    assert np.allclose(u, [0.6, -0.8, 0.0], atol=1e-12)   # ybar - xbar, not reversed
    assert np.array_equal(oracle.centroid_direction(A, A), [1.0, 0.0, 0.0])  # e_1 fallback
    tiny = A.astype(np.float64) + 1e-11
    assert np.array_equal(oracle.centroid_direction(A, tiny), [1.0, 0.0, 0.0])


def test_extreme_indices_against_rank_definition():
    # Brute force: the rank of i under (value, index) is the number of j that
    # precede it; the k smallest are rank < k, the k largest have descending
    # rank < k.  Integer-valued data forces many ties.
    g = np.random.default_rng(15)
    for trial in range(40):
        n = int(g.integers(1, 30))
        p = g.integers(-3, 4, size=n).astype(np.float64)
        if trial % 5 == 0:
            p[p == 0] = -0.0
        k = int(g.integers(1, n + 3))
        want = set()
        for i in range(n):
            asc = sum(1 for j in range(n) if (p[j], j) < (p[i], i))
            desc = sum(1 for j in range(n) if (-p[j], j) < (-p[i], i))
            if asc < min(k, n) or desc < min(k, n):
                want.add(i)
        got = oracle.extreme_indices(p, k)
        assert sorted(want) == list(got), (p, k)
        assert list(got) == list(oracle.extreme_indices(-p, k))  # end symmetry


def test_largest_indices_against_rank_definition():
    # Brute force as above, the largest end alone: i is kept when fewer than
    # k entries precede it in (-value, index); empty input and k = 0 keep none.
    g = np.random.default_rng(16)
    for trial in range(40):
        n = int(g.integers(0, 30))
        p = g.integers(-3, 4, size=n).astype(np.float64)
        if trial % 4 == 0:
            p[p == 0] = -0.0
        if trial % 7 == 0 and n:
            p[g.integers(0, n)] = np.inf
        k = int(g.integers(0, n + 3))
        want = [i for i in range(n)
                if sum(1 for j in range(n) if (-p[j], j) < (-p[i], i)) < min(k, n)]
        assert list(oracle.largest_indices(p, k)) == want, (p, k)


def test_select_union_over_directions():
    P = np.array([[5.0, 1.0, 3.0, 2.0, 4.0], [0.0, 9.0, 8.0, 7.0, 6.0]])
    IA, IB = oracle.select(P, P[::-1], [1, 1], [2, 1])
    # dir0 k=1: min idx1, max idx0; dir1 k=1: min idx0, max idx1 -> {0,1}
    assert list(IA) == [0, 1]
    # B: dir0 = P[1] k=2: min {0,4}, max {1,2}; dir1 = P[0] k=1: {1,0}
    assert list(IB) == [0, 1, 2, 4]


# ------------------------------------------------------------ Alg. 2 pieces
def test_principal_directions_match_sklearn():
    g = np.random.default_rng(16)
    scales = np.array([9.0, 6.0, 4.0, 2.5, 1.0, 0.5])
    A = (g.standard_normal((700, 6)) * scales + 50.0).astype(np.float32)  # far from origin
    B = (g.standard_normal((500, 6)) * scales + 51.0).astype(np.float32)
    U, ev = oracle.principal_directions(A, B, 4)
    Z = np.vstack([A, B]).astype(np.float64)
    ref = PCA(n_components=4, svd_solver="full").fit(Z)
    for r in range(4):
        assert abs(U[r] @ ref.components_[r]) == pytest.approx(1.0, abs=1e-10)
    assert np.allclose(ev[:4], ref.explained_variance_, rtol=1e-10)
    assert np.all(np.diff(ev) <= 0)
    assert np.allclose(U @ U.T, np.eye(4), atol=1e-12)
    for r in range(4):  # canonical sign
        assert U[r][np.argmax(np.abs(U[r]))] > 0


# ------------------------------------------------------- Sec. II-E theorems
def test_projected_hd_matches_bruteforce():
    g = np.random.default_rng(17)
    pa, pb = g.standard_normal(40), g.standard_normal(27) + 0.5
    want = max(max(min(abs(a - b) for b in pb) for a in pa), max(min(abs(a - b) for a in pa) for b in pb))
    assert oracle.hd_1d(pa, pb) == pytest.approx(want, abs=1e-15)


def test_delta_closed_form():
    A = np.array([[1.0, 0.0], [2.0, 0.0]])
    B = np.array([[0.0, 1.0], [3.0, -2.0]])
    assert oracle.delta(A, B, [1.0, 0.0]) == pytest.approx(2.0)
    assert oracle.delta(A, B, [0.0, 1.0]) == pytest.approx(3.0)


def test_bounds_theorems_random():
    g = np.random.default_rng(18)
    for trial in range(6):
        D = [2, 3, 5, 8, 16, 4][trial]
        A = g.standard_normal((300, D)) * g.uniform(0.2, 3, D)
        B = g.standard_normal((260, D)) * g.uniform(0.2, 3, D) + g.standard_normal(D)
        H = oracle.exact_hd(A, B)["H"]
        U = g.standard_normal((5, D))
        U /= np.linalg.norm(U, axis=1, keepdims=True)
        for u in U:
            Hu = oracle.hd_1d(A @ u, B @ u)
            assert Hu <= H + 1e-12
            assert H <= Hu + 2 * oracle.delta(A, B, u) + 1e-12
        assert oracle.hd_directions(A, B, U[:2]) <= oracle.hd_directions(A, B, U) + 1e-15
        assert oracle.hd_directions(A, B, U) <= H + 1e-12
        # outer max over candidates, inner min over all: never above H,
        # and monotone as candidates are added
        prev = 0.0
        for k in (1, 5, 20, 150):
            f = oracle.prohd(A, B, k=k, m=1, inner="full")["H"]
            assert f <= H + 1e-12
            assert f >= prev - 1e-15
            prev = f


def test_delta_through_a_point_and_certificate():
    # delta about a line through c equals delta about the origin after
    # translating both sets by -c (hand values), and the certificate's
    # interval contains the exact distance for lines through any point
    A = np.array([[1.0, 0.0], [2.0, 0.0]])
    B = np.array([[0.0, 1.0], [3.0, -2.0]])
    c = np.array([0.5, -1.0])
    assert oracle.delta(A, B, [1.0, 0.0], c) == pytest.approx(2.0)     # |y - (-1)| max: B[0]
    assert oracle.delta(A, B, [0.0, 1.0], c) == pytest.approx(2.5)     # |x - 0.5| max: B[1]
    assert oracle.delta(A + 7.0, B + 7.0, [1.0, 0.0], c + 7.0) == pytest.approx(2.0)
    g = np.random.default_rng(19)
    for trial in range(5):
        D = [2, 3, 6, 10, 4][trial]
        A = g.standard_normal((200, D)) * g.uniform(0.3, 2, D) + 5.0
        B = g.standard_normal((180, D)) * g.uniform(0.3, 2, D) + 5.0 + g.standard_normal(D)
        H = oracle.exact_hd(A, B)["H"]
        U = g.standard_normal((4, D))
        for cc in (None, np.vstack([A, B]).mean(0), g.standard_normal(D) * 3):
            cert = oracle.certificate(A, B, U, cc)
            assert cert["lb"] <= H + 1e-12 <= cert["ub"] + 2e-12
        # the centroid line is at least as tight as the origin line here
        assert oracle.certificate(A, B, U, np.vstack([A, B]).mean(0))["ub"] <= \
            oracle.certificate(A, B, U)["ub"] + 1e-12


# ------------------------------------------------ learned-proposal scorer
def test_mlp_finite_differences():
    # the manual backward of the FP64 scorer against central differences
    from oracle import mlp
    D = 3
    g = np.random.default_rng(21)
    p = g.standard_normal(mlp.param_count(D)) * 0.2
    F = mlp.features(g.standard_normal((7, D)), g.standard_normal(D))
    y = np.array([1, 0, 0, 1, 0, 0, 0], dtype=np.float64)
    loss, grad = mlp.loss_grad(p, F, y, D, pos_weight=3.0)
    idx = g.choice(p.size, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_grad(p + e, F, y, D, 3.0)[0] - mlp.loss_grad(p - e, F, y, D, 3.0)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])) + 1e-9, (i, fd, grad[i])


def test_mlp_hand_example():
    # all weights zero except b3 = s0: every score is s0, the loss is
    # pw*y*softplus(-s0) + (1-y)*softplus(s0); only b3 has a gradient,
    # mean(pw*y*(sig-1) + (1-y)*sig)
    from oracle import mlp
    D = 2
    p = np.zeros(mlp.param_count(D))
    p[-1] = 0.3
    F = mlp.features(np.ones((4, D)), np.zeros(D))
    y = np.array([1.0, 0.0, 0.0, 0.0])
    loss, grad = mlp.loss_grad(p, F, y, D, pos_weight=2.0)
    sig = 1.0 / (1.0 + math.exp(-0.3))
    want = (2.0 * math.log1p(math.exp(-0.3)) + 3 * math.log1p(math.exp(0.3))) / 4
    assert loss == pytest.approx(want, rel=1e-14)
    assert grad[-1] == pytest.approx((2.0 * (sig - 1.0) + 3 * sig) / 4, rel=1e-14)
    assert np.count_nonzero(grad[:-1]) == 0
    # features of a point: [x, x - c]
    assert np.array_equal(mlp.features([[1.0, 2.0]], [0.5, -1.0]), [[1.0, 2.0, 0.5, 3.0]])


def test_adamw_first_step():
    # first step moves each weight by lr * sign(g) (bias-corrected m/sqrt v = g/|g|) plus decay
    from oracle import mlp
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -4.0])
    p2, m, v = mlp.adamw(p, g, np.zeros(2), np.zeros(2), t=1, lr=0.1, wd=0.01, eps=0.0)
    assert np.allclose(p2, p - 0.1 * (np.sign(g) + 0.01 * p), rtol=1e-14)


def test_certificate_hand_example():
    # A = {(0,0), (4,0)}, B = {(0,3), (4,0)}, directions e1 and e2, spread
    # measured from the origin line (Eq. (2)).
    #   e1: projections A {0, 4}, B {0, 4}  -> H_e1 = 0;  delta(e1) = 3 (point (0,3))
    #   e2: projections A {0, 0}, B {3, 0}  -> H_e2 = 3;  delta(e2) = 4 (point (4,0))
    # Sec. II-E: lb = max_u H_u = 3, ub = min_u (H_u + 2 delta(u)) = min(6, 11) = 6,
    # around H = 3 (each point's nearest neighbour in the other set is at 0 or 3).
    A = [[0.0, 0.0], [4.0, 0.0]]
    B = [[0.0, 3.0], [4.0, 0.0]]
    c = oracle.certificate(A, B, [[1.0, 0.0], [0.0, 1.0]])
    assert list(c["hu"]) == [0.0, 3.0] and list(c["delta"]) == [3.0, 4.0]
    assert (c["lb"], c["ub"]) == (3.0, 6.0)
    assert oracle.exact_hd(A, B)["H"] == 3.0


@pytest.mark.parametrize("nA,nB,D,br,bc", [(300, 250, 5, 64, 37), (97, 130, 3, 1000, 1000),
                                           (40, 700, 17, 7, 128)])
def test_one_pass_matches_per_direction_search(nA, nB, D, br, bc):
    """Both directions' minima from one pass (nn_both) equal the brute-force
    nearest neighbours, blocks of any shape, ties to the smallest index."""
    A = _rand(20 + D, nA, D)
    B = _rand(21 + D, nB, D, shift=0.2)
    B[5] = A[3]
    B[9] = A[3]              # tie in A's row 3, and between B rows 5 and 9
    A[11] = A[12]            # equal A rows: ties for the column minima
    dA, jA, dB, iB = oracle.nn_both(A, B, block_rows=br, block_cols=bc)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    for i in range(nA):
        d = np.sqrt(((A64[i] - B64) ** 2).sum(1))
        assert jA[i] == int(np.argmin(d)) and dA[i] == pytest.approx(d.min(), rel=1e-13, abs=1e-300)
    for j in range(nB):
        d = np.sqrt(((B64[j] - A64) ** 2).sum(1))
        assert iB[j] == int(np.argmin(d)) and dB[j] == pytest.approx(d.min(), rel=1e-13, abs=1e-300)
    r1, r2 = oracle.exact_hd(A, B), oracle.exact_hd(A, B, one_pass=True)
    for k in ("H", "hAB", "hBA", "ab_a", "ab_b", "ba_b", "ba_a"):
        assert r1[k] == r2[k]


def test_adaptive_alpha_on_a_line_stops_certified():
    """D = 1: every direction is the line itself, delta(u) = 0, so the
    Sec. II-E bounds close: H_U = H = ub, and the schedule stops at once
    with the certified-gap rule and the exact value."""
    g = np.random.default_rng(31)
    A = g.uniform(0, 10, size=(500, 1)).astype(np.float32)
    B = g.uniform(1, 12, size=(400, 1)).astype(np.float32)
    H = oracle.exact_hd(A, B)["H"]
    r = oracle.adaptive_alpha(A, B, alpha0=0.01, tol=1e-9)
    assert (r["reason"], r["steps"]) == (1, 1)
    assert r["lb"] == pytest.approx(H, rel=1e-12) and r["ub"] == pytest.approx(H, rel=1e-12)
    assert r["H"] <= H * (1 + 1e-12)


def test_adaptive_alpha_schedule_on_random_clouds():
    """The paper's random clouds (U[0,1]^D against the same plus 0.1): the
    returned value is the inner-full value at the last alpha, never above H;
    the values are non-decreasing (nested candidate sets); the stop is the
    first step whose gain is within tol, else alpha_max; the Sec. II-E
    upper bound is far from H here, so the certified rule does not fire."""
    A, B = synth.uniform_clouds(2000, 2000, 4, seed=3)
    H = oracle.exact_hd(A, B)["H"]
    tol = 1e-3
    r = oracle.adaptive_alpha(A, B, alpha0=0.005, growth=2.0, alpha_max=0.32, tol=tol)
    v = r["values"]
    assert r["reason"] in (2, 3) and r["steps"] == len(v)
    assert all(b >= a for a, b in zip(v, v[1:]))
    assert r["H"] == v[-1] <= H * (1 + 1e-12) and r["ub"] > 1.5 * H
    assert r["alpha"] == min(0.005 * 2.0 ** (len(v) - 1), 0.32)
    for j in range(1, len(v) - 1):
        assert v[j] - v[j - 1] > tol * v[j]
    if r["reason"] == 2:
        assert v[-1] - v[-2] <= tol * v[-1]
    full = oracle.prohd(A, B, alpha=r["alpha"], inner="full")
    assert full["H"] == r["H"] and full["nA_sel"] == r["nA_sel"]


def test_adaptive_alpha_full_selection_is_exact():
    """alpha0 = alpha_max = 0.5: every row is a candidate (k >= n / 2 per
    end), so the single step returns H itself (reason 3)."""
    A, B = synth.uniform_clouds(600, 500, 3, seed=5)
    H = oracle.exact_hd(A, B)["H"]
    r = oracle.adaptive_alpha(A, B, alpha0=0.5, alpha_max=0.5, tol=0.0)
    assert (r["reason"], r["steps"], r["nA_sel"], r["nB_sel"]) == (3, 1, 600, 500)
    assert r["H"] == H
