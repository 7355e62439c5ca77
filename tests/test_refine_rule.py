"""Which rows the distance search must re-measure: a CPU emulation (no GPU).

(The certified lower bound L and the rule "re-measure every row whose U
reaches the largest L" that the single-pair kernels follow are emulated at
the end of this file; the earlier rule, 256 rows first and then every row
whose U exceeds the largest re-measured minimum, is what the batched form
runs.)

The distance kernels search with the expanded form |x|^2 + |y|^2 - 2 x.y in
float32 (or on bfloat16 / e4m3 copies), then re-measure rows in float64.
This test emulates the float32 search with numpy's float32 arithmetic on a
case where the expansion cannot resolve the nearest-neighbour distances: a
cloud in [0, 100]^64 against a copy of itself moved by 0.01-0.02 per row,
one row moved by 0.05 (the directed distance is 0.05, Eq. (1)).

* Re-measuring only the 256 rows with the largest approximate minima misses
  the witness and returns a value far too low.
* The rule the kernels follow (rank rows by an upper bound U of their true
  minimum, derived from the float32 error of the expansion; re-measure the
  256 highest, then every other row whose U exceeds the largest re-measured
  minimum) returns the oracle's value exactly, and U bounds every row's true
  minimum.

The bound is written out here from its derivation, independently of the
HIP source; the reference values come from oracle.nn_dist (FP64).
"""

import math

import numpy as np
import pytest

import oracle

U_F32 = 2.0 ** -24


def min_upper(m2, S, K, uq=0.0, a=0.0, eta=0.0):
    """Upper bound of a row's true minimum distance from the approximate
    squared minimum m2 of the search and S >= |x| (see the module text of
    the distance kernels for the derivation)."""
    c = 2.0 * (K + 4) * U_F32
    rc = math.sqrt(c)
    p, b = 1.0 - uq, 2.0 * (uq * S + a)
    r, e = rc * (1.0 + uq), rc * (2.0 * (1.0 + uq) * S + 2.0 * a)
    den = p * p - r * r
    g = p * e + r * b
    return ((p * b + r * e) + np.sqrt(g * g + den * (m2 + eta))) / den


def perturbed_copy(n=8000, D=64, seed=0):
    g = np.random.default_rng(seed)
    A = g.uniform(0.0, 100.0, size=(n, D)).astype(np.float32)
    v = g.standard_normal((n, D))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    step = g.uniform(0.01, 0.02, size=n)
    j = int(g.integers(n))
    step[j] = 0.05
    B = (A.astype(np.float64) + v * step[:, None]).astype(np.float32)
    return A, B, j


def float32_search(X, Y):
    """Approximate squared row minima as the float32 tile forms them."""
    xn = np.einsum("ij,ij->i", X, X, dtype=np.float32)
    yn = np.einsum("ij,ij->i", Y, Y, dtype=np.float32)
    dot = X @ Y.T  # float32 product
    d2 = (xn[:, None] + yn[None, :]).astype(np.float32) - np.float32(2.0) * dot
    return np.maximum(d2.min(axis=1), np.float32(0.0)).astype(np.float64), xn


@pytest.fixture(scope="module")
def case():
    A, B, j = perturbed_copy()
    s = A[0]
    X = (A - s).astype(np.float32)   # the kernels shift both sets by one row of A
    Y = (B - s).astype(np.float32)
    m2, xn = float32_search(X, Y)
    nn, _ = oracle.nn_dist(X, Y)     # FP64 true minima of the shifted rows
    return X, Y, j, m2, xn, nn


def test_top_rows_alone_miss_the_witness(case):
    X, Y, j, m2, xn, nn = case
    h = nn.max()
    assert abs(h - 0.05) < 1e-4                       # the moved row decides Eq. (1)
    top = np.argsort(-m2, kind="stable")[:256]
    h_top = nn[top].max()
    assert j not in set(top.tolist())
    assert h_top < 0.5 * h                             # silently far too low


def test_bound_rule_returns_the_exact_value(case):
    X, Y, j, m2, xn, nn = case
    K = X.shape[1]
    S = np.sqrt(xn.astype(np.float64) * (1.0 + 2.0 * (K + 2) * U_F32))
    U = min_upper(m2, S, K)
    assert np.all(nn <= U * (1 + 1e-12))               # U bounds every true minimum
    order = np.lexsort((np.arange(U.size), -U))
    first = order[:256]
    h1 = nn[first].max()                               # first refinement
    rest = np.setdiff1d(np.arange(U.size), first)
    second = rest[U[rest] ** 2 > (h1 ** 2) * (1 - 2.0 ** -20)]
    h = max(h1, nn[second].max() if second.size else 0.0)
    assert h == nn.max()
    assert j in set(first.tolist()) | set(second.tolist())


def test_bound_is_tight_when_the_expansion_resolves_the_distances():
    """On ordinary data (nearest-neighbour distances comparable to the
    spread) the second pass is empty: the bound adds little to m2."""
    g = np.random.default_rng(3)
    A = g.standard_normal((3000, 32)).astype(np.float32)
    B = (g.standard_normal((2000, 32)) + 0.2).astype(np.float32)
    X = (A - A[0]).astype(np.float32)
    Y = (B - A[0]).astype(np.float32)
    m2, xn = float32_search(X, Y)
    nn, _ = oracle.nn_dist(X, Y)
    K = 32
    S = np.sqrt(xn.astype(np.float64) * (1.0 + 2.0 * (K + 2) * U_F32))
    U = min_upper(m2, S, K)
    assert np.all(nn <= U * (1 + 1e-12))
    assert np.all(U <= nn * 1.01 + 1e-3)
    order = np.lexsort((np.arange(U.size), -U))
    h1 = nn[order[:256]].max()
    rest = order[256:]
    assert not np.any(U[rest] ** 2 > h1 ** 2 * (1 - 2.0 ** -20))
    assert h1 == nn.max()


@pytest.mark.parametrize("uq, name", [(2.0 ** -8, "bf16"), (2.0 ** -3, "e4m3")])
def test_bound_covers_rounded_copies(uq, name):
    """The quantised forms: rows rounded to nearest with unit roundoff uq
    (8 significant bits for bfloat16, 4 for e4m3 in its normal range; the
    kernels' e4m3 constant is one unit in the last place, 2^-3, twice the
    round-to-nearest bound), searched with the float32 expansion; U bounds
    every true minimum."""
    g = np.random.default_rng(5)
    A = g.standard_normal((1500, 64)).astype(np.float32)
    B = (g.standard_normal((1200, 64)) * 1.1 + 0.1).astype(np.float32)
    X = (A - A[0]).astype(np.float32)
    Y = (B - A[0]).astype(np.float32)
    bits = 8 if name == "bf16" else 4

    def rnd(Z):
        m, e = np.frexp(Z.astype(np.float64))          # Z = m 2^e, 0.5 <= |m| < 1
        return (np.round(m * 2.0 ** bits) / 2.0 ** bits * 2.0 ** e).astype(np.float32)

    Xq, Yq = rnd(X), rnd(Y)
    assert np.all(np.abs(Xq.astype(np.float64) - X) <= 2.0 ** -bits * np.abs(X) * (1 + 1e-12))
    m2, _ = float32_search(Xq, Yq)
    xn = np.einsum("ij,ij->i", X, X, dtype=np.float32)
    nn, _ = oracle.nn_dist(X, Y)
    K = 64
    S = np.sqrt(xn.astype(np.float64) * (1.0 + 2.0 * (K + 2) * U_F32))
    U = min_upper(m2, S, K, uq=uq)
    assert np.all(nn <= U * (1 + 1e-12))


def test_pruned_rule_returns_the_exact_value():
    """The pruned search (PROHD_PRUNE): each row's float32 minimum over every
    16th row of the other set gives, through the same bound U, an upper bound
    of its minimum over the whole set; the 256 rows with the largest bounds
    are re-measured exactly, rows whose bound does not exceed the largest
    re-measured minimum are dropped, and the rest go through the full search
    and the bound rule.  On clustered data with a few far rows the rule
    returns the exact directed distance and drops most rows."""
    g = np.random.default_rng(11)
    A = (g.standard_normal((6000, 32)) * 0.3 + g.integers(0, 4, size=(6000, 1))).astype(np.float32)
    A[:20] += 6.0 * g.standard_normal((20, 32)).astype(np.float32)   # far rows: the witnesses
    B = (g.standard_normal((5000, 32)) * 0.3 + g.integers(0, 4, size=(5000, 1))).astype(np.float32)
    X = (A - A[0]).astype(np.float32)
    Y = (B - A[0]).astype(np.float32)
    K = 32
    nn, _ = oracle.nn_dist(X, Y)
    sub = Y[::16]
    m2s, xn = float32_search(X, sub)
    S = np.sqrt(xn.astype(np.float64) * (1.0 + 2.0 * (K + 2) * U_F32))
    Us = min_upper(m2s, S, K)
    assert np.all(nn <= Us * (1 + 1e-12))              # subset bound >= true minimum
    order = np.lexsort((np.arange(Us.size), -Us))
    first = order[:256]
    h1 = nn[first].max()
    rest = order[256:]
    keep = rest[Us[rest] ** 2 > h1 ** 2 * (1 - 2.0 ** -20)]
    assert keep.size < 0.5 * X.shape[0]                # most rows dropped
    m2f, _ = float32_search(X[keep], Y)
    Uf = min_upper(m2f, S[keep], K)
    second = keep[Uf ** 2 > h1 ** 2 * (1 - 2.0 ** -20)]
    h = max(h1, nn[second].max() if second.size else 0.0)
    assert h == nn.max()



def min_lower(m2, S, K, uq=0.0, a=0.0, eta=0.0):
    """Lower bound of a row's true minimum t' from the approximate squared
    minimum m2 (written out from its derivation, independently of the HIP
    source): for the true nearest row y', m2 <= d~(x, y') <= ((1 + uq) t' +
    b)^2 + (r t' + e)^2 + eta with b, r, e as in min_upper; the right side
    increases with t', so t' is at least the root of equality."""
    c = 2.0 * (K + 4) * U_F32
    rc = math.sqrt(c)
    P, b = 1.0 + uq, 2.0 * (uq * S + a)
    r, e = rc * (1.0 + uq), rc * (2.0 * (1.0 + uq) * S + 2.0 * a)
    w = np.asarray(m2 - eta - b * b - e * e, dtype=np.float64)
    A2, B1 = P * P + r * r, P * b + r * e
    out = np.zeros_like(w)
    pos = w > 0
    out[pos] = w[pos] / (B1[pos] + np.sqrt(B1[pos] ** 2 + A2 * w[pos])) if np.ndim(B1) else \
        w[pos] / (B1 + np.sqrt(B1 ** 2 + A2 * w[pos]))
    return out


def _bounds(X, Y, uq=0.0, Xq=None, Yq=None):
    K = X.shape[1]
    m2, _ = float32_search(X if Xq is None else Xq, Y if Yq is None else Yq)
    xn = np.einsum("ij,ij->i", X, X, dtype=np.float32)
    S = np.sqrt(xn.astype(np.float64) * (1.0 + 2.0 * (K + 2) * U_F32))
    return min_lower(m2, S, K, uq=uq), min_upper(m2, S, K, uq=uq)


def test_lower_bound_rule_on_the_moved_copy(case):
    """L <= true minimum <= U for every row; re-measuring the rows whose U
    reaches max L returns the exact directed distance (here nearly every row
    is re-measured: the expansion cannot resolve these distances)."""
    X, Y, j, m2, xn, nn = case
    L, U = _bounds(X, Y)
    assert np.all(L <= nn * (1 + 1e-12)) and np.all(nn <= U * (1 + 1e-12))
    keep = U >= L.max()
    assert keep[j]
    assert nn[keep].max() == nn.max()


def test_lower_bound_rule_is_tight_on_ordinary_data():
    """Clustered data with far rows: the rule keeps a handful of rows, the
    witness among them."""
    g = np.random.default_rng(12)
    A = (g.standard_normal((4000, 32)) * 0.3 + g.integers(0, 4, size=(4000, 1))).astype(np.float32)
    A[:15] += 5.0 * g.standard_normal((15, 32)).astype(np.float32)
    B = (g.standard_normal((3500, 32)) * 0.3 + g.integers(0, 4, size=(3500, 1))).astype(np.float32)
    X = (A - A[0]).astype(np.float32)
    Y = (B - A[0]).astype(np.float32)
    nn, _ = oracle.nn_dist(X, Y)
    L, U = _bounds(X, Y)
    assert np.all(L <= nn * (1 + 1e-12)) and np.all(nn <= U * (1 + 1e-12))
    keep = np.flatnonzero(U >= L.max())
    assert 1 <= keep.size <= 4, keep.size
    assert nn[keep].max() == nn.max()


@pytest.mark.parametrize("uq, bits", [(2.0 ** -8, 8), (2.0 ** -3, 4)])
def test_lower_bound_covers_rounded_copies(uq, bits):
    g = np.random.default_rng(13)
    A = g.standard_normal((1500, 64)).astype(np.float32)
    B = (g.standard_normal((1200, 64)) * 1.1 + 0.1).astype(np.float32)
    X = (A - A[0]).astype(np.float32)
    Y = (B - A[0]).astype(np.float32)

    def rnd(Z):
        m, e = np.frexp(Z.astype(np.float64))
        return (np.round(m * 2.0 ** bits) / 2.0 ** bits * 2.0 ** e).astype(np.float32)

    nn, _ = oracle.nn_dist(X, Y)
    L, U = _bounds(X, Y, uq=uq, Xq=rnd(X), Yq=rnd(Y))
    assert np.all(L <= nn * (1 + 1e-12)) and np.all(nn <= U * (1 + 1e-12))
    keep = U >= L.max()
    assert nn[keep].max() == nn.max()
