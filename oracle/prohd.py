"""ProHD (projection-based Hausdorff approximation), FP64 -- test infrastructure only.

Follows the paper's three algorithms in their order and notation:

* Alg. 1 (CentroidIndices): centroids of the two sets, the axis
  ``u = ybar - xbar`` (replaced by ``e_1`` when its norm is below 1e-9, else
  normalised), projections of both sets, and per set the ``k`` smallest and
  ``k`` largest projections with ``k = max(1, floor(alpha * n))``.
* Alg. 2 (PCAProjIndices): the top ``m`` principal components of the stacked
  union ``[X; Y]``, each normalised, and the same extreme selection per
  component.
* Alg. 3 (ProjHausdorff): ``m = floor(sqrt(D))``, ``alpha' = alpha / m`` on the
  principal components, union of all kept indices, and the full-dimensional
  Hausdorff distance of the two selected subsets.

Readings where the paper is silent, ambiguous or inconsistent:

R1  The value ProHD returns is Alg. 3's ``H(A_sel, B_sel)``.  The paper's
    claims that this equals ``H_U`` and never exceeds ``H`` do not hold for
    it (restricting the inner minimum to ``B_sel`` can raise it); the
    theorem ``H_U <= H`` is about the projected distance only.
R2  Principal components are eigenvectors of the centred covariance of the
    union (exact eigendecomposition, not a randomised SVD).  Descending
    eigenvalue order; sign fixed so the largest-magnitude component is
    positive (first index on ties).  The sign cannot change a selection.
R3  Ties in the projections are broken by the total order (value, index) at
    both ends: the k smallest are the first k of that order, the k largest
    are the first k of (-value, index).  -0.0 equals +0.0.
R4  ``k`` counts per end per set; ``k <= n`` is enforced by ``min(k, n)``.
    In alpha mode ``floor`` is taken of ``alpha * n + 1e-9`` so that a decimal
    alpha does not lose an integer to binary rounding.
R5  The 1e-9 threshold of the centroid fallback is absolute, in FP64.
R6  Explicit mode: a caller may give ``k`` per direction instead of ``alpha``
    (the same ``k`` at both ends and for every direction unless a list is
    given), and may inject directions.
"""

from __future__ import annotations

import math

import numpy as np

from .hausdorff import exact_hd, nn_dist

__all__ = [
    "k_rule",
    "centroid_direction",
    "principal_directions",
    "canonical_sign",
    "extreme_indices",
    "largest_indices",
    "select",
    "subset_hd",
    "prohd",
    "adaptive_alpha",
]


def _f64(X) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim == 1:
        X = X[:, None]
    return np.ascontiguousarray(X, dtype=np.float64)


def k_rule(alpha: float, n: int) -> int:
    """k = max(1, floor(alpha * n)) of Alg. 1 / Alg. 2, clipped to n (R4)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    return min(n, max(1, int(math.floor(alpha * n + 1e-9))))


def centroid_direction(A, B) -> np.ndarray:
    """Alg. 1 with X = A, Y = B (as Alg. 3 calls it): unit ``ybar - xbar``.

    Falls back to the first basis vector ``e_1`` when ``||ybar - xbar||`` is
    below 1e-9 (absolute, R5).
    """
    A = _f64(A)
    B = _f64(B)
    u = B.mean(axis=0) - A.mean(axis=0)
    nrm = float(np.sqrt(u @ u))
    if nrm < 1e-9:
        e1 = np.zeros_like(u)
        e1[0] = 1.0
        return e1
    return u / nrm


def canonical_sign(v) -> np.ndarray:
    """Flip ``v`` so that its largest-magnitude entry is positive (R2)."""
    v = np.asarray(v, dtype=np.float64)
    i = int(np.argmax(np.abs(v)))
    return -v if v[i] < 0 else v.copy()


def principal_directions(A, B, m: int):
    """Alg. 2's first two steps: top-m principal components of [A; B].

    Returns ``(U, evals)`` where ``U`` is ``m x D`` (unit rows, descending
    eigenvalue, canonical sign) and ``evals`` all eigenvalues of the
    covariance in descending order (for eigengap reporting).
    """
    Z = np.vstack([_f64(A), _f64(B)])
    n, D = Z.shape
    if not 1 <= m <= D:
        raise ValueError("need 1 <= m <= D")
    Zc = Z - Z.mean(axis=0)
    C = (Zc.T @ Zc) / max(n - 1, 1)
    w, V = np.linalg.eigh(C)
    order = np.argsort(-w, kind="stable")
    U = np.empty((m, D))
    for r, c in enumerate(order[:m]):
        v = V[:, c] / np.linalg.norm(V[:, c])
        U[r] = canonical_sign(v)
    return U, w[order]


def largest_indices(p, k: int) -> np.ndarray:
    """Indices of the k largest entries of ``p`` (R3: the first k of the
    order (-value, index); -0.0 equals +0.0), ascending.  ``k`` is clipped to
    the length; an empty array or ``k = 0`` gives no index."""
    p = np.asarray(p, dtype=np.float64).ravel()
    if np.isnan(p).any():
        raise ValueError("NaN entry")
    k = min(int(k), p.size)
    if k <= 0:
        return np.zeros(0, dtype=np.int64)
    p = p + 0.0  # -0.0 -> +0.0
    return np.sort(np.lexsort((np.arange(p.size), -p))[:k])


def extreme_indices(p, k: int) -> np.ndarray:
    """Indices of the k smallest and k largest entries of ``p`` (R3), unioned.

    Returns the sorted unique indices (Alg. 1's "keep the unique indices").
    """
    p = np.asarray(p, dtype=np.float64).ravel()
    n = p.size
    if n == 0:
        raise ValueError("empty projection")
    if np.isnan(p).any():
        raise ValueError("NaN projection")
    k = min(int(k), n)
    if k < 1:
        raise ValueError("k must be >= 1")
    p = p + 0.0  # -0.0 -> +0.0
    idx = np.arange(n)
    bottom = np.lexsort((idx, p))[:k]
    return np.union1d(bottom, largest_indices(p, k))


def select(projA, projB, kA, kB):
    """Union over directions of the per-direction extremes (Alg. 2, Alg. 3).

    ``projA`` is ``ndirs x nA`` (one row per direction), likewise ``projB``;
    ``kA``/``kB`` are per-direction counts.  Returns sorted unique
    ``(IA, IB)`` as int64 arrays.
    """
    projA = np.atleast_2d(np.asarray(projA, dtype=np.float64))
    projB = np.atleast_2d(np.asarray(projB, dtype=np.float64))
    IA = np.zeros(0, dtype=np.int64)
    IB = np.zeros(0, dtype=np.int64)
    for d in range(projA.shape[0]):
        IA = np.union1d(IA, extreme_indices(projA[d], kA[d]))
        IB = np.union1d(IB, extreme_indices(projB[d], kB[d]))
    return IA.astype(np.int64), IB.astype(np.int64)


def subset_hd(A, B, IA, IB, inner: str = "candidates"):
    """Hausdorff distance over selected rows, witnesses as ORIGINAL indices.

    ``inner="candidates"``: Alg. 3's ``H(A_sel, B_sel)`` (both minima over
    the selected rows only).  ``inner="full"``: ``max{h(A_sel, B),
    h(B_sel, A)}`` -- outer maximum over the candidates, inner minimum over
    the whole other set, hence never above ``H(A,B)``.
    """
    A = _f64(A)
    B = _f64(B)
    IA = np.asarray(IA, dtype=np.int64)
    IB = np.asarray(IB, dtype=np.int64)
    if inner == "candidates":
        r = exact_hd(A[IA], B[IB])
        return {
            "H": r["H"], "hAB": r["hAB"], "hBA": r["hBA"],
            "ab_a": int(IA[r["ab_a"]]), "ab_b": int(IB[r["ab_b"]]),
            "ba_b": int(IB[r["ba_b"]]), "ba_a": int(IA[r["ba_a"]]),
        }
    if inner == "full":
        dA, aA = nn_dist(A[IA], B)
        dB, aB = nn_dist(B[IB], A)
        ia, ib = int(np.argmax(dA)), int(np.argmax(dB))
        hAB, hBA = float(dA[ia]), float(dB[ib])
        return {
            "H": max(hAB, hBA), "hAB": hAB, "hBA": hBA,
            "ab_a": int(IA[ia]), "ab_b": int(aA[ia]),
            "ba_b": int(IB[ib]), "ba_a": int(aB[ib]),
        }
    raise ValueError("inner must be 'candidates' or 'full'")


def prohd(A, B, alpha: float = 0.01, m: int | None = None, k=None,
          dirs=None, inner: str = "candidates"):
    """ProjHausdorff (Alg. 3) end to end.

    alpha mode (default): ``m = floor(sqrt(D))``; the centroid axis keeps
    ``k_rule(alpha, n)`` per end, each principal component
    ``k_rule(alpha / m, n)`` per end, per set.
    explicit mode: ``k`` is an int (same for every direction end) or a list of
    ``m + 1`` ints; ``m`` must then be given or defaults to floor(sqrt(D)).
    ``dirs`` (``(m+1) x D``, row 0 the centroid axis) injects directions
    instead of computing them (R6).

    Returns a dict with ``H, hAB, hBA`` (Euclidean), witnesses (original
    indices), ``IA, IB`` (sorted unique), ``nA_sel, nB_sel``, ``dirs``, the
    ``kA, kB`` lists and the covariance eigenvalues when computed.
    """
    A = _f64(A)
    B = _f64(B)
    nA, D = A.shape
    nB = B.shape[0]
    if B.shape[1] != D:
        raise ValueError("A and B must have the same dimension")
    if nA < 1 or nB < 1:
        raise ValueError("empty set")
    if m is None:
        m = math.isqrt(D) if dirs is None else np.atleast_2d(dirs).shape[0] - 1
    evals = None
    if dirs is None:
        u0 = centroid_direction(A, B)
        P, evals = principal_directions(A, B, m)
        U = np.vstack([u0[None, :], P])
    else:
        U = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
        if U.shape != (m + 1, D):
            raise ValueError("dirs must be (m+1) x D")
    if k is None:
        kA = [k_rule(alpha, nA)] + [k_rule(alpha / m, nA)] * m
        kB = [k_rule(alpha, nB)] + [k_rule(alpha / m, nB)] * m
    else:
        ks = [int(k)] * (m + 1) if np.isscalar(k) else [int(x) for x in k]
        if len(ks) != m + 1:
            raise ValueError("k list must have m+1 entries")
        kA = [min(max(1, x), nA) for x in ks]
        kB = [min(max(1, x), nB) for x in ks]
    projA = U @ A.T
    projB = U @ B.T
    IA, IB = select(projA, projB, kA, kB)
    r = subset_hd(A, B, IA, IB, inner=inner)
    r.update({
        "IA": IA, "IB": IB, "nA_sel": int(IA.size), "nB_sel": int(IB.size),
        "dirs": U, "kA": kA, "kB": kB, "evals": evals,
    })
    return r


def adaptive_alpha(A, B, alpha0: float = 0.005, growth: float = 2.0, alpha_max: float = 0.32,
                   tol: float = 1e-3):
    """Adaptive alpha under an error budget (a reading: the paper's
    Conclusion names adaptive alpha schedules for strict error budgets as
    future work and Sec. III shows the error falling as alpha grows; the
    schedule below is this implementation's).

    Directions are found once (Alg. 1, Alg. 2; m = floor(sqrt(D))).  For
    alpha_j = min(alpha0 growth^j, alpha_max), j = 0, 1, ...:
      F_j  = the inner-full value max{h(A_sel, B), h(B_sel, A)} over the
             alpha_j candidates -- never above H(A, B);
      lb_j = max(H_U, F_j) and ub = min_u (H_u + 2 delta(u)) over the same
             directions, delta measured from the line through the centroid
             of A u B (Sec. II-E bounds: lb_j <= H <= ub);
    and the schedule stops at the first j with
      (ub - lb_j) <= tol lb_j                   reason 1 (certified gap),
      j >= 1 and F_j - F_{j-1} <= tol F_j       reason 2 (converged),
      alpha_j >= alpha_max                      reason 3.
    Returns a dict: alpha, H (= F_j) with witnesses, lb, ub, reason, steps,
    the per-step values and the candidate-set sizes.
    """
    A = _f64(A)
    B = _f64(B)
    nA, D = A.shape
    nB = B.shape[0]
    m = math.isqrt(D)
    u0 = centroid_direction(A, B)
    P, _ = principal_directions(A, B, m)
    U = np.vstack([u0[None, :], P])
    projA = U @ A.T
    projB = U @ B.T
    from .hausdorff import certificate
    cert = certificate(A, B, U, c=np.vstack([A, B]).mean(axis=0))
    hU, ub = float(cert["lb"]), float(cert["ub"])
    values = []
    alpha = float(alpha0)
    j = 0
    while True:
        a = min(alpha, alpha_max)
        kA = [k_rule(a, nA)] + [k_rule(a / m, nA)] * m
        kB = [k_rule(a, nB)] + [k_rule(a / m, nB)] * m
        IA, IB = select(projA, projB, kA, kB)
        r = subset_hd(A, B, IA, IB, inner="full")
        F = r["H"]
        values.append(F)
        lb = max(hU, F)
        if ub - lb <= tol * lb:
            reason = 1
        elif j >= 1 and F - values[-2] <= tol * F:
            reason = 2
        elif a >= alpha_max:
            reason = 3
        else:
            alpha *= growth
            j += 1
            continue
        r.update({"alpha": a, "lb": lb, "ub": ub, "reason": reason, "steps": j + 1,
                  "values": values, "nA_sel": int(IA.size), "nB_sel": int(IB.size), "m": m})
        return r
