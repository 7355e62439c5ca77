"""Exact and projected Hausdorff distances, FP64 -- test infrastructure only.

Definitions followed (ProHD paper, Sec. II-A "Background and Notation"):

* Eq. (1): ``h(A,B) = max_{a in A} min_{b in B} ||a - b||_2`` and
  ``H(A,B) = max{h(A,B), h(B,A)}``.  Distances are Euclidean, not squared.
* Eq. (2): ``delta(u) = max_{p in A u B} ||p - (p^T u) u||``, the largest
  distance of any point from the line through the origin along unit ``u``.
* Sec. II-E.1 (single-direction bound): ``h_u(A,B) = max_a min_b
  |a^T u - b^T u|`` and ``H_u = max{h_u(A,B), h_u(B,A)}``; Sec. II-E.2 takes
  ``H_U = max_{u in U} H_u`` over a direction set.

Tie rule (a reading; the paper is silent): witnesses are the smallest index
among equal values, both for the arg-max over the outer set and for the
arg-min over the inner set.

All inputs are converted to float64 first (an exact upcast of float32 data).
"""

from __future__ import annotations

import ctypes
import math

import numpy as np

__all__ = [
    "directed_hd_bruteforce",
    "hd_bruteforce",
    "nn_dist",
    "nn_both",
    "exact_hd",
    "directed_hd_1d",
    "hd_1d",
    "hd_directions",
    "delta",
    "certificate",
]


def _f64(X) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim == 1:
        X = X[:, None]
    return np.ascontiguousarray(X, dtype=np.float64)


# --------------------------------------------------------------------------
# Eq. (1) written out literally: pure-Python loops, tiny inputs only.
# --------------------------------------------------------------------------
def directed_hd_bruteforce(A, B):
    """h(A,B) by the definition of Eq. (1), with explicit loops.

    Returns ``(value, i_star, j_star)``: the directed distance, the outer
    witness (row of A) and its nearest row of B.  O(nA*nB*D) Python steps,
    so only for a few hundred points.
    """
    A = _f64(A)
    B = _f64(B)
    best, bi, bj = -1.0, -1, -1
    for i in range(A.shape[0]):
        dmin, jmin = math.inf, -1
        for j in range(B.shape[0]):
            s = 0.0
            for t in range(A.shape[1]):
                diff = A[i, t] - B[j, t]
                s += diff * diff
            d = math.sqrt(s)
            if d < dmin:
                dmin, jmin = d, j
        if dmin > best:
            best, bi, bj = dmin, i, jmin
    return best, bi, bj


def hd_bruteforce(A, B):
    """H(A,B) of Eq. (1) from two literal directed computations."""
    return max(directed_hd_bruteforce(A, B)[0], directed_hd_bruteforce(B, A)[0])


# --------------------------------------------------------------------------
# Nearest-neighbour distances, blocked.  A library matrix product serves as
# the step that forms a.b; every returned value is re-measured by a direct
# difference so that the expansion's rounding never reaches a result.
# --------------------------------------------------------------------------
def nn_dist(Q, R, block_elems: int = 1 << 25):
    """For every row q of Q: ``min_{r in R} ||q - r||`` and the arg-min.

    Squared distances are formed as ``|q|^2 + |r|^2 - 2 q.r`` in FP64 for the
    search; each row's minimum is then recomputed as a direct difference
    ``||q - r*||`` at the arg-min (smallest index on ties).  Returns
    ``(dist[nQ], arg[nQ])`` in float64 / int64.
    """
    Q = _f64(Q)
    R = _f64(R)
    nQ, nR = Q.shape[0], R.shape[0]
    if nQ == 0 or nR == 0:
        raise ValueError("nn_dist needs non-empty sets")
    rn = np.einsum("ij,ij->i", R, R)
    dist = np.empty(nQ)
    arg = np.empty(nQ, dtype=np.int64)
    step = max(1, block_elems // max(nR, 1))
    for s in range(0, nQ, step):
        q = Q[s:s + step]
        d2 = np.einsum("ij,ij->i", q, q)[:, None] + rn[None, :] - 2.0 * (q @ R.T)
        j = np.argmin(d2, axis=1)
        arg[s:s + step] = j
        diff = q - R[j]
        dist[s:s + step] = np.sqrt(np.einsum("ij,ij->i", diff, diff))
    return dist, arg


def nn_both(A, B, block_rows: int = 4096, block_cols: int = 65536):
    """Nearest-neighbour distances of both directions from one pass.

    The same squared distances as ``nn_dist`` (``|a|^2 + |b|^2 - 2 a.b`` in
    FP64, the product from the BLAS library), taken block by block over the
    ``nA x nB`` matrix; each block serves both the minima over B of its A
    rows and the minima over A of its B rows (the plain loops of
    ``nnpass.c``, one read of the block), so the distance matrix is formed once, not once per
    direction.  Ties keep the smallest index, as in ``nn_dist``; each minimum
    is then re-measured as a direct difference at its arg-min.

    Returns ``(distA, argA, distB, argB)``: for every row of A its NN
    distance in B and the index, and the same for every row of B in A.
    """
    from . import _native

    lib = _native.load()
    A = _f64(A)
    B = _f64(B)
    nA, nB = A.shape[0], B.shape[0]
    if nA == 0 or nB == 0:
        raise ValueError("nn_both needs non-empty sets")
    an = np.ascontiguousarray(np.einsum("ij,ij->i", A, A))
    bn = np.ascontiguousarray(np.einsum("ij,ij->i", B, B))
    rowd = np.full(nA, np.inf)
    rowj = np.full(nA, -1, dtype=np.int64)
    cold = np.full(nB, np.inf)
    coli = np.full(nB, -1, dtype=np.int64)
    def dp(a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def ip(a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    for i0 in range(0, nA, block_rows):
        i1 = min(nA, i0 + block_rows)
        rd = np.ascontiguousarray(rowd[i0:i1])
        rj = np.ascontiguousarray(rowj[i0:i1])
        qn = np.ascontiguousarray(an[i0:i1])
        for j0 in range(0, nB, block_cols):
            j1 = min(nB, j0 + block_cols)
            G = np.ascontiguousarray(A[i0:i1] @ B[j0:j1].T)
            rn = np.ascontiguousarray(bn[j0:j1])
            cd = np.ascontiguousarray(cold[j0:j1])
            ci = np.ascontiguousarray(coli[j0:j1])
            if lib.nn_block(dp(G), i1 - i0, j1 - j0, dp(qn), dp(rn), i0, j0, dp(rd), ip(rj),
                            dp(cd), ip(ci)):
                raise MemoryError("nn_block: allocation failed")
            cold[j0:j1] = cd
            coli[j0:j1] = ci
        rowd[i0:i1] = rd
        rowj[i0:i1] = rj
    dA = A - B[rowj]
    dB = B - A[coli]
    return (np.sqrt(np.einsum("ij,ij->i", dA, dA)), rowj,
            np.sqrt(np.einsum("ij,ij->i", dB, dB)), coli)


def exact_hd(A, B, block_elems: int = 1 << 25, one_pass: bool = False):
    """Exact H(A,B) of Eq. (1) with both directed parts and witnesses.

    ``one_pass`` takes both directions' minima from one pass over the
    distance matrix (``nn_both``) instead of one pass per direction.

    Returns a dict:
      ``H, hAB, hBA``        Euclidean distances (float)
      ``ab_a, ab_b``         witness of h(A,B): row of A and its NN in B
      ``ba_b, ba_a``         witness of h(B,A): row of B and its NN in A
      ``nnA, nnB``           per-row NN distance of A to B and of B to A
      ``argA, argB``         per-row NN index
    """
    A = _f64(A)
    B = _f64(B)
    if A.shape[1] != B.shape[1]:
        raise ValueError("A and B must have the same dimension")
    if one_pass:
        nnA, argA, nnB, argB = nn_both(A, B)
    else:
        nnA, argA = nn_dist(A, B, block_elems)
        nnB, argB = nn_dist(B, A, block_elems)
    ia = int(np.argmax(nnA))
    ib = int(np.argmax(nnB))
    hAB = float(nnA[ia])
    hBA = float(nnB[ib])
    return {
        "H": max(hAB, hBA),
        "hAB": hAB,
        "hBA": hBA,
        "ab_a": ia,
        "ab_b": int(argA[ia]),
        "ba_b": ib,
        "ba_a": int(argB[ib]),
        "nnA": nnA,
        "nnB": nnB,
        "argA": argA,
        "argB": argB,
    }


# --------------------------------------------------------------------------
# Sec. II-E: projected (1-D) distances and the off-axis spread delta(u).
# --------------------------------------------------------------------------
def directed_hd_1d(pa, pb) -> float:
    """h_u(A,B) for already-projected scalars: max_a min_b |pa - pb|.

    The nearest scalar of a sorted ``pb`` is one of the two neighbours of the
    insertion point, so a sort plus a binary search gives the exact value.
    """
    pa = np.asarray(pa, dtype=np.float64).ravel()
    pb = np.sort(np.asarray(pb, dtype=np.float64).ravel())
    pos = np.searchsorted(pb, pa)
    lo = np.clip(pos - 1, 0, pb.size - 1)
    hi = np.clip(pos, 0, pb.size - 1)
    near = np.minimum(np.abs(pa - pb[lo]), np.abs(pa - pb[hi]))
    return float(near.max())


def hd_1d(pa, pb) -> float:
    """H_u = max{h_u(A,B), h_u(B,A)} on projected scalars."""
    return max(directed_hd_1d(pa, pb), directed_hd_1d(pb, pa))


def hd_directions(A, B, U) -> float:
    """H_U = max over the rows u of U of H_u(A,B) (Sec. II-E.2)."""
    A = _f64(A)
    B = _f64(B)
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    return max(hd_1d(A @ u, B @ u) for u in U)


def delta(A, B, u, c=None) -> float:
    """delta(u) of Eq. (2): max over A u B of the distance to the line R*u.

    ``u`` must be a unit vector; the line passes through the origin (the
    definition is not translation invariant), or through ``c`` when given:
    the bound H <= H_u + 2 delta(u) of Sec. II-E then still holds, because
    H and H_u do not change when both sets are translated by -c.
    Computed as the norm of the direct residual ``p - (p^T u) u``.
    """
    u = np.asarray(u, dtype=np.float64).ravel()
    P = np.vstack([_f64(A), _f64(B)])
    if c is not None:
        P = P - np.asarray(c, dtype=np.float64)[None, :]
    res = P - np.outer(P @ u, u)
    return float(np.sqrt(np.einsum("ij,ij->i", res, res)).max())


def certificate(A, B, U, c=None):
    """Interval [lb, ub] around H(A,B) from directions U (Sec. II-E):
    lb = max_u H_u, ub = min_u (H_u + 2 delta(u)) with delta measured from
    the line through ``c`` (origin when None).  Rows of U are normalised.
    Returns a dict with lb, ub, the per-direction H_u and delta."""
    A = _f64(A)
    B = _f64(B)
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    U = U / np.linalg.norm(U, axis=1, keepdims=True)
    hu = np.array([hd_1d(A @ u, B @ u) for u in U])
    de = np.array([delta(A, B, u, c) for u in U])
    return {"lb": float(hu.max()), "ub": float((hu + 2 * de).min()), "hu": hu, "delta": de}
