"""ctypes binding of libprohd.so (see include/prohd.h for the contract).

Argument marshalling only: tensors become device pointers, the current torch
stream becomes the hipStream_t, host integer lists become int32 arrays.
"""

from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

DIRS_GIVEN = 1 << 0
INNER_FULL = 1 << 1
PREC_BF16 = 1 << 2
PREC_FP8 = 1 << 3
SYNC = 1 << 4
PRUNE = 1 << 5
PREC = {"fp32": 0, "bf16": PREC_BF16, "fp8": PREC_FP8}

STATUS = {0: "OK", 1: "EINVAL", 2: "ENONFINITE", 3: "EWORKSPACE", 4: "EDEVICE", 5: "EUNSUPPORTED"}

# prohd_cert, as laid out by the C struct
CERT_DTYPE = np.dtype([
    ("lb", "<f8"), ("ub", "<f8"), ("hu_lo", "<f8"), ("hu_hi", "<f8"),
    ("delta_min", "<f8"), ("proj_err", "<f8"), ("best_dir", "<i4"), ("status", "<i4"),
])

# prohd_result, as laid out by the C struct
RESULT_DTYPE = np.dtype([
    ("H", "<f8"), ("hAB", "<f8"), ("hBA", "<f8"),
    ("ab_a", "<i8"), ("ab_b", "<i8"), ("ba_b", "<i8"), ("ba_a", "<i8"),
    ("nA_sel", "<i8"), ("nB_sel", "<i8"),
    ("status", "<i4"), ("refined", "<i4"),
])
RESULT_BYTES = RESULT_DTYPE.itemsize

# prohd_adaptive_result (host struct)
ADAPTIVE_DTYPE = np.dtype([
    ("alpha", "<f8"), ("H", "<f8"), ("lb", "<f8"), ("ub", "<f8"), ("change", "<f8"),
    ("nA_sel", "<i8"), ("nB_sel", "<i8"), ("steps", "<i4"), ("reason", "<i4"),
])


class ProhdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def library_path() -> str:
    return os.path.join(HERE, "libprohd.so")


def lib() -> C.CDLL:
    """Load libprohd.so (built in-tree).  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ProhdError(5, f"{path} is missing: build it with "
                            "`python -m paper_2511_18207_amd.build`")
    L = C.CDLL(path)
    i64, i32, u32, vp, sz = C.c_int64, C.c_int32, C.c_uint32, C.c_void_p, C.c_size_t
    L.prohd_workspace_size.restype = sz
    L.prohd_workspace_size.argtypes = [i64, i64, i32, i32, i64, i64]
    L.prohd_default_m.restype = i32
    L.prohd_default_m.argtypes = [i32]
    L.prohd_prune_levels.restype = i32
    L.prohd_prune_levels.argtypes = [i64, i64, i64, i64, u32]
    L.prohd_alpha_k.restype = C.c_int
    L.prohd_alpha_k.argtypes = [C.c_double, i64, i32, vp]
    L.prohd_project.restype = C.c_int
    L.prohd_project.argtypes = [vp, i64, vp, i64, i32, i32, u32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.prohd_select.restype = C.c_int
    L.prohd_select.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp, i64, vp, vp, i64, vp, vp, sz, vp]
    L.prohd_hd.restype = C.c_int
    L.prohd_hd.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp, vp, i64, i64, u32, vp, vp, sz, vp]
    L.exact_hd.restype = C.c_int
    L.exact_hd.argtypes = [vp, i64, vp, i64, i32, u32, vp, vp, vp, vp, sz, vp]
    L.exact_hd_noalloc.restype = C.c_int
    L.exact_hd_noalloc.argtypes = [vp, i64, vp, i64, i32, u32, vp, vp, vp, vp]
    L.prohd_adaptive_workspace_size.restype = sz
    L.prohd_adaptive_workspace_size.argtypes = [i64, i64, i32, C.c_double, u32]
    L.prohd_adaptive.restype = C.c_int
    L.prohd_adaptive.argtypes = [vp, i64, vp, i64, i32, C.c_double, C.c_double, C.c_double,
                                 C.c_double, u32, vp, vp, vp, sz, vp]
    L.prohd_mlp_param_count.restype = sz
    L.prohd_mlp_param_count.argtypes = [i32]
    L.prohd_mlp_workspace_size.restype = sz
    L.prohd_mlp_workspace_size.argtypes = [i64, i32]
    L.prohd_mlp_init.restype = C.c_int
    L.prohd_mlp_init.argtypes = [vp, i32, C.c_uint64, vp]
    L.prohd_mlp_score.restype = C.c_int
    L.prohd_mlp_score.argtypes = [vp, i64, i32, vp, vp, vp, vp, sz, vp]
    L.prohd_mlp_grad.restype = C.c_int
    L.prohd_mlp_grad.argtypes = [vp, i32, vp, vp, vp, i64, C.c_float, vp, vp, vp, vp, sz, vp]
    L.prohd_mlp_adamw.restype = C.c_int
    L.prohd_mlp_adamw.argtypes = [vp, vp, vp, vp, i32, i64, C.c_float, C.c_float, C.c_float,
                                  C.c_float, C.c_float, vp]
    L.prohd_mlp_train_step.restype = C.c_int
    L.prohd_mlp_train_step.argtypes = [vp, i32, vp, vp, vp, i64, C.c_float, vp, vp, vp, vp, i64,
                                       C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, vp,
                                       vp, sz, vp]
    L.prohd_centroid.restype = C.c_int
    L.prohd_centroid.argtypes = [vp, i64, i32, vp, vp, sz, vp]
    L.prohd_top_keys.restype = C.c_int
    L.prohd_top_keys.argtypes = [vp, i64, vp, i32, vp, vp, vp, sz, vp]
    L.prohd_certificate_workspace_size.restype = sz
    L.prohd_certificate_workspace_size.argtypes = [i32, i32]
    L.prohd_certificate.restype = C.c_int
    L.prohd_certificate.argtypes = [vp, i64, vp, i64, i32, vp, i32, vp, vp, vp, vp, vp, sz, vp]
    L.prohd_select_scored.restype = C.c_int
    L.prohd_select_scored.argtypes = [vp, i64, i32, vp, i64, i32, vp, i64, vp, vp, i64, vp, vp, sz,
                                      vp]
    L.prohd_batch_create.restype = C.c_int
    L.prohd_batch_create.argtypes = [i32, vp, vp, vp, C.c_double, C.POINTER(vp)]
    L.prohd_batch_destroy.restype = None
    L.prohd_batch_destroy.argtypes = [vp]
    L.prohd_batch_workspace_size.restype = sz
    L.prohd_batch_workspace_size.argtypes = [vp, u32]
    L.prohd_batch_run.restype = C.c_int
    L.prohd_batch_run.argtypes = [vp, u32, vp, vp, vp, vp, sz, u32, vp]
    L.prohd_batch_tune.restype = C.c_int
    L.prohd_batch_tune.argtypes = [vp, u32, vp, vp, vp, vp, sz, vp, C.c_char_p]
    L.prohd_batch_load_tuning.restype = C.c_int
    L.prohd_batch_load_tuning.argtypes = [vp, C.c_char_p]
    L.prohd_last_error.restype = C.c_char_p
    L.prohd_last_error.argtypes = []
    L.prohd_version.restype = C.c_char_p
    L.prohd_version.argtypes = []
    L.prohd_profile_enable.restype = C.c_int
    L.prohd_profile_enable.argtypes = [i32]
    L.prohd_profile_reset.restype = C.c_int
    L.prohd_profile_reset.argtypes = []
    L.prohd_profile_read.restype = C.c_int
    L.prohd_profile_read.argtypes = [C.c_char_p, C.POINTER(i64), C.POINTER(C.c_double)]
    _LIB = L
    return L


def _check(code: int):
    if code != 0:
        raise ProhdError(code, lib().prohd_last_error().decode())


def _torch():
    import torch
    return torch


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _f32_2d(X, name):
    torch = _torch()
    if not isinstance(X, torch.Tensor) or not X.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
        raise TypeError(f"{name} must be a contiguous 2-D float32 tensor")
    return X


def version() -> str:
    return lib().prohd_version().decode()


def workspace_size(nA, nB, D, ndirs=1, capA=0, capB=0) -> int:
    return int(lib().prohd_workspace_size(nA, nB, D, ndirs, capA, capB))


class Workspace:
    """A device byte buffer reused across calls (grown on demand)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=self.device)
        return self.buf


_DEFAULT_WS = {}


def _ws(ws, nbytes):
    if ws is None:
        dev = _torch().cuda.current_device()
        ws = _DEFAULT_WS.setdefault(dev, Workspace(f"cuda:{dev}"))
    buf = ws.get(nbytes)
    return buf, buf.numel()


def decode_result(res_dev) -> dict:
    """Device prohd_result bytes (uint8 tensor) -> dict (synchronises)."""
    arr = np.frombuffer(res_dev.cpu().numpy().tobytes(), dtype=RESULT_DTYPE)[0]
    return {k: arr[k].item() for k in RESULT_DTYPE.names}


def prohd_project(A, B, m, dirs=None, sync=False, ws=None, evals=True):
    """Directions (row 0 centroid axis, rows 1..m principal components) and
    projections of both sets.  With ``dirs`` given, uses them as is.
    Returns ``(dirs, projA, projB, evals, status)`` (device tensors)."""
    torch = _torch()
    A = _f32_2d(A, "A")
    B = _f32_2d(B, "B")
    nA, D = A.shape
    nB = B.shape[0]
    flags = SYNC if sync else 0
    if dirs is None:
        dirs = torch.empty((m + 1, D), dtype=torch.float32, device=A.device)
    else:
        dirs = _f32_2d(dirs, "dirs")
        if dirs.shape != (m + 1, D):
            raise ValueError("dirs must be (m+1) x D")
        flags |= DIRS_GIVEN
    projA = torch.empty((m + 1, nA), dtype=torch.float32, device=A.device)
    projB = torch.empty((m + 1, nB), dtype=torch.float32, device=A.device)
    ev = torch.empty(D, dtype=torch.float64, device=A.device) if evals else None
    status = torch.zeros(1, dtype=torch.int32, device=A.device)
    buf, nbytes = _ws(ws, workspace_size(nA, nB, D, m + 1))
    _check(lib().prohd_project(A.data_ptr(), nA, B.data_ptr(), nB, D, m, flags, dirs.data_ptr(),
                               projA.data_ptr(), projB.data_ptr(), _ptr(ev), status.data_ptr(),
                               buf.data_ptr(), nbytes, _stream()))
    return dirs, projA, projB, ev, status


def prohd_select(projA, projB, kA, kB, capA=None, capB=None, ws=None):
    """Union of per-direction extremes.  ``kA``/``kB``: one k per direction.
    Returns ``(idxA, nselA, idxB, nselB)``; idx tensors have capacity length,
    the device counts say how many entries are valid."""
    torch = _torch()
    ndirs, nA = projA.shape
    nB = projB.shape[1]
    kA = np.ascontiguousarray(kA, dtype=np.int32)
    kB = np.ascontiguousarray(kB, dtype=np.int32)
    if kA.size != ndirs or kB.size != ndirs:
        raise ValueError("need one k per direction")
    if capA is None:
        capA = int(min(nA, 2 * np.minimum(kA.astype(np.int64), nA).sum()))
    if capB is None:
        capB = int(min(nB, 2 * np.minimum(kB.astype(np.int64), nB).sum()))
    idxA = torch.empty(max(capA, 1), dtype=torch.int32, device=projA.device)
    idxB = torch.empty(max(capB, 1), dtype=torch.int32, device=projA.device)
    cnt = torch.zeros(2, dtype=torch.int64, device=projA.device)
    D_dummy = 1
    buf, nbytes = _ws(ws, workspace_size(nA, nB, D_dummy, ndirs))
    _check(lib().prohd_select(projA.data_ptr(), nA, projB.data_ptr(), nB, ndirs,
                              kA.ctypes.data, kB.ctypes.data, idxA.data_ptr(), capA,
                              cnt.data_ptr(), idxB.data_ptr(), capB, cnt.data_ptr() + 8,
                              buf.data_ptr(), nbytes, _stream()))
    return idxA, cnt[0:1], idxB, cnt[1:2]


def prohd_hd(A, B, idxA, nselA, idxB, nselB, capA=None, capB=None, inner_full=False,
             sync=False, ws=None, out=None, prec="fp32", prune=True):
    """Hausdorff distance over the selected rows.  ``prec`` selects the
    distance-search tiles ("fp32", "bf16", "fp8"; refinement is float64 in
    every case); ``prune`` the pruned search (PROHD_PRUNE: same result, used
    in the default mode on candidate sets of at least 16384 rows each).
    Returns the device result buffer (uint8[80]); decode with
    ``decode_result``."""
    torch = _torch()
    A = _f32_2d(A, "A")
    B = _f32_2d(B, "B")
    nA, D = A.shape
    nB = B.shape[1 - 1]
    capA = idxA.numel() if capA is None else capA
    capB = idxB.numel() if capB is None else capB
    flags = (INNER_FULL if inner_full else 0) | (SYNC if sync else 0) | PREC[prec] | \
        (PRUNE if prune else 0)
    if out is None:
        out = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=A.device)
    buf, nbytes = _ws(ws, workspace_size(nA, nB, D, 1, capA, capB))
    _check(lib().prohd_hd(A.data_ptr(), nA, B.data_ptr(), nB, D, idxA.data_ptr(),
                          nselA.data_ptr(), idxB.data_ptr(), nselB.data_ptr(), capA, capB, flags,
                          out.data_ptr(), buf.data_ptr(), nbytes, _stream()))
    return out


def exact_hd(A, B, sync=False, ws=None, out=None, nn2=False, prec="fp32", prune=True):
    """Exact Hausdorff distance (``prec`` and ``prune`` as in prohd_hd; with
    ``nn2`` the search is never pruned).  Returns the device result buffer,
    and with ``nn2=True`` also the per-row squared NN distance arrays of the
    tile search."""
    torch = _torch()
    A = _f32_2d(A, "A")
    B = _f32_2d(B, "B")
    nA, D = A.shape
    nB = B.shape[0]
    if out is None:
        out = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=A.device)
    nnA = torch.empty(nA, dtype=torch.float32, device=A.device) if nn2 else None
    nnB = torch.empty(nB, dtype=torch.float32, device=A.device) if nn2 else None
    buf, nbytes = _ws(ws, workspace_size(nA, nB, D, 1))
    flags = (SYNC if sync else 0) | PREC[prec] | (PRUNE if prune else 0)
    _check(lib().exact_hd(A.data_ptr(), nA, B.data_ptr(), nB, D, flags,
                          out.data_ptr(), _ptr(nnA), _ptr(nnB), buf.data_ptr(), nbytes,
                          _stream()))
    return (out, nnA, nnB) if nn2 else out


NOALLOC_SCRATCH_BYTES = 64 << 20


def exact_hd_noalloc(A, B, out=None, nn2=False, prec="fp32"):
    """exact_hd through the no-allocation entry point (library-held scratch
    of NOALLOC_SCRATCH_BYTES per GPU; calls on one GPU must not overlap).
    Returns the device result buffer (and the nn2 arrays with nn2=True)."""
    torch = _torch()
    A = _f32_2d(A, "A")
    B = _f32_2d(B, "B")
    nA, D = A.shape
    nB = B.shape[0]
    if out is None:
        out = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=A.device)
    nnA = torch.empty(nA, dtype=torch.float32, device=A.device) if nn2 else None
    nnB = torch.empty(nB, dtype=torch.float32, device=A.device) if nn2 else None
    _check(lib().exact_hd_noalloc(A.data_ptr(), nA, B.data_ptr(), nB, D, PREC[prec],
                                  out.data_ptr(), _ptr(nnA), _ptr(nnB), _stream()))
    return (out, nnA, nnB) if nn2 else out


def prune_levels(nA, nB, capA=None, capB=None, inner_full=False, prune=True) -> int:
    """Subset levels of the pruned search for these sizes (prohd_prune_levels;
    0: not pruned).  The first level's stride is 16 ** levels."""
    capA = nA if capA is None else capA
    capB = nB if capB is None else capB
    flags = (INNER_FULL if inner_full else 0) | (PRUNE if prune else 0)
    return int(lib().prohd_prune_levels(int(nA), int(nB), int(capA), int(capB), flags))


def default_m(D: int) -> int:
    """m = floor(sqrt(D)) (prohd_default_m)."""
    m = int(lib().prohd_default_m(int(D)))
    if m < 1:
        raise ProhdError(1, f"D={D} outside [1, 256]")
    return m


def alpha_k(alpha: float, n: int, m: int) -> list:
    """Per-direction counts of the alpha mode (prohd_alpha_k): k on the
    centroid axis, then k for each of the m principal components."""
    k = np.zeros(m + 1, dtype=np.int32)
    _check(lib().prohd_alpha_k(float(alpha), int(n), int(m), k.ctypes.data))
    return [int(x) for x in k]


def k_rule(alpha: float, n: int) -> int:
    """k = max(1, floor(alpha * n)) per end (Alg. 1), <= n (prohd_alpha_k)."""
    return alpha_k(alpha, n, 1)[0]


def prohd(A, B, alpha=0.01, m=None, k=None, dirs=None, inner_full=False, ws=None, prec="fp32",
          prune=True):
    """ProHD end to end on the device: project -> select -> hd.

    alpha mode: m = floor(sqrt(D)), k = k_rule(alpha, n) on the centroid axis
    and k_rule(alpha/m, n) per principal component.  explicit mode: ``k`` an
    int (every direction end) or a list of m+1 ints.  Returns a dict with the
    device tensors and the decoded result (one host synchronisation at the
    end)."""
    nA, D = A.shape
    nB = B.shape[0]
    if m is None:
        m = default_m(D) if dirs is None else dirs.shape[0] - 1
    if k is None:
        kA = alpha_k(alpha, nA, m)
        kB = alpha_k(alpha, nB, m)
    else:
        ks = [int(k)] * (m + 1) if np.isscalar(k) else [int(x) for x in k]
        kA = [min(max(1, x), nA) for x in ks]
        kB = [min(max(1, x), nB) for x in ks]
    d, pA, pB, ev, st = prohd_project(A, B, m, dirs=dirs, ws=ws)
    idxA, nA_sel, idxB, nB_sel = prohd_select(pA, pB, kA, kB, ws=ws)
    out = prohd_hd(A, B, idxA, nA_sel, idxB, nB_sel, inner_full=inner_full, ws=ws, prec=prec,
                   prune=prune)
    res = decode_result(out)
    res.update({"dirs": d, "projA": pA, "projB": pB, "evals": ev, "project_status": st,
                "idxA": idxA, "nselA": nA_sel, "idxB": idxB, "nselB": nB_sel,
                "kA": kA, "kB": kB})
    return res


def adaptive(A, B, alpha0=0.005, growth=2.0, alpha_max=0.32, tol=1e-3, prec="fp32", ws=None,
             out=None):
    """ProHD with alpha chosen under an error budget (prohd_adaptive; blocks).
    Returns a dict: the schedule's outcome (alpha, H = inner-full value,
    lb, ub, change, steps, reason) and the last step's decoded result
    (witnesses) under "result"."""
    torch = _torch()
    A = _f32_2d(A, "A")
    B = _f32_2d(B, "B")
    nA, D = A.shape
    nB = B.shape[0]
    if out is None:
        out = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=A.device)
    res = np.zeros(1, dtype=ADAPTIVE_DTYPE)
    need = int(lib().prohd_adaptive_workspace_size(nA, nB, D, float(alpha_max), PREC[prec]))
    buf, nbytes = _ws(ws, need)
    _check(lib().prohd_adaptive(A.data_ptr(), nA, B.data_ptr(), nB, D, float(alpha0), float(growth),
                                float(alpha_max), float(tol), PREC[prec], out.data_ptr(),
                                res.ctypes.data, buf.data_ptr(), nbytes, _stream()))
    d = {k: res[0][k].item() for k in ADAPTIVE_DTYPE.names}
    d["result"] = decode_result(out)
    return d


def mlp_param_count(D: int) -> int:
    return int(lib().prohd_mlp_param_count(D))


def mlp_workspace_size(rows: int, D: int) -> int:
    return int(lib().prohd_mlp_workspace_size(rows, D))


def _f32_1d(t, name, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
            or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA (HIP) tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} entries")
    return t


def mlp_init(D: int, seed: int = 0, device="cuda"):
    """A fresh float32 parameter vector (Glorot-uniform weights, zero biases)."""
    torch = _torch()
    p = torch.empty(mlp_param_count(D), dtype=torch.float32, device=device)
    _check(lib().prohd_mlp_init(p.data_ptr(), D, seed, _stream()))
    return p


def mlp_score(X, c_other, params, out=None, ws=None):
    """Scores of every row of X (features [x, x - c_other])."""
    torch = _torch()
    X = _f32_2d(X, "X")
    n, D = X.shape
    _f32_1d(c_other, "c_other", D)
    _f32_1d(params, "params", mlp_param_count(D))
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=X.device)
    buf, nbytes = _ws(ws, mlp_workspace_size(min(n, 65536), D))
    _check(lib().prohd_mlp_score(X.data_ptr(), n, D, c_other.data_ptr(), params.data_ptr(),
                                 out.data_ptr(), buf.data_ptr(), nbytes, _stream()))
    return out


def mlp_grad(X, c_other, labels, idx, params, pos_weight=1.0, grad=None, loss=None, ws=None):
    """Gradient and loss of the weighted BCE over rows X[idx] (device int32
    idx, float32 0/1 labels per row of X).  Returns (grad, loss) tensors."""
    torch = _torch()
    X = _f32_2d(X, "X")
    n, D = X.shape
    _f32_1d(c_other, "c_other", D)
    _f32_1d(labels, "labels", n)
    P = mlp_param_count(D)
    _f32_1d(params, "params", P)
    if idx.dtype != torch.int32 or not idx.is_cuda or not idx.is_contiguous():
        raise TypeError("idx must be a contiguous int32 CUDA (HIP) tensor")
    batch = idx.numel()
    if grad is None:
        grad = torch.empty(P, dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    buf, nbytes = _ws(ws, mlp_workspace_size(max(batch, 1), D))
    _check(lib().prohd_mlp_grad(X.data_ptr(), D, c_other.data_ptr(), labels.data_ptr(),
                                idx.data_ptr(), batch, float(pos_weight), params.data_ptr(),
                                grad.data_ptr(), loss.data_ptr(), buf.data_ptr(), nbytes,
                                _stream()))
    return grad, loss


def mlp_adamw(params, grad, m, v, D, t, lr, weight_decay=0.01, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW step, in place on params, m and v."""
    P = mlp_param_count(D)
    for name, x in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _f32_1d(x, name, P)
    _check(lib().prohd_mlp_adamw(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                 D, t, lr, weight_decay, beta1, beta2, eps, _stream()))


def mlp_train_step(X, c_other, labels, idx, params, grad, m, v, t, lr, pos_weight=1.0,
                   weight_decay=0.01, beta1=0.9, beta2=0.999, eps=1e-8, loss=None, ws=None):
    """prohd_mlp_grad followed by prohd_mlp_adamw (in place); returns the
    device loss tensor."""
    torch = _torch()
    X = _f32_2d(X, "X")
    n, D = X.shape
    P = mlp_param_count(D)
    _f32_1d(c_other, "c_other", D)
    _f32_1d(labels, "labels", n)
    for name, x in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _f32_1d(x, name, P)
    if idx.dtype != torch.int32 or not idx.is_cuda or not idx.is_contiguous():
        raise TypeError("idx must be a contiguous int32 CUDA (HIP) tensor")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    batch = idx.numel()
    buf, nbytes = _ws(ws, mlp_workspace_size(max(batch, 1), D))
    _check(lib().prohd_mlp_train_step(X.data_ptr(), D, c_other.data_ptr(), labels.data_ptr(),
                                      idx.data_ptr(), batch, float(pos_weight), params.data_ptr(),
                                      grad.data_ptr(), m.data_ptr(), v.data_ptr(), int(t), lr,
                                      weight_decay, beta1, beta2, eps, loss.data_ptr(),
                                      buf.data_ptr(), nbytes, _stream()))
    return loss


def centroid(X, out=None, ws=None):
    """Column mean of X (float64 accumulation) as a float32 device vector."""
    torch = _torch()
    X = _f32_2d(X, "X")
    n, D = X.shape
    if out is None:
        out = torch.empty(D, dtype=torch.float32, device=X.device)
    buf, nbytes = _ws(ws, 1024 * D * 8 + 256)
    _check(lib().prohd_centroid(X.data_ptr(), n, D, out.data_ptr(), buf.data_ptr(), nbytes,
                                _stream()))
    return out


TOPK_WS_BYTES = 512 * 1024 + 256


def prohd_top_keys(vals, k, dev_n=None, ws=None):
    """The k <= 64 largest entries of a 1-D float32 device tensor (equal
    values: smaller index first) through prohd_top_keys.  ``dev_n``: an
    optional device int64 tensor holding the length (clipped to the size).
    Returns ``(idx, count)``: ascending indices (capacity max(k, 1)) and the
    device count min(k, length)."""
    torch = _torch()
    if vals.dtype != torch.float32 or vals.dim() != 1 or not vals.is_contiguous():
        raise ValueError("vals must be a contiguous 1-D float32 tensor")
    idx = torch.empty(max(int(k), 1), dtype=torch.int32, device=vals.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=vals.device)
    buf, nbytes = _ws(ws, TOPK_WS_BYTES)
    _check(lib().prohd_top_keys(vals.data_ptr(), vals.numel(), _ptr(dev_n), int(k), idx.data_ptr(),
                                cnt.data_ptr(), buf.data_ptr(), nbytes, _stream()))
    return idx, cnt


top_keys = prohd_top_keys


def certificate(A, B, dirs, projA, projB, lower=None, ws=None):
    """Certified interval [lb, ub] around H(A,B) from ProHD's directions and
    projections (prohd_certificate).  ``lower``: device result of prohd_hd
    with inner_full=True (a lower bound of H), or None.  Returns a dict."""
    torch = _torch()
    A = _f32_2d(A, "A")
    B = _f32_2d(B, "B")
    nA, D = A.shape
    nB = B.shape[0]
    ndirs = dirs.shape[0]
    out = torch.zeros(CERT_DTYPE.itemsize, dtype=torch.uint8, device=A.device)
    buf, nbytes = _ws(ws, int(lib().prohd_certificate_workspace_size(D, ndirs)))
    _check(lib().prohd_certificate(A.data_ptr(), nA, B.data_ptr(), nB, D, dirs.data_ptr(), ndirs,
                                   projA.data_ptr(), projB.data_ptr(), _ptr(lower), out.data_ptr(),
                                   buf.data_ptr(), nbytes, _stream()))
    arr = np.frombuffer(out.cpu().numpy().tobytes(), dtype=CERT_DTYPE)[0]
    return {k: arr[k].item() for k in CERT_DTYPE.names}


def select_scored(scoresA, sA, scoresB, sB, idxA, nselA, idxB, nselB, ws=None):
    """Adds the sA / sB best-scoring rows to the selected index lists, in
    place (ascending unique union).  The index tensors' lengths are their
    capacities."""
    nA = scoresA.numel()
    nB = scoresB.numel()
    _f32_1d(scoresA, "scoresA")
    _f32_1d(scoresB, "scoresB")
    need = workspace_size(nA, nB, 1, 2)
    buf, nbytes = _ws(ws, need)
    _check(lib().prohd_select_scored(scoresA.data_ptr(), nA, int(sA), scoresB.data_ptr(), nB,
                                     int(sB), idxA.data_ptr(), idxA.numel(), nselA.data_ptr(),
                                     idxB.data_ptr(), idxB.numel(), nselB.data_ptr(),
                                     buf.data_ptr(), nbytes, _stream()))


BATCH_MODES = {"prohd": 0, "exact": 1}
BATCH_EAGER = 1 << 5


class BatchPlan:
    """Plan for many independent pairs (prohd_batch_*).  ``nA``, ``nB``, ``D``
    are per-pair sizes; the point sets are passed packed (``pack``)."""

    def __init__(self, nA, nB, D, alpha=0.01):
        self.nA = np.ascontiguousarray(nA, dtype=np.int64)
        self.nB = np.ascontiguousarray(nB, dtype=np.int64)
        self.D = np.ascontiguousarray(D, dtype=np.int32)
        if not (self.nA.size == self.nB.size == self.D.size):
            raise ValueError("nA, nB and D need one entry per pair")
        self.P = int(self.nA.size)
        self.alpha = float(alpha)
        h = C.c_void_p()
        _check(lib().prohd_batch_create(self.P, self.nA.ctypes.data, self.nB.ctypes.data,
                                        self.D.ctypes.data, self.alpha, C.byref(h)))
        self._h = h
        sizes_a = self.nA * self.D
        sizes_b = self.nB * self.D
        self.offA = np.concatenate([[0], np.cumsum(sizes_a)]).astype(np.int64)
        self.offB = np.concatenate([[0], np.cumsum(sizes_b)]).astype(np.int64)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().prohd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self, mode="prohd"):
        return int(lib().prohd_batch_workspace_size(self._h, BATCH_MODES[mode]))

    def pack(self, As, Bs, device="cuda"):
        """Packed float32 device buffers from per-pair arrays (host numpy)."""
        torch = _torch()
        hA = np.empty(int(self.offA[-1]), dtype=np.float32)
        hB = np.empty(int(self.offB[-1]), dtype=np.float32)
        for i, (a, b) in enumerate(zip(As, Bs)):
            hA[self.offA[i]:self.offA[i + 1]] = np.ascontiguousarray(a, dtype=np.float32).ravel()
            hB[self.offB[i]:self.offB[i + 1]] = np.ascontiguousarray(b, dtype=np.float32).ravel()
        return torch.from_numpy(hA).to(device), torch.from_numpy(hB).to(device)

    def _args(self, A, B, out, ws, mode):
        torch = _torch()
        if A.dtype != torch.float32 or B.dtype != torch.float32 or not A.is_cuda or not B.is_cuda:
            raise TypeError("A and B must be packed float32 CUDA (HIP) tensors")
        if A.numel() != int(self.offA[-1]) or B.numel() != int(self.offB[-1]):
            raise ValueError("packed sets do not match the plan's sizes")
        if out is None:
            out = torch.zeros((self.P, RESULT_BYTES), dtype=torch.uint8, device=A.device)
        buf, nbytes = _ws(ws, self.workspace_size(mode))
        return out, buf, nbytes

    def run(self, A, B, mode="prohd", out=None, ws=None, eager=False, sync=False):
        """Runs the batch (graph launch unless ``eager``); returns the device
        result array (P x 80 bytes)."""
        out, buf, nbytes = self._args(A, B, out, ws, mode)
        flags = (BATCH_EAGER if eager else 0) | (SYNC if sync else 0)
        _check(lib().prohd_batch_run(self._h, BATCH_MODES[mode], A.data_ptr(), B.data_ptr(),
                                     out.data_ptr(), buf.data_ptr(), nbytes, flags, _stream()))
        return out

    def tune(self, A, B, mode="prohd", out=None, ws=None, json_path=None):
        out, buf, nbytes = self._args(A, B, out, ws, mode)
        _check(lib().prohd_batch_tune(self._h, BATCH_MODES[mode], A.data_ptr(), B.data_ptr(),
                                      out.data_ptr(), buf.data_ptr(), nbytes, _stream(),
                                      json_path.encode() if json_path else None))

    def load_tuning(self, path):
        _check(lib().prohd_batch_load_tuning(self._h, path.encode()))

    @staticmethod
    def results(out):
        """Device result array -> list of dicts (synchronises)."""
        arr = np.frombuffer(out.cpu().numpy().tobytes(), dtype=RESULT_DTYPE)
        return [{k: a[k].item() for k in RESULT_DTYPE.names} for a in arr]


def profile_enable(on: bool = True):
    _check(lib().prohd_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib().prohd_profile_reset())


def profile_read(name: str):
    """(launches, total_ms) of kernels whose name contains ``name``."""
    n = C.c_int64(0)
    ms = C.c_double(0.0)
    _check(lib().prohd_profile_read(name.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value
