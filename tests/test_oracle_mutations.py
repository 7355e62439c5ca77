"""Planted mistakes in the oracle must fail its pins (CPU only).

Each case copies ``oracle/`` into a temporary directory, plants one plausible
slip in the copy's source (a minimum for a maximum, a dropped term or factor,
a transposed operand, the wrong end of a sort, a wrong ``k``, ...) and runs
``tests/test_oracle_pins.py`` against the copy in a subprocess: the pins must
fail.  An unmodified copy must pass (the harness itself works).  The real
oracle is never modified.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (file, text to replace, replacement, what the slip is)
MUTATIONS = [
    ("hausdorff.py", '"lb": float(hu.max())', '"lb": float(hu.min())',
     "certificate: lower bound as the smallest H_u"),
    ("hausdorff.py", '"ub": float((hu + 2 * de).min())', '"ub": float((hu + 2 * de).max())',
     "certificate: upper bound as the largest H_u + 2 delta"),
    ("hausdorff.py", '"ub": float((hu + 2 * de).min())', '"ub": float((hu + de).min())',
     "certificate: dropped factor 2 on delta"),
    ("hausdorff.py", '"H": max(hAB, hBA)', '"H": min(hAB, hBA)',
     "exact distance: smaller directed part"),
    ("hausdorff.py", "rn[None, :] - 2.0 * (q @ R.T)", "rn[None, :] - (q @ R.T)",
     "nearest neighbours: dropped factor 2 of the cross term"),
    ("hausdorff.py", "j = np.argmin(d2, axis=1)", "j = np.argmax(d2, axis=1)",
     "nearest neighbours: arg-max for arg-min"),
    ("hausdorff.py", "return float(near.max())", "return float(near.min())",
     "projected distance: min over the outer set"),
    ("hausdorff.py", "res = P - np.outer(P @ u, u)", "res = P",
     "delta: distance to the origin instead of the line"),
    ("hausdorff.py", "nnA, argA, nnB, argB = nn_both(A, B)", "nnB, argB, nnA, argA = nn_both(A, B)",
     "one-pass exact distance: directions swapped"),
    ("prohd.py", "u = B.mean(axis=0) - A.mean(axis=0)", "u = B.mean(axis=0)",
     "centroid axis: dropped the first centroid"),
    ("prohd.py", "if nrm < 1e-9:", "if nrm < 0.0:", "centroid axis: no e_1 fallback"),
    ("prohd.py", "Zc = Z - Z.mean(axis=0)", "Zc = Z", "principal components: no centring"),
    ("prohd.py", "order = np.argsort(-w, kind=\"stable\")", "order = np.argsort(w, kind=\"stable\")",
     "principal components: smallest eigenvalues"),
    ("prohd.py", "v = V[:, c] / np.linalg.norm(V[:, c])", "v = V[c, :] / np.linalg.norm(V[c, :])",
     "principal components: transposed eigenvectors"),
    ("prohd.py", "return np.sort(np.lexsort((np.arange(p.size), -p))[:k])",
     "return np.sort(np.lexsort((np.arange(p.size), p))[-k:])",
     "selection: stable slice at the top end (ties to larger indices)"),
    ("prohd.py", "bottom = np.lexsort((idx, p))[:k]", "bottom = np.lexsort((idx, p))[:k - 1]",
     "selection: one short at the bottom end"),
    ("prohd.py", "kA = [k_rule(alpha, nA)] + [k_rule(alpha / m, nA)] * m",
     "kA = [k_rule(alpha, nA)] + [k_rule(alpha, nA)] * m", "k rule: alpha not divided by m"),
    ("prohd.py", "return min(n, max(1, int(math.floor(alpha * n + 1e-9))))",
     "return min(n, max(1, int(math.ceil(alpha * n))))", "k rule: ceiling for floor"),
    ("prohd.py", "dA, aA = nn_dist(A[IA], B)", "dA, aA = nn_dist(A[IA], B[IB])",
     "inner-full mode: inner minimum over the candidates only"),
    ("prohd.py", "        if ub - lb <= tol * lb:", "        if ub - lb >= tol * lb:",
     "adaptive alpha: certified-gap rule reversed"),
    ("prohd.py", "        elif j >= 1 and F - values[-2] <= tol * F:", "        elif F - values[-1] <= tol * F:",
     "adaptive alpha: gain measured against the current step"),
    ("prohd.py", "        r = subset_hd(A, B, IA, IB, inner=\"full\")\n        F = r[\"H\"]",
     "        r = subset_hd(A, B, IA, IB)\n        F = r[\"H\"]", "adaptive alpha: candidate-mode value"),
    ("mlp.py", "return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))",
     "return 0.5 * z * (1.0 + erf(z / 2.0))", "GELU: wrong argument scale"),
    ("mlp.py", "dz1 = (dz2 @ W2) * _gelu_grad(z1)", "dz1 = (dz2 @ W2) * _gelu_grad(z2 @ W2)",
     "backward: GELU derivative at the wrong layer"),
    ("mlp.py", "mh = m / (1.0 - b1 ** t)", "mh = m", "AdamW: no bias correction of the first moment"),
    ("mlp.py", "p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)",
     "p = p - lr * (mh / (np.sqrt(vh) + eps)) + wd * p", "AdamW: weight decay not scaled by lr"),
]


def _copy_oracle(dst, mutation):
    src = os.path.join(ROOT, "oracle")
    shutil.copytree(src, os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"), copy_function=shutil.copy2)
    os.symlink(os.path.join(ROOT, "synth"), os.path.join(dst, "synth"))
    shutil.copy2(PINS, os.path.join(dst, "test_pins.py"))
    if mutation is not None:
        fname, old, new, _ = mutation
        path = os.path.join(dst, "oracle", fname)
        with open(path) as fh:
            text = fh.read()
        assert text.count(old) == 1, f"mutation anchor not unique in {fname}: {old!r}"
        with open(path, "w") as fh:
            fh.write(text.replace(old, new))


def _run_pins(dst):
    env = dict(os.environ)
    env.pop("PYTHONPATH", None)
    env["OMP_NUM_THREADS"] = "1"
    env["OPENBLAS_NUM_THREADS"] = "1"
    r = subprocess.run([sys.executable, "-m", "pytest", "test_pins.py", "-x", "-q",
                        "-p", "no:cacheprovider", "--rootdir", dst],
                       cwd=dst, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_pins_pass_on_an_unmodified_copy(tmp_path):
    _copy_oracle(str(tmp_path), None)
    rc, out = _run_pins(str(tmp_path))
    assert rc == 0, out


def test_every_planted_mistake_fails_a_pin(tmp_path):
    dirs = []
    for i, m in enumerate(MUTATIONS):
        d = tmp_path / f"m{i}"
        d.mkdir()
        _copy_oracle(str(d), m)
        dirs.append(str(d))
    with ThreadPoolExecutor(max(1, min(8, len(os.sched_getaffinity(0))))) as ex:
        results = list(ex.map(_run_pins, dirs))
    survivors = [MUTATIONS[i][3] for i, (rc, _) in enumerate(results) if rc == 0]
    assert not survivors, f"mistakes no pin caught: {survivors}"
