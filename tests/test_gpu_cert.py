"""GPU: the error certificate (prohd_certificate, Sec. II-E bounds) against
the oracle.  The certified interval must contain the exact distance; its
projected-distance bounds must contain the oracle's H_U on the same
directions, and its spreads must bound the oracle's delta from above while
staying within float32 slack of it."""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n,D,m,k,seed", [
    ("gauss", 5000, 32, 3, 100, 0),
    ("gauss", 3001, 33, 5, 40, 1),
    ("mix", 40000, 128, 8, 1000, 2),
    ("uniform", 20000, 4, 2, 50, 3),
])
def test_certificate_contains_exact(name, n, D, m, k, seed):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"certificate {name} n={n} D={D} m={m}")
    if name == "gauss":
        A, B = synth.gauss_outliers(n, n, D, seed)
    elif name == "mix":
        A, B = synth.mixture(n, n, D, seed, K=64, normalize=True)
    else:
        A, B = synth.uniform_clouds(n, n, D, seed)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    r = ph.prohd(dA, dB, m=m, k=k, inner_full=True)
    full = ph.prohd_hd(dA, dB, r["idxA"], r["nselA"], r["idxB"], r["nselB"], inner_full=True)
    cert = ph.certificate(dA, dB, r["dirs"], r["projA"], r["projB"], lower=full)
    H = oracle.exact_hd(A, B)["H"]
    U = r["dirs"].cpu().numpy().astype(np.float64)
    c = np.vstack([A.astype(np.float64), B.astype(np.float64)]).mean(0)
    want = oracle.certificate(A, B, U, c)
    print(f"[cert] H={H:.6f} lb={cert['lb']:.6f} ub={cert['ub']:.6f} oracle lb={want['lb']:.6f} "
          f"ub={want['ub']:.6f} full={r['H']:.6f}", flush=True)
    assert cert["status"] == 0
    assert cert["lb"] <= H * (1 + 1e-12) and H <= cert["ub"] * (1 + 1e-12)
    assert cert["lb"] >= r["H"] * (1 - 1e-12)          # the inner-full value is a lower bound
    # projected distance: the oracle's H_U lies inside the GPU bounds, which
    # are tight to a few bins plus the projection error
    assert cert["hu_lo"] <= want["lb"] * (1 + 1e-12) + 1e-12
    assert want["lb"] <= cert["hu_hi"] * (1 + 1e-12)
    span = max(float(np.ptp(np.concatenate([A @ u, B @ u]))) for u in U.astype(np.float32))
    assert cert["hu_hi"] - cert["hu_lo"] <= 4 * span / 8192 + 4 * cert["proj_err"] + 1e-12
    # spreads: never below the oracle's, and close to it
    dmin = float(want["delta"].min())
    assert cert["delta_min"] >= dmin * (1 - 1e-6)
    assert cert["delta_min"] <= dmin * (1 + 1e-4) + 1e-6
    assert cert["ub"] <= want["ub"] * (1 + 1e-3) + 4 * span / 8192 + 4 * cert["proj_err"]
