"""GPU parity of adaptive alpha (prohd_adaptive through the C ABI) against
the oracle's schedule (oracle.adaptive_alpha) on the paper's random clouds
(U[0,1]^D against the same plus 0.1) and a clustered set: the same number
of steps, stopping rule and final alpha, the inner-full value within 1e-5
(float32 directions and projections: candidate sets equal up to
projection near-ties, checked through the value and the sizes), and the
certified interval containing the exact distance.  On a line (D = 1) the
Sec. II-E bounds close (H_U = H = ub in exact arithmetic); the library's
upper bound carries the float32 projection and binning slack of the
certificate (a few 1e-3 relative there), so that case runs with a 1e-2
budget, which both sides meet at the first step with the certified rule.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, rel, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,n,D,prec", [("clouds", 20000, 4, "fp32"), ("clouds", 20000, 16, "fp32"),
                                           ("clouds", 12000, 8, "bf16"), ("mix", 15000, 64, "fp32"),
                                           ("line", 5000, 1, "fp32")])
def test_adaptive_matches_oracle(kind, n, D, prec):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"adaptive alpha {kind} n={n} D={D} prec={prec}")
    if kind == "clouds":
        A, B = synth.uniform_clouds(n, n, D, seed=D)
    elif kind == "mix":
        A, B = synth.mixture(n, n, D, seed=7, K=16)
    else:
        g = np.random.default_rng(2)
        A = g.uniform(0, 10, size=(n, 1)).astype(np.float32)
        B = g.uniform(1, 12, size=(n - 700, 1)).astype(np.float32)
    kw = dict(alpha0=0.005, growth=2.0, alpha_max=0.32, tol=1e-2 if kind == "line" else 1e-3)
    o = oracle.adaptive_alpha(A, B, **kw)
    r = ph.adaptive(to_dev(torch, A), to_dev(torch, B), prec=prec, **kw)
    H = oracle.exact_hd(A, B, one_pass=True)["H"]
    print(f"[adaptive] {kind} D={D}: gpu alpha {r['alpha']} steps {r['steps']} reason {r['reason']} "
          f"F {r['H']:.9g} | oracle alpha {o['alpha']} steps {o['steps']} reason {o['reason']} "
          f"F {o['H']:.9g} | H {H:.9g} ub {r['ub']:.6g}", flush=True)
    assert r["result"]["status"] == 0
    assert (r["steps"], r["reason"]) == (o["steps"], o["reason"])
    assert r["alpha"] == pytest.approx(o["alpha"], rel=1e-12)
    assert rel(r["H"], o["H"]) <= 1e-5
    assert abs(r["nA_sel"] - o["nA_sel"]) <= 2 and abs(r["nB_sel"] - o["nB_sel"]) <= 2
    assert r["lb"] <= H * (1 + 1e-6) and r["ub"] >= H * (1 - 1e-6)
    assert r["H"] <= H * (1 + 1e-6)
    if kind == "line":
        assert r["reason"] == 1 and rel(r["H"], H) <= 1e-6
