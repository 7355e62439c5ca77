"""exact_hd_noalloc (the no-allocation entry point, library-held scratch)
through the C ABI, against exact_hd (the workspace entry point) on the same
inputs: two calls in a row, the second with a smaller input in another
precision, so the second runs on scratch that still holds the first call's
contents.  Sets too large for the scratch, and PROHD_SYNC, are rejected
before any launch.
"""

import numpy as np
import pytest

import synth
from gpu_common import banner, rel, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def _same(r, q):
    for k in ("H", "hAB", "hBA"):
        assert rel(r[k], q[k]) <= 1e-4, (k, r[k], q[k])
    assert r["status"] == q["status"] == 0


def test_noalloc_matches_exact_hd_on_two_calls():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    cases = [(28000, 26000, 256, "fp32", 1), (3000, 2500, 64, "bf16", 2)]
    for nA, nB, D, prec, seed in cases:
        banner(f"exact_hd_noalloc nA={nA} nB={nB} D={D} prec={prec}")
        A, B = synth.mixture(nA, nB, D, seed=seed, K=32, outlier_frac=0.001)
        dA, dB = to_dev(torch, A), to_dev(torch, B)
        o1, a1, b1 = ph.exact_hd_noalloc(dA, dB, nn2=True, prec=prec)
        r1 = ph.decode_result(o1)
        o2, a2, b2 = ph.exact_hd(dA, dB, nn2=True, prec=prec)
        r2 = ph.decode_result(o2)
        _same(r1, r2)
        # same kernels on the same inputs: identical results
        assert (r1["H"], r1["ab_a"], r1["ab_b"], r1["ba_b"], r1["ba_a"]) == \
               (r2["H"], r2["ab_a"], r2["ab_b"], r2["ba_b"], r2["ba_a"])
        assert torch.equal(a1, a2) and torch.equal(b1, b2)


def test_noalloc_rejects_what_does_not_fit():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("exact_hd_noalloc rejections")
    L = ph.lib()
    big = torch.zeros((40000, 256), dtype=torch.float32, device=dev)
    out = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)
    code = L.exact_hd_noalloc(big.data_ptr(), 40000, big.data_ptr(), 40000, 256, 0,
                              out.data_ptr(), None, None, None)
    assert code == 3 and "PROHD_NOALLOC_SCRATCH_BYTES" in L.prohd_last_error().decode()
    small = torch.zeros((10, 4), dtype=torch.float32, device=dev)
    code = L.exact_hd_noalloc(small.data_ptr(), 10, small.data_ptr(), 10, 4, ph.SYNC,
                              out.data_ptr(), None, None, None)
    assert code == 1
    # a call after the rejections still works
    A, B = synth.gauss_outliers(900, 700, 16, seed=4)
    r = ph.decode_result(ph.exact_hd_noalloc(to_dev(torch, A), to_dev(torch, B)))
    q = ph.decode_result(ph.exact_hd(to_dev(torch, A), to_dev(torch, B)))
    _same(r, q)
