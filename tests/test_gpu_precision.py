"""GPU parity of the precision form: bfloat16 / float8 distance-search tiles
with float64 refinement, through the C ABI, against the FP64 oracle.

The low-precision tiles only rank rows; the reported distance is the
float64 distance of a refined pair, so it must meet the same 1e-4 bar as the
float32 path whenever the true witness row is among the refined rows (it is
for every case here; the row minima of the search are checked against the
quantisation error bound separately).
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, rel, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def _data(kind, nA, nB, D, seed):
    if kind == "gauss":
        return synth.gauss_outliers(nA, nB, D, seed=seed)
    if kind == "mix":
        return synth.mixture(nA, nB, D, seed=seed, K=64, normalize=True)
    return synth.mixture(nA, nB, D, seed=seed, K=128, outlier_frac=0.001)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("kind,nA,nB,D", [("gauss", 5000, 5000, 32), ("heavy", 9000, 7000, 256),
                                          ("mix", 6000, 6500, 128), ("gauss", 700, 900, 10),
                                          ("heavy", 3000, 2000, 64)])
def test_exact_low_precision(kind, nA, nB, D, prec):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"exact_hd prec={prec} {kind} nA={nA} nB={nB} D={D}")
    A, B = _data(kind, nA, nB, D, seed=D + 1)
    o = oracle.exact_hd(A, B)
    out, n2A, n2B = ph.exact_hd(to_dev(torch, A), to_dev(torch, B), sync=True, nn2=True, prec=prec)
    r = ph.decode_result(out)
    assert r["status"] == 0
    assert rel(r["H"], o["H"]) <= 1e-4, (r["H"], o["H"])
    assert rel(r["hAB"], o["hAB"]) <= 1e-4 and rel(r["hBA"], o["hBA"]) <= 1e-4
    # search minima: squared distances between quantised points; error bound
    # |d_q - d| <= |x_q - x| + |y_q - y| with relative rounding u per element
    u = 2.0 ** -8 if prec == "bf16" else 2.0 ** -3
    s = A[0].astype(np.float64)
    R = max(np.linalg.norm(A - s, axis=1).max(), np.linalg.norm(B - s, axis=1).max())
    dq = np.sqrt(np.maximum(n2A.cpu().numpy().astype(np.float64), 0))
    assert np.max(np.abs(dq - o["nnA"])) <= 2 * u * R + 1e-3 * R


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_exact_tiny_coordinates(prec):
    """Coordinates near 1e-18: the FP8 scale 2^floor(log2(224 / max|x - s|))
    would be 2^64 here, whose square overflows float32; the scale is capped
    at 2^60 and the refined distance still meets the 1e-4 bar."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"exact_hd prec={prec} tiny coordinates")
    A, B = synth.gauss_outliers(3000, 2500, 64, seed=11)
    A *= np.float32(1e-18)
    B *= np.float32(1e-18)
    s = A[0].astype(np.float64)
    m = max(np.abs(A - s).max(), np.abs(B - s).max())
    assert np.floor(np.log2(224.0 / m)) >= 64   # the uncapped scale would overflow
    o = oracle.exact_hd(A, B)
    out = ph.exact_hd(to_dev(torch, A), to_dev(torch, B), sync=True, prec=prec)
    r = ph.decode_result(out)
    assert r["status"] == 0
    assert rel(r["H"], o["H"]) <= 1e-4, (r["H"], o["H"])
    assert rel(r["hAB"], o["hAB"]) <= 1e-4 and rel(r["hBA"], o["hBA"]) <= 1e-4


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("inner_full", [False, True])
def test_prohd_hd_low_precision(prec, inner_full):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd_hd prec={prec} full={inner_full}")
    A, B = _data("heavy", 20000, 18000, 256, seed=3)
    g = np.random.default_rng(5)
    IA = np.sort(g.choice(20000, 3000, replace=False))
    IB = np.sort(g.choice(18000, 2500, replace=False))
    o = oracle.subset_hd(A, B, IA, IB, inner="full" if inner_full else "candidates")
    cnt = torch.tensor([IA.size, IB.size], dtype=torch.int64, device=dev)
    out = ph.prohd_hd(to_dev(torch, A), to_dev(torch, B), torch.from_numpy(IA.astype(np.int32)).cuda(),
                      cnt[0:1], torch.from_numpy(IB.astype(np.int32)).cuda(), cnt[1:2],
                      inner_full=inner_full, sync=True, prec=prec)
    r = ph.decode_result(out)
    assert r["status"] == 0 and rel(r["H"], o["H"]) <= 1e-4


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_prohd_end_to_end_low_precision(prec):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"prohd end-to-end prec={prec}")
    A, B = _data("gauss", 5000, 5000, 32, seed=0)
    r32 = ph.prohd(to_dev(torch, A), to_dev(torch, B), m=3, k=100)
    rlp = ph.prohd(to_dev(torch, A), to_dev(torch, B), m=3, k=100, prec=prec)
    IA = r32["idxA"][: int(r32["nselA"].item())].cpu().numpy()
    IB = r32["idxB"][: int(r32["nselB"].item())].cpu().numpy()
    o = oracle.subset_hd(A, B, IA, IB)
    assert rel(rlp["H"], o["H"]) <= 1e-4 and rel(r32["H"], o["H"]) <= 1e-5


def test_precision_flags_exclusive():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    L = ph.lib()
    z = torch.zeros((10, 4), device=dev)
    out = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)
    ws = torch.empty(1 << 24, dtype=torch.uint8, device=dev)
    code = L.exact_hd(z.data_ptr(), 10, z.data_ptr(), 10, 4, ph.PREC_BF16 | ph.PREC_FP8, out.data_ptr(),
                      None, None, ws.data_ptr(), 1 << 24, None)
    assert code == 1
