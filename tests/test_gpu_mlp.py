"""GPU parity: the learned candidate-proposal scorer (prohd_mlp_* through the
C ABI) against the float64 reference in oracle/mlp.py, and prohd_select_scored
against the definition of a top-s union.

Tolerances: the kernels round weights, features and activations to bfloat16
(8 significant bits) and accumulate in float32.  Each layer then carries a
relative error of order 2^-8 on its outputs; three layers and the backward
chain stay well inside 3e-2 relative L2 error on scores and gradients, with
the gradient direction (cosine) above 0.999.  AdamW runs in float32 on
float32 inputs: 1e-5 relative.
"""

import numpy as np
import pytest

import oracle.mlp as om
import synth
from gpu_common import banner, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def _setup(torch, ph, n, D, seed):
    X = synth.gauss_outliers(n, 1, D, seed=seed)[0]
    c = (X.mean(axis=0) + 0.5).astype(np.float32)
    p = ph.mlp_init(D, seed=seed + 11)
    return X, c, p


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_init_deterministic_and_scaled():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("mlp_init D=40")
    D = 40
    p1 = ph.mlp_init(D, seed=3).cpu().numpy()
    p2 = ph.mlp_init(D, seed=3).cpu().numpy()
    p3 = ph.mlp_init(D, seed=4).cpu().numpy()
    assert np.array_equal(p1, p2)
    assert not np.array_equal(p1, p3)
    W1, b1, W2, b2, w3, b3 = om.unpack(p1, D)
    for W, fan in ((W1, 2 * D + om.H1), (W2, om.H1 + om.H2), (w3, om.H2 + 1)):
        a = np.sqrt(6.0 / fan)
        assert np.abs(W).max() <= a
        # uniform on (-a, a): mean 0 and variance a^2 / 3, within 4 standard
        # errors of the sample mean (a / sqrt(3N)) and of the sample variance
        # (relative sqrt(0.8 / N), kurtosis 9/5)
        N = W.size
        assert abs(W.mean()) < 4 * a / np.sqrt(3 * N)
        assert abs(W.var() / (a * a / 3) - 1) < 4 * np.sqrt(0.8 / N)
    assert not b1.any() and not b2.any() and not b3.any()


@pytest.mark.parametrize("n,D,seed", [(1, 8, 0), (777, 33, 1), (70001, 16, 2), (5000, 256, 3)])
def test_score_matches_oracle(n, D, seed):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"mlp_score n={n} D={D}")
    X, c, p = _setup(torch, ph, n, D, seed)
    # a non-trivial bias so every part of the network matters
    pn = p.cpu().numpy().astype(np.float64)
    g = np.random.default_rng(seed)
    W1, b1, W2, b2, w3, b3 = om.unpack(pn, D)
    b1[:] = g.normal(0, 0.1, b1.shape)
    b2[:] = g.normal(0, 0.1, b2.shape)
    b3[:] = 0.3
    p = to_dev(torch, pn)
    got = ph.mlp_score(to_dev(torch, X), to_dev(torch, c), p).cpu().numpy()
    want, _ = om.forward(pn, om.features(X, c), D)
    assert got.shape == (n,)
    assert np.isfinite(got).all()
    assert _relerr(got, want) < 3e-2
    if n > 1:
        assert np.corrcoef(got, want)[0, 1] > 0.999


@pytest.mark.parametrize("n,D,batch,seed", [(100, 8, 100, 0), (3000, 33, 1000, 1),
                                            (20000, 256, 4096, 2), (70000, 64, 65536, 3)])
def test_grad_matches_oracle(n, D, batch, seed):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"mlp_grad n={n} D={D} batch={batch}")
    X, c, p = _setup(torch, ph, n, D, seed)
    g = np.random.default_rng(seed + 100)
    y = (g.random(n) < 0.1).astype(np.float32)
    idx = g.integers(0, n, size=batch).astype(np.int32)
    pw = 5.0
    grad, loss = ph.mlp_grad(to_dev(torch, X), to_dev(torch, c), to_dev(torch, y),
                             torch.from_numpy(idx).cuda(), p, pos_weight=pw)
    pn = p.cpu().numpy().astype(np.float64)
    F = om.features(X[idx], c)
    want_loss, want = om.loss_grad(pn, F, y[idx], D, pos_weight=pw)
    got = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - want_loss) <= 1e-2 * abs(want_loss)
    cos = float(got @ want / (np.linalg.norm(got) * np.linalg.norm(want)))
    assert cos > 0.999, cos
    assert _relerr(got, want) < 3e-2
    # each parameter block individually
    for gb, wb in zip(om.unpack(got, D), om.unpack(want, D)):
        assert _relerr(gb.ravel(), wb.ravel()) < 5e-2


@pytest.mark.parametrize("t", [1, 7])
def test_adamw_matches_oracle(t):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"mlp_adamw t={t}")
    D = 24
    P = ph.mlp_param_count(D)
    g = np.random.default_rng(t)
    p, gr = g.normal(size=P).astype(np.float32), g.normal(size=P).astype(np.float32)
    m = (0.1 * g.normal(size=P)).astype(np.float32)
    v = (0.01 * g.random(P)).astype(np.float32)
    hp = dict(lr=1e-3, wd=0.01, b1=0.9, b2=0.999, eps=1e-8)
    hp32 = {k: float(np.float32(x)) for k, x in hp.items()}
    pd, md, vd = to_dev(torch, p), to_dev(torch, m), to_dev(torch, v)
    ph.mlp_adamw(pd, to_dev(torch, gr), md, vd, D, t, hp32["lr"], hp32["wd"], hp32["b1"],
                 hp32["b2"], hp32["eps"])
    wp, wm, wv = om.adamw(p.astype(np.float64), gr.astype(np.float64), m.astype(np.float64),
                          v.astype(np.float64), t, hp32["lr"], hp32["wd"], hp32["b1"], hp32["b2"],
                          hp32["eps"])
    # float32 rounding bounds, per element (u = 2^-24): the moment updates
    # are two products and a sum; the parameter update adds the moment
    # errors carried through the bias-corrected ratio
    u = 2.0 ** -24
    m64, v64, g64, p64 = (x.astype(np.float64) for x in (m, v, gr, p))
    Sm = np.abs(hp32["b1"] * m64) + np.abs((1 - hp32["b1"]) * g64)
    Sv = np.abs(hp32["b2"] * v64) + np.abs((1 - hp32["b2"]) * g64 * g64)
    c1 = 1 - hp32["b1"] ** t
    c2 = 1 - hp32["b2"] ** t
    den = np.sqrt(wv / c2) + hp32["eps"]
    ratio = (wm / c1) / den
    tol_m = 4 * u * Sm
    tol_v = 5 * u * Sv
    tol_p = (4 * u * np.abs(wp) + hp32["lr"] * (
        20 * u * (np.abs(ratio) + hp32["wd"] * np.abs(p64))
        + tol_m / c1 / den + np.abs(ratio) * tol_v / c2 / (2 * (wv / c2) + 1e-300) * (den - hp32["eps"]) / den))
    assert (np.abs(md.cpu().numpy() - wm) <= tol_m).all()
    assert (np.abs(vd.cpu().numpy() - wv) <= tol_v).all()
    assert (np.abs(pd.cpu().numpy() - wp) <= tol_p).all()


def _top(scores, s):
    order = np.lexsort((np.arange(scores.size), -scores.astype(np.float64)))
    return order[:s]


@pytest.mark.parametrize("nA,nB,sA,sB,seed", [(1, 1, 1, 0, 0), (100, 90, 7, 0, 1),
                                              (50000, 70001, 500, 333, 2), (4000, 4000, 4000, 10, 3)])
def test_select_scored_union(nA, nB, sA, sB, seed):
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner(f"select_scored nA={nA} nB={nB} sA={sA} sB={sB}")
    g = np.random.default_rng(seed)
    scA = g.integers(-50, 50, size=nA).astype(np.float32)  # many ties
    scB = g.normal(size=nB).astype(np.float32)
    exA = np.unique(g.integers(0, nA, size=max(1, nA // 10))).astype(np.int32)
    exB = np.unique(g.integers(0, nB, size=max(1, nB // 10))).astype(np.int32)
    wantA = np.union1d(exA, _top(scA, sA))
    wantB = np.union1d(exB, _top(scB, sB))
    capA = min(nA, exA.size + sA)
    capB = min(nB, exB.size + sB)
    idxA = torch.full((capA,), -1, dtype=torch.int32, device=dev)
    idxB = torch.full((capB,), -1, dtype=torch.int32, device=dev)
    idxA[:exA.size] = torch.from_numpy(exA).cuda()
    idxB[:exB.size] = torch.from_numpy(exB).cuda()
    cnt = torch.tensor([exA.size, exB.size], dtype=torch.int64, device=dev)
    ph.select_scored(to_dev(torch, scA), sA, to_dev(torch, scB), sB, idxA, cnt[0:1], idxB, cnt[1:2])
    na, nb = (int(x) for x in cnt.cpu())
    assert np.array_equal(idxA[:na].cpu().numpy(), wantA)
    assert np.array_equal(idxB[:nb].cpu().numpy(), wantB)
