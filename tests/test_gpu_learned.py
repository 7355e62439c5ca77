"""GPU: the learned candidate proposal end to end -- labels from the exact
search, training with the library's kernels, and what the trained scorer
gains over plain ProHD at an equal candidate budget.

Workload: pairs drawn from one Student-t(30) mixture (32 clusters, D=64,
fixed centres, new samples per pair).  The gain is asserted in the
certified mode (inner minimum over the full other set, a lower bound of H):
there, adding a true witness can only raise the value towards H.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, to_dev, torch_gpu

pytestmark = pytest.mark.gpu

N, D, K, NU, CENTRES = 50_000, 64, 32, 30.0, 77


def _pair(torch, seed, n=N):
    A, B = synth.t_mixture(n, n, D, seed, K=K, nu=NU, centre_seed=CENTRES)
    return A, B, to_dev(torch, A), to_dev(torch, B)


def test_labels_match_oracle_nn():
    """Positives = rows whose exact NN distance is in the top 0.1 % of their
    set; the GPU labels (float32 tile search) must equal the oracle's (float64)
    up to swaps between rows whose distances tie within float32 error."""
    torch, dev = torch_gpu()
    from paper_2511_18207_amd import learned as LN
    banner("learned labels vs oracle nn_dist n=20000 D=64")
    A, B, dA, dB = _pair(torch, 5, n=20_000)
    yA, yB, ex = LN.witness_labels(dA, dB, frac=0.001)
    for y, Q, R in ((yA, A, B), (yB, B, A)):
        d, _ = oracle.nn_dist(Q.astype(np.float64), R.astype(np.float64))
        s = max(1, int(math.floor(0.001 * Q.shape[0])))
        order = np.lexsort((np.arange(d.size), -d))
        want = set(order[:s].tolist())
        got = set(np.flatnonzero(y.cpu().numpy()).tolist())
        assert len(got) == s
        kth = d[order[s - 1]]
        for i in got ^ want:  # only near-ties at the boundary may differ
            assert abs(d[i] - kth) <= 1e-5 * kth, (i, d[i], kth)
    want_H = oracle.exact_hd(A, B)["H"]
    assert abs(ex["H"] - want_H) <= 1e-4 * want_H


def test_centroid_matches_numpy():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("prohd_centroid")
    for n, d in ((1, 5), (999, 33), (300_001, 256)):
        X = synth.uniform_clouds(n, 1, d, seed=n)[0] * np.float32(100) - np.float32(50)
        got = ph.centroid(to_dev(torch, X)).cpu().numpy()
        want = X.astype(np.float64).mean(axis=0)
        assert np.allclose(got, want, rtol=0, atol=1e-6 * max(1.0, np.abs(want).max()) + 1e-5)


def test_training_reduces_loss_and_save_load(tmp_path):
    torch, dev = torch_gpu()
    from paper_2511_18207_amd import learned as LN
    banner("learned training loss + save/load")
    pairs = [LN.TrainPair(*_pair(torch, 100 + s)[2:]) for s in range(2)]
    sc = LN.Scorer(D, seed=3)
    losses = LN.train(sc, pairs, 400, batch=8192, lr=2e-3, pos_share=0.5, seed=1)
    assert np.isfinite(losses).all()
    assert losses[-50:].mean() < 0.5 * losses[:20].mean()
    path = str(tmp_path / "scorer.safetensors")
    sc.save(path)
    sc2 = LN.Scorer.load(path)
    A = pairs[0].A[:1000].contiguous()
    assert torch.equal(sc.score(A, pairs[0].cB), sc2.score(A, pairs[0].cB))


def test_learned_gain_at_equal_budget():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    from paper_2511_18207_amd import learned as LN
    banner(f"learned gain t({NU}) mixture n={N} D={D}")
    pairs = [LN.TrainPair(*_pair(torch, 1000 + s)[2:]) for s in range(4)]
    sc = LN.Scorer(D, seed=1)
    LN.train(sc, pairs, 1500, batch=16384, lr=2e-3, lr_final=1e-4, pos_share=0.5, seed=0)
    errs = {"learned": [], "plain": [], "prohd": []}
    for s in range(4):
        A, B, dA, dB = _pair(torch, 2000 + s)
        H = ph.decode_result(ph.exact_hd(dA, dB))["H"]
        rep = LN.equal_budget(dA, dB, sc, alpha=0.01, H=H)
        f = rep["full"]
        print(f"[learned] pair {s} H={H:.5f} full: prohd {f['prohd_err']:.3e} learned "
              f"{f['learned_err']:.3e} plain@{f['plain_budget']} {f['plain_err']:.3e}; "
              f"candidates: prohd {rep['candidates']['prohd_err']:.3e} learned "
              f"{rep['candidates']['learned_err']:.3e} plain {rep['candidates']['plain_err']:.3e}",
              flush=True)
        # certified mode: every value is a lower bound of H, and the learned
        # set is a superset of ProHD's, so it can only be closer
        assert f["learned"] <= H * (1 + 1e-6) and f["plain"] <= H * (1 + 1e-6)
        assert f["learned"] >= f["prohd"] * (1 - 1e-7)
        assert abs(f["learned_budget"] - f["plain_budget"]) <= 0.01 * f["learned_budget"] + 1
        for k in errs:
            errs[k].append(f[k + "_err"])
    mean = {k: float(np.mean(v)) for k, v in errs.items()}
    print(f"[learned] mean full-mode error {mean}", flush=True)
    assert mean["learned"] < mean["plain"]
    assert mean["learned"] < mean["prohd"]
