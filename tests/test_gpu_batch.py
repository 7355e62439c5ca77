"""GPU parity: the batched form (prohd_batch_* through the C ABI) against the
oracle pair by pair, on many uneven pairs with mixed dimensions.

ProHD per pair follows Alg. 3 in alpha mode (alpha = 0.01, m = floor(sqrt D));
the exact mode is Eq. (1).  Tolerances as the single-pair path: 1e-5
relative on H (float32 tiles, float64 refinement), candidate-set sizes equal
up to float32 projection near-ties.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import banner, rel, torch_gpu

pytestmark = pytest.mark.gpu


def _pairs(P, seed, lo, hi, dims):
    nA, nB, D = synth.batch_sizes(P, seed, lo=lo, hi=hi, dims=dims)
    As, Bs = [], []
    for i in range(P):
        A, B = synth.gauss_outliers(int(nA[i]), int(nB[i]), int(D[i]), seed=1000 * seed + i)
        As.append(A)
        Bs.append(B)
    return nA, nB, D, As, Bs


def test_batch_exact_and_prohd_match_oracle():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    P = 24
    nA, nB, D, As, Bs = _pairs(P, 1, 40, 3000, (3, 16, 33, 64, 128, 256))
    nA[0], nB[0] = 1, 2          # degenerate pair sizes
    As[0], Bs[0] = synth.gauss_outliers(1, 2, int(D[0]), seed=77)
    banner(f"batch P={P} sizes {nA.min()}..{max(nA.max(), nB.max())} dims {sorted(set(D.tolist()))}")
    plan = ph.BatchPlan(nA, nB, D, alpha=0.01)
    dA, dB = plan.pack(As, Bs)
    ex = plan.results(plan.run(dA, dB, mode="exact", sync=True))
    pr = plan.results(plan.run(dA, dB, mode="prohd", sync=True))
    for i in range(P):
        A, B = As[i], Bs[i]
        we = oracle.exact_hd(A, B)
        assert ex[i]["status"] == 0
        assert rel(ex[i]["H"], we["H"]) <= 1e-5, (i, ex[i]["H"], we["H"])
        assert rel(ex[i]["hAB"], we["hAB"]) <= 1e-5 and rel(ex[i]["hBA"], we["hBA"]) <= 1e-5
        m = int(np.floor(np.sqrt(D[i]) + 1e-9))
        wp = oracle.prohd(A, B, alpha=0.01, m=m)
        assert pr[i]["status"] == 0
        assert rel(pr[i]["H"], wp["H"]) <= 1e-5, (i, int(nA[i]), int(nB[i]), int(D[i]), pr[i]["H"], wp["H"])
        assert abs(pr[i]["nA_sel"] - wp["nA_sel"]) <= 2 and abs(pr[i]["nB_sel"] - wp["nB_sel"]) <= 2
    plan.close()


def test_batch_graph_replay_eager_and_single_pair_agree():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    P = 40
    nA, nB, D, As, Bs = _pairs(P, 2, 256, 8192, (64, 128, 256))
    banner(f"batch replay P={P}")
    plan = ph.BatchPlan(nA, nB, D, alpha=0.01)
    dA, dB = plan.pack(As, Bs)
    for mode in ("prohd", "exact"):
        out = torch.zeros((P, ph.RESULT_BYTES), dtype=torch.uint8, device=dev)
        first = plan.run(dA, dB, mode=mode, out=out).clone()
        # replays with eager host work in between, each checked against the first
        for _ in range(3):
            out.zero_()
            torch.cuda.synchronize()
            plan.run(dA, dB, mode=mode, out=out)
            torch.cuda.synchronize()
            assert torch.equal(out, first)
        eager = plan.run(dA, dB, mode=mode, eager=True)
        assert torch.equal(eager, first)
        got = plan.results(first)
        for i in (0, 7, P - 1):
            A = torch.from_numpy(As[i]).to(dev)
            B = torch.from_numpy(Bs[i]).to(dev)
            if mode == "exact":
                single = ph.decode_result(ph.exact_hd(A, B))
            else:
                single = ph.prohd(A, B, alpha=0.01)
            assert rel(got[i]["H"], single["H"]) <= 1e-6
    plan.close()


def test_batch_tuner_writes_table_and_keeps_results(tmp_path):
    torch, dev = torch_gpu()
    import json
    import paper_2511_18207_amd as ph
    P = 16
    nA, nB, D, As, Bs = _pairs(P, 3, 256, 20000, (64, 256))
    banner(f"batch tune P={P}")
    plan = ph.BatchPlan(nA, nB, D, alpha=0.01)
    dA, dB = plan.pack(As, Bs)
    ref = {m: plan.results(plan.run(dA, dB, mode=m, sync=True)) for m in ("prohd", "exact")}
    for mode in ("prohd", "exact"):
        path = str(tmp_path / f"tune_{mode}.json")
        plan.tune(dA, dB, mode=mode, json_path=path)
        rec = json.load(open(path))
        assert rec["mode"] == mode and rec["pairs"] == P and len(rec["trials"]) >= 6
        got = plan.results(plan.run(dA, dB, mode=mode, sync=True))
        for a, b in zip(got, ref[mode]):
            assert rel(a["H"], b["H"]) <= 1e-6
        plan2 = ph.BatchPlan(nA, nB, D, alpha=0.01)
        plan2.load_tuning(path)
        got2 = plan2.results(plan2.run(dA, dB, mode=mode, sync=True))
        for a, b in zip(got2, got):
            assert a["H"] == b["H"]
        plan2.close()
    plan.close()


def test_batch_largest_pairs_of_the_bench_batch():
    """The largest pairs of the 4 096-pair batch bench.py times
    (synth.batch_sizes(4096, 0): pair 3210 is 63 206 x 63 310 at D = 256,
    pairs 2948 and 3548 the next by work and by rows), drawn exactly as there
    (synth.batch_pair), run as one batch with two small pairs of the same
    batch; ProHD and the exact distance per pair against the oracle."""
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    nA_all, nB_all, D_all = synth.batch_sizes(4096, 0)
    pick = [3210, 2948, 3548, 2953, 2439]
    nA, nB, D = nA_all[pick], nB_all[pick], D_all[pick]
    banner(f"batch largest pairs {list(zip(nA.tolist(), nB.tolist(), D.tolist()))}")
    As, Bs = [], []
    for i in pick:
        a, b = synth.batch_pair(0, i, nA_all[i], nB_all[i], D_all[i])
        As.append(a)
        Bs.append(b)
    plan = ph.BatchPlan(nA, nB, D, alpha=0.01)
    dA, dB = plan.pack(As, Bs)
    try:
        ex = plan.results(plan.run(dA, dB, mode="exact", sync=True))
        pr = plan.results(plan.run(dA, dB, mode="prohd", sync=True))
    finally:
        plan.close()
    for j, i in enumerate(pick):
        ox = oracle.exact_hd(As[j], Bs[j], one_pass=True)
        op = oracle.prohd(As[j], Bs[j], alpha=0.01, m=int(np.floor(np.sqrt(D[j]) + 1e-9)))
        print(f"[batch] pair {i} {nA[j]}x{nB[j]} D={D[j]}: exact {ex[j]['H']:.9g} vs {ox['H']:.9g}, "
              f"prohd {pr[j]['H']:.9g} vs {op['H']:.9g}", flush=True)
        assert ex[j]["status"] == 0 and pr[j]["status"] == 0
        assert rel(ex[j]["H"], ox["H"]) <= 1e-5
        assert rel(ex[j]["hAB"], ox["hAB"]) <= 1e-5 and rel(ex[j]["hBA"], ox["hBA"]) <= 1e-5
        assert rel(pr[j]["H"], op["H"]) <= 1e-5
        assert abs(pr[j]["nA_sel"] - op["nA_sel"]) <= 2 and abs(pr[j]["nB_sel"] - op["nB_sel"]) <= 2
