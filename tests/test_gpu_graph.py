"""The ProHD step (prohd_project -> prohd_select -> prohd_hd, pruned search)
captured once as a HIP graph through torch and replayed: every replay must
give the eager result bit for bit, with eager work and synchronisations
between replays, and after the inputs are overwritten in place the replay
must give the eager result on the new inputs.  (The library launches only
kernels on the caller's stream in this path: no memset nodes, no host
synchronisation.)"""

import numpy as np
import pytest

import synth
from gpu_common import banner, to_dev, torch_gpu

pytestmark = pytest.mark.gpu

KEYS = ("H", "hAB", "hBA", "ab_a", "ab_b", "ba_b", "ba_a", "nA_sel", "nB_sel", "status", "refined")


def test_step_graph_replays_match_eager():
    torch, dev = torch_gpu()
    import paper_2511_18207_amd as ph
    banner("graph-captured ProHD step, gauss 60000 x 50000 x 64, alpha 0.2")
    A, B = synth.gauss_outliers(60000, 50000, 64, seed=21)
    A2, B2 = synth.gauss_outliers(60000, 50000, 64, seed=22)
    dA, dB = to_dev(torch, A), to_dev(torch, B)
    nA, D = A.shape
    nB = B.shape[0]
    m = ph.default_m(D)
    kA, kB = ph.alpha_k(0.2, nA, m), ph.alpha_k(0.2, nB, m)
    capA = min(nA, 2 * sum(kA))
    capB = min(nB, 2 * sum(kB))
    assert ph.prune_levels(nA, nB, capA, capB) >= 2
    ws = ph.Workspace(dev)
    ws.get(ph.workspace_size(nA, nB, D, m + 1, capA, capB))
    out = torch.zeros(ph.RESULT_BYTES, dtype=torch.uint8, device=dev)

    def step():
        _, pA, pB, _, _ = ph.prohd_project(dA, dB, m, ws=ws, evals=False)
        iA, cA, iB, cB = ph.prohd_select(pA, pB, kA, kB, capA=capA, capB=capB, ws=ws)
        ph.prohd_hd(dA, dB, iA, cA, iB, cB, capA=capA, capB=capB, ws=ws, out=out)

    def result():
        r = ph.decode_result(out)
        return {k: r[k] for k in KEYS}

    step()
    want = result()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for i in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert result() == want, i
        # eager work between replays
        ph.exact_hd(dA, dB, sync=True)
        torch.cuda.synchronize()
    # new inputs in the same buffers: the replay follows them
    dA.copy_(torch.from_numpy(A2))
    dB.copy_(torch.from_numpy(B2))
    step()
    want2 = result()
    assert want2["H"] != want["H"]
    out.zero_()
    g.replay()
    torch.cuda.synchronize()
    assert result() == want2
