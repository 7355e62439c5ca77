"""The C-ABI library loads and exports every symbol include/prohd.h declares;
host-side validation rejects bad arguments before touching a device.

No compute call runs here (no GPU on this machine): every call below fails
validation, which happens before any HIP call.
"""

import ctypes as C
import os
import re

import pytest

import paper_2511_18207_amd as ph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prohd.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(prohd_\w+|exact_hd\w*)\s*\(", src)) - {"prohd_status"})


def test_library_exports_every_declared_symbol():
    L = ph.lib()
    names = _declared_functions()
    assert {"prohd_project", "prohd_select", "prohd_hd", "exact_hd"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    # and nm agrees (C linkage, not mangled)
    out = os.popen(f"nm -D --defined-only {ph.library_path()}").read()
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_version_and_result_layout():
    assert ph.version().startswith("prohd-gfx950")
    assert ph.RESULT_BYTES == 80


def test_workspace_size_rules():
    assert ph.workspace_size(0, 5, 8) == 0
    assert ph.workspace_size(5, 5, 0) == 0
    assert ph.workspace_size(5, 5, 257) == 0
    assert ph.workspace_size(5, 5, 8, ndirs=65) == 0
    small = ph.workspace_size(1000, 1000, 32, 4)
    big = ph.workspace_size(100000, 100000, 32, 4)
    assert 0 < small < big
    # 2M x 2M, D=256: dominated by the padded float32 copies of both sets
    # (4.1 GB) plus their bfloat16 copies for the precision form (2.0 GB)
    full = ph.workspace_size(2_000_000, 2_000_000, 256, 17, 80_000, 80_000)
    assert 6.0e9 < full < 7.0e9


def _err(code_fn):
    L = ph.lib()
    code = code_fn(L)
    return code, L.prohd_last_error().decode()


FAKE = 0x1000  # never dereferenced: validation fails first


@pytest.mark.parametrize("call,code,msg", [
    (lambda L: L.exact_hd(None, 1, FAKE, 1, 4, 0, FAKE, None, None, FAKE, 1 << 20, None), 1, "non-null"),
    (lambda L: L.exact_hd(FAKE, 0, FAKE, 1, 4, 0, FAKE, None, None, FAKE, 1 << 20, None), 1, ">= 1"),
    (lambda L: L.exact_hd(FAKE, 1, FAKE, 1, 0, 0, FAKE, None, None, FAKE, 1 << 20, None), 1, "D must"),
    (lambda L: L.exact_hd(FAKE, 1, FAKE, 1, 300, 0, FAKE, None, None, FAKE, 1 << 20, None), 5, "MAX_DIM"),
    (lambda L: L.exact_hd(FAKE, 1, FAKE, 1, 4, 1 << 9, FAKE, None, None, FAKE, 1 << 20, None), 1, "flag"),
    (lambda L: L.exact_hd(FAKE, 10, FAKE, 10, 4, 0, FAKE, None, None, FAKE, 16, None), 3, "workspace"),
    (lambda L: L.exact_hd(FAKE, 10, FAKE, 10, 4, 0, None, None, None, FAKE, 1 << 20, None), 1, "out"),
    (lambda L: L.prohd_project(FAKE, 10, FAKE, 10, 4, 0, 0, FAKE, FAKE, FAKE, None, None, FAKE, 1 << 24, None), 1, "m must"),
    (lambda L: L.prohd_project(FAKE, 10, FAKE, 10, 4, 5, 0, FAKE, FAKE, FAKE, None, None, FAKE, 1 << 24, None), 1, "m must"),
    (lambda L: L.prohd_project(FAKE, 10, FAKE, 10, 200, 64, 0, FAKE, FAKE, FAKE, None, None, FAKE, 1 << 30, None), 5, "MAX_DIRS"),
    (lambda L: L.prohd_project(FAKE, 10, FAKE, 10, 4, 2, 0, None, FAKE, FAKE, None, None, FAKE, 1 << 24, None), 1, "non-null"),
    (lambda L: L.prohd_project(FAKE, 10, FAKE, 10, 4, 2, 0, FAKE, FAKE, FAKE, None, None, FAKE, 8, None), 3, "workspace"),
    (lambda L: L.prohd_hd(FAKE, 10, FAKE, 10, 4, FAKE, FAKE, FAKE, FAKE, 0, 5, 0, FAKE, FAKE, 1 << 24, None), 1, "capA"),
    (lambda L: L.prohd_hd(FAKE, 10, FAKE, 10, 4, FAKE, FAKE, FAKE, FAKE, 11, 5, 0, FAKE, FAKE, 1 << 24, None), 1, "capA"),
    (lambda L: L.prohd_hd(FAKE, 10, FAKE, 10, 4, None, FAKE, FAKE, FAKE, 5, 5, 0, FAKE, FAKE, 1 << 24, None), 1, "index"),
    (lambda L: L.prohd_hd(FAKE, 10, FAKE, 10, 4, FAKE, FAKE, FAKE, FAKE, 5, 5, 1 << 6, FAKE, FAKE, 1 << 24, None), 1, "flag"),
    (lambda L: L.prohd_hd(FAKE, 10, FAKE, 10, 4, FAKE, FAKE, FAKE, FAKE, 5, 5, 12, FAKE, FAKE, 1 << 24, None), 1, "exclusive"),
    (lambda L: L.exact_hd(FAKE, 10, FAKE, 10, 4, 2, FAKE, None, None, FAKE, 1 << 24, None), 1, "flag"),
    (lambda L: L.prohd_top_keys(FAKE, 10, None, 65, FAKE, FAKE, FAKE, 1 << 20, None), 1, "k must"),
    (lambda L: L.prohd_top_keys(FAKE, 10, None, -1, FAKE, FAKE, FAKE, 1 << 20, None), 1, "k must"),
    (lambda L: L.prohd_top_keys(FAKE, -1, None, 4, FAKE, FAKE, FAKE, 1 << 20, None), 1, "n must"),
    (lambda L: L.prohd_top_keys(FAKE, 1 << 31, None, 4, FAKE, FAKE, FAKE, 1 << 20, None), 1, "n must"),
    (lambda L: L.prohd_top_keys(None, 10, None, 4, FAKE, FAKE, FAKE, 1 << 20, None), 1, "non-null"),
    (lambda L: L.prohd_top_keys(FAKE, 10, None, 4, None, FAKE, FAKE, 1 << 20, None), 1, "non-null"),
    (lambda L: L.prohd_top_keys(FAKE, 10, None, 4, FAKE, FAKE, FAKE, 1 << 18, None), 3, "workspace"),
])
def test_validation_errors(call, code, msg):
    got, text = _err(call)
    assert got == code, text
    assert msg in text


def test_select_validation():
    L = ph.lib()
    k = (C.c_int32 * 2)(10, 10)
    k0 = (C.c_int32 * 2)(10, 0)
    # capacity below min(n, sum 2k)
    assert L.prohd_select(FAKE, 100, FAKE, 100, 2, k, k, FAKE, 39, FAKE, FAKE, 40, FAKE, FAKE, 1 << 24, None) == 1
    assert "capA" in L.prohd_last_error().decode()
    # k < 1
    assert L.prohd_select(FAKE, 100, FAKE, 100, 2, k0, k, FAKE, 40, FAKE, FAKE, 40, FAKE, FAKE, 1 << 24, None) == 1
    # too many directions
    assert L.prohd_select(FAKE, 100, FAKE, 100, 65, k, k, FAKE, 40, FAKE, FAKE, 40, FAKE, FAKE, 1 << 24, None) == 5


def test_mlp_and_scored_validation():
    import oracle.mlp as om
    L = ph.lib()
    for D in (1, 17, 256):
        assert ph.mlp_param_count(D) == om.param_count(D)
    assert ph.mlp_param_count(0) == 0 and ph.mlp_param_count(257) == 0
    assert ph.mlp_workspace_size(0, 8) == 0
    assert ph.mlp_workspace_size(1000, 8) < ph.mlp_workspace_size(100000, 8)
    assert L.prohd_mlp_init(None, 8, 0, None) == 1
    assert L.prohd_mlp_init(FAKE, 300, 0, None) == 5
    assert L.prohd_mlp_score(FAKE, 0, 8, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == 1
    assert L.prohd_mlp_score(FAKE, 100, 8, FAKE, FAKE, FAKE, FAKE, 16, None) == 3
    assert L.prohd_mlp_grad(FAKE, 8, FAKE, FAKE, FAKE, 65537, 1.0, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == 1
    assert "batch" in L.prohd_last_error().decode()
    assert L.prohd_mlp_grad(FAKE, 8, FAKE, FAKE, FAKE, 64, 0.0, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == 1
    assert L.prohd_mlp_adamw(FAKE, FAKE, FAKE, FAKE, 8, 0, 1e-3, 0.0, 0.9, 0.999, 1e-8, None) == 1
    assert L.prohd_mlp_adamw(FAKE, FAKE, FAKE, FAKE, 8, 1, 1e-3, 0.0, 1.0, 0.999, 1e-8, None) == 1
    assert L.prohd_select_scored(FAKE, 100, 5, FAKE, 100, 5, FAKE, 4, FAKE, FAKE, 10, FAKE, FAKE,
                                 1 << 30, None) == 1
    assert "capacities" in L.prohd_last_error().decode()
    assert L.prohd_select_scored(FAKE, 100, -1, FAKE, 100, 5, FAKE, 10, FAKE, FAKE, 10, FAKE, FAKE,
                                 1 << 30, None) == 1


def test_batch_plan_validation():
    L = ph.lib()
    h = C.c_void_p()
    nA = (C.c_int64 * 2)(10, 0)
    nB = (C.c_int64 * 2)(10, 10)
    D = (C.c_int32 * 2)(8, 8)
    assert L.prohd_batch_create(2, nA, nB, D, 0.01, C.byref(h)) == 1
    assert "sizes" in L.prohd_last_error().decode()
    D2 = (C.c_int32 * 2)(8, 300)
    nA2 = (C.c_int64 * 2)(10, 10)
    assert L.prohd_batch_create(2, nA2, nB, D2, 0.01, C.byref(h)) == 5
    assert L.prohd_batch_create(2, nA2, nB, D, 0.0, C.byref(h)) == 1
    assert L.prohd_batch_create(0, nA2, nB, D, 0.01, C.byref(h)) == 1
    plan = ph.BatchPlan([100, 2000, 1], [50, 3000, 2], [16, 256, 3])
    assert plan.workspace_size("prohd") > 0 and plan.workspace_size("exact") > 0
    assert list(plan.offA) == [0, 1600, 1600 + 512000, 1600 + 512000 + 3]
    assert L.prohd_batch_run(plan._h, 7, FAKE, FAKE, FAKE, FAKE, 1 << 20, 0, None) == 1
    assert L.prohd_batch_run(plan._h, 0, None, FAKE, FAKE, FAKE, 1 << 20, 0, None) == 1
    assert L.prohd_batch_run(plan._h, 0, FAKE, FAKE, FAKE, FAKE, 1 << 20, 1 << 9, None) == 1
    plan.close()


def test_k_rule_matches_oracle():
    import oracle
    for a, n in [(0.01, 2_000_000), (0.01 / 16, 2_000_000), (0.29, 100), (0.5, 3), (0.001, 10)]:
        assert ph.k_rule(a, n) == oracle.k_rule(a, n)


def test_profile_api_without_gpu():
    ph.profile_enable(False)
    ph.profile_reset()
    assert ph.profile_read("hd_tile") == (0, 0.0)


def test_alpha_mode_helper_matches_the_oracle_k_rule():
    """prohd_default_m / prohd_alpha_k (host functions of the C ABI) against
    the oracle's k rule (Alg. 1, Alg. 2 with alpha / m, Alg. 3's m)."""
    import math

    import oracle
    for D in range(1, 257):
        assert ph.default_m(D) == math.isqrt(D)
    L = ph.lib()
    assert L.prohd_default_m(0) == 0 and L.prohd_default_m(257) == 0
    for alpha in (0.01, 0.29, 0.07, 0.001, 0.5, 1.0, 1e-4, 0.3, 2.5):
        for n in (1, 2, 7, 100, 999, 5000, 65_536, 2_000_000):
            for m in (1, 2, 3, 5, 16):
                k = ph.alpha_k(alpha, n, m)
                assert k == [oracle.k_rule(alpha, n)] + [oracle.k_rule(alpha / m, n)] * m, (alpha, n, m)
    buf = (C.c_int32 * 64)()
    for alpha, n, m in ((0.0, 10, 1), (float("nan"), 10, 1), (float("inf"), 10, 1), (0.1, 0, 1),
                        (0.1, 1 << 31, 1), (0.1, 10, 0), (0.1, 10, 64)):
        assert L.prohd_alpha_k(alpha, n, m, buf) == 1
    assert L.prohd_alpha_k(0.1, 10, 2, None) == 1


def test_adaptive_validation():
    L = ph.lib()
    assert L.prohd_adaptive_workspace_size(0, 10, 4, 0.3, 0) == 0
    assert L.prohd_adaptive_workspace_size(10, 10, 4, 0.0, 0) == 0
    small = L.prohd_adaptive_workspace_size(1000, 1000, 16, 0.05, 0)
    assert 0 < small < L.prohd_adaptive_workspace_size(1000, 1000, 16, 0.5, 0)
    res = (C.c_char * 64)()
    big = 1 << 30
    for args, code in (((0.0, 2.0, 0.3, 1e-3, 0), 1), ((0.4, 2.0, 0.3, 1e-3, 0), 1),
                       ((0.01, 1.0, 0.3, 1e-3, 0), 1), ((0.01, 2.0, 0.3, -1.0, 0), 1),
                       ((0.01, 2.0, 0.3, 1e-3, 1 << 1), 1), ((0.01, 2.0, 0.3, 1e-3, 12), 1)):
        assert L.prohd_adaptive(FAKE, 100, FAKE, 100, 8, *args, FAKE, res, FAKE, big, None) == code
    assert L.prohd_adaptive(FAKE, 100, FAKE, 100, 8, 0.01, 2.0, 0.3, 1e-3, 0, FAKE, None, FAKE, big, None) == 1
    assert L.prohd_adaptive(FAKE, 100, FAKE, 100, 8, 0.01, 2.0, 0.3, 1e-3, 0, FAKE, res, FAKE, 16, None) == 3


def test_prune_levels():
    """Levels of the pruned search (host rule, no device work): strides
    16^L with the coarsest subset of the smaller inner set at least 16 rows,
    L in [1, 4]; no pruning below 16384 outer rows or without the flag."""
    assert ph.prune_levels(16383, 50000) == 0
    assert ph.prune_levels(16384, 16384) == 2          # 16384 / 256 = 64, / 4096 = 4
    assert ph.prune_levels(65535, 65535) == 2          # 65535 / 4096 = 15.99
    assert ph.prune_levels(65536, 65536) == 3
    assert ph.prune_levels(2_000_000, 2_000_000) == 4  # 2M / 65536 = 30
    assert ph.prune_levels(2_000_000, 2_000_000, 78_966, 78_462) == 3
    assert ph.prune_levels(2_000_000, 2_000_000, 78_966, 78_462, inner_full=True) == 4
    assert ph.prune_levels(2_000_000, 2_000_000, prune=False) == 0
    assert ph.prune_levels(1 << 31, 1 << 31) == 4
    assert ph.prune_levels(5, 5, 6, 5) == 0             # invalid capacity
