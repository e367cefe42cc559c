"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")
PKG = os.path.join(ROOT, "paper_1308_2166_amd")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def libtc():
    path = os.path.join(PKG, "libtc.so")
    if not os.path.exists(path):
        from paper_1308_2166_amd import build
        build.build()
    import torch  # noqa: F401  (same HIP runtime as the binding uses)
    return ctypes.CDLL(path)


def test_header_declares_the_main_entry_points():
    names = _declared()
    for n in ("tc_create", "tc_process_batch", "tc_estimate", "tc_read_state",
              "tc_destroy", "tc_multi_create", "tc_multi_process"):
        assert n in names


def test_library_exports_every_declared_symbol(libtc):
    missing = [n for n in _declared() if not hasattr(libtc, n)]
    assert missing == []


def test_binding_names_match_the_header():
    import paper_1308_2166_amd as tc
    assert sorted(tc.EXPORTS) == _declared()
    for n in _declared():
        assert callable(getattr(tc, n)), n


def test_error_codes_match_the_header():
    import paper_1308_2166_amd as tc
    src = open(HEADER).read()
    for name in ("TC_OK", "TC_EINVAL", "TC_EBADEDGE", "TC_EOVERFLOW",
                 "TC_ENOMEM", "TC_EHIP"):
        m = re.search(rf"#define {name} \(?(-?\d+)\)?", src)
        assert m and int(m.group(1)) == getattr(tc, name), name
    assert tc.TC_MAX_BATCH == 1 << 28


def test_product_code_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def test_kernels_are_plain_hip_for_gfx950():
    from paper_1308_2166_amd import build
    assert "--offload-arch=gfx950" in build.FLAGS
    for f in build.SOURCES:
        text = open(os.path.join(PKG, "csrc", f)).read()
        assert "__CUDA" not in text and "__HIP_PLATFORM" not in text


def test_estimators_needed_matches_oracle():
    # Theorem 2's sizing is a pure host function of the library: no GPU
    import numpy as np
    import oracle as O
    import paper_1308_2166_amd as tc
    rng = np.random.default_rng(3)
    for _ in range(200):
        eps, delta = float(rng.uniform(0.01, 1.0)), float(rng.uniform(0.001, 0.99))
        m, deg = int(rng.integers(1, 10**9)), int(rng.integers(1, 10**5))
        tau = float(rng.uniform(1.0, 1e12))
        assert tc.tc_estimators_needed(eps, delta, m, deg, tau) == \
            O.estimators_needed(eps, delta, m, deg, tau)
    assert tc.tc_estimators_needed(0.5, 0.1, 30, 6, 10.0) == 15916
    assert tc.tc_estimators_needed(0.5, 1.5, 30, 6, 10.0) == 0


def test_kernel_names_in_launch_order():
    # the per-kernel timing table: a host function of the library, no GPU
    import paper_1308_2166_amd as tc
    want = ["k_hist", "k_fold_step1", "k_cscan<0>", "k_scat<0>"]
    for p in (1, 2, 3):
        want += [f"k_cnt<{p}>", f"k_csum<{p}>", f"k_cscan<{p}>", f"k_scat<{p}>"]
    want += ["k_dir", "k_est", "k_pcnt", "k_pscan", "k_pscat", "k_pjoin", "k_small"]
    assert [tc.tc_kernel_name(k) for k in range(tc.tc_num_kernels())] == want
    bench = __import__("bench")
    assert [n for n in bench.STEP_ORDER] == want


def test_binding_refuses_w_beyond_the_tensor():
    # a w above the tensor's rows would make the kernels read past its end:
    # the binding refuses it before any library call (no GPU needed)
    import torch
    import paper_1308_2166_amd as tc
    e = torch.zeros((5, 2), dtype=torch.int32)
    for f in (tc.tc_process_batch, tc.tc_process_batch_naive, tc.tc_process_batch_noalloc):
        with pytest.raises(ValueError):
            f(0, e, w=6)


def test_step_bytes_bound_holds():
    # the serving admission bound: any step of at most n chunks and E edges
    # in all needs no more scratch than tc_step_bytes_max(n, r_max, E)
    # (pure host functions of the library, no GPU)
    import numpy as np
    import paper_1308_2166_amd as tc
    rng = np.random.default_rng(11)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        ws = [int(x) for x in np.exp(rng.uniform(0, np.log(3e6), n)).astype(np.int64) + 1]
        if rng.random() < 0.3:  # just above powers of two: the most rounding
            ws = [(1 << int(rng.integers(0, 22))) + 1 for _ in range(n)]
        rs = [int(x) for x in rng.integers(1, 1 << 18, n)]
        got = tc.tc_step_bytes(rs, ws)
        bound = tc.tc_step_bytes_max(n, max(rs), sum(ws))
        assert 0 < got <= bound, (ws, rs)
        # and the bound is not loose by more than the rounding it covers
        assert bound <= 4 * got + (64 << 20), (got, bound)
    assert tc.tc_step_bytes([5], [(1 << 28) + 1]) == 0
    assert tc.tc_step_bytes_max(0, 5, 5) == 0


def test_slots_for_budget_is_the_largest_fit():
    import paper_1308_2166_amd as tc
    from paper_1308_2166_amd import serve
    r, cap = 1 << 16, 1 << 23
    assert tc.tc_bank_bytes(r) == 36 * r + 16
    for budget in (1 << 30, 2 << 30, 3 << 30, 7 << 30):
        s = serve.slots_for_budget(budget, r, cap)
        assert s == 0 or serve.server_bytes(s, r, cap) <= budget
        assert serve.server_bytes(s + 1, r, cap) > budget


def test_probe_line_rate_refuses_bad_arguments():
    # argument checks happen before any HIP call (no GPU needed)
    import ctypes
    import paper_1308_2166_amd as tc
    L = tc.lib()
    d = ctypes.c_double()
    dummy = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below is refused
    for args in ((None, 128, 1, 1, 0, 1, dummy), (dummy, 100, 1, 1, 0, 1, dummy),
                 (dummy, 0, 1, 1, 0, 1, dummy), (dummy, 128, 0, 1, 0, 1, dummy),
                 (dummy, 128, 1, 0, 0, 1, dummy), (dummy, 128, 1, 9, 0, 1, dummy),
                 (dummy, 128, 1, 1, 0, 0, dummy), (dummy, 128, 1, 1, 0, 1, None)):
        assert L.tc_probe_line_rate(*args, ctypes.byref(d), None) == tc.TC_EINVAL, args
    assert L.tc_probe_line_rate(dummy, 128, 1, 1, 0, 1, dummy, None, None) == tc.TC_EINVAL
