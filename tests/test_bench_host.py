"""Host-side pieces of the benchmark that need no GPU."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.timeout(120)
def test_all_cores_oracle_baseline_runs_every_worker():
    from paper_1308_2166_amd import inputs
    bench = _bench()
    G, r, w, seed = inputs.workload("gnm-2k")
    E = G.numpy().view(np.uint32)
    res = bench.cpu_baseline_all_cores(E, r, seed, w, 3, 2)
    assert res["cores"] == 2 and res["kind"] == "oracle"
    assert res["value"] > 0 and np.isfinite(res["value"])
    assert "r/2 = 2048" in res["sample"]


def _write_csv(path, header, rows):
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        wr = csv.writer(f)
        wr.writerow(header)
        wr.writerows(rows)


def test_summarize_calibrates_with_the_first_copy(tmp_path):
    """The calibration copy is the run's first copy dispatch, even when a
    later copy (the input stream) is larger; traffic per launch is each
    counter times its calibration factor; the timed region is the last
    `timed` launches."""
    bench = _bench()
    mib = 4
    trace = ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    ctr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    copy = "__amd_rocclr_copyBuffer"
    t_rows = [[1, copy, 0, 1000], [2, copy, 2000, 9000]]
    f_rows = [[1, copy, "FETCH_SIZE", mib * 1024 / 2], [2, copy, "FETCH_SIZE", 99999.0]]
    w_rows = [[1, copy, "WRITE_SIZE", mib * 1024], [2, copy, "WRITE_SIZE", 88888.0]]
    durs = [10.0, 20.0, 30.0]  # us
    for k, d in enumerate(durs):
        t_rows.append([3 + k, "tc::k_est(tc::StepArgs)", 10000 * k, 10000 * k + int(d * 1000)])
        f_rows.append([3 + k, "tc::k_est(tc::StepArgs)", "FETCH_SIZE", 100.0])
        w_rows.append([3 + k, "tc::k_est(tc::StepArgs)", "WRITE_SIZE", 50.0])
    _write_csv(str(tmp_path / "t" / "run_kernel_trace.csv"), trace, t_rows)
    _write_csv(str(tmp_path / "f" / "run_counter_collection.csv"), ctr, f_rows)
    _write_csv(str(tmp_path / "w" / "run_counter_collection.csv"), ctr, w_rows)
    out = tmp_path / "out"
    bench.summarize(str(tmp_path / "t"), str(tmp_path / "f"), str(tmp_path / "w"), mib,
                    str(out), "cmd", timed=2, workload="rmat20")
    import json
    rec = json.load(open(out / "traffic_rmat20.json"))
    assert rec["fetch_factor"] == pytest.approx(2.0)
    assert rec["write_factor"] == pytest.approx(1.0)
    k = rec["per_kernel"]["k_est"]
    assert k["launches"] == 3
    assert k["avg_us"] == pytest.approx(20.0)
    assert k["avg_us_timed"] == pytest.approx(25.0)
    assert k["hbm_bytes"] == pytest.approx(100.0 * 1024 * 2.0 + 50.0 * 1024 * 1.0)
    assert "cmd" in (out / "step_kernels_rmat20.md").read_text()


def test_radix_passes_follow_the_library_choice():
    """The algorithmic bytes count the passes the library runs: 8-bit digits,
    or two 10-bit passes when bound - 1 has 17 to 20 bits; a pass whose
    digit is zero in every id skips."""
    rp = _bench().radix_passes
    assert rp(1 << 20, (1 << 20) - 1) == [True, True, False, False]   # 10-bit, C2
    assert rp(1 << 24, (1 << 24) - 1) == [True, True, True, False]    # 8-bit, C3
    assert rp(2000, 1999) == [True, True, False, False]               # 11 bits: 8-bit
    assert rp(1 << 16, 200) == [True, False, False, False]            # skipped on device
    assert rp((1 << 16) + 1, 1 << 16) == [True, True, False, False]   # 17 bits: 10-bit
    assert rp(1 << 20, 900) == [True, False, False, False]            # 10-bit, top digit 0
    assert rp(2 ** 32, 5000) == [True, True, False, False]            # no bound
    assert rp(2 ** 32, 2 ** 32 - 1) == [True] * 4


def test_profile_names_map_to_launch_names():
    short = _bench()._short
    assert short("void tc::k_scat4<1, 10>(tc::StepArgs)") == "k_scat<1>"
    assert short("void tc::k_scat<0, 8>(tc::StepArgs)") == "k_scat<0>"
    assert short("void tc::k_hist<10>(tc::StepArgs)") == "k_hist"
    assert short("void tc::k_fold_step1<8>(tc::StepArgs)") == "k_fold_step1"
    assert short("void tc::k_cscan<2, 8>(tc::StepArgs)") == "k_cscan<2>"
    assert short("tc::k_pjoin(tc::StepArgs)") == "k_pjoin"
    assert short("tc::k_est(tc::StepArgs)") == "k_est"
    assert short("void tc::k_est<true>(tc::StepArgs)") == "k_est"
    assert short("void tc::k_fold_step1<8, false>(tc::StepArgs)") == "k_fold_step1"


def test_tuning_cache_round_trip(tmp_path):
    # the tuner's JSON cache: keys by architecture, w and r buckets and key
    # bits; entries merge; a malformed entry is not returned (no GPU)
    from paper_1308_2166_amd import tune
    import paper_1308_2166_amd as tc
    k = tune.key("gfx950", 3 * 2**18, 2**16 + 5, 22)
    assert k == "gfx950|w2^19|r2^16|b22"
    path = str(tmp_path / "t.json")
    assert tune.lookup(k, path) is None
    cfg = dict(tc.DEFAULT_TUNING, chunk_tiles=16)
    tune.save({k: {"tuning": cfg, "ms_per_step": 1.0}}, path)
    tune.save({"other": {"tuning": {"chunk_tiles": 8}}}, path)
    assert tune.lookup(k, path) == cfg
    assert tune.lookup("other", path) is None
    assert set(tune.CANDIDATES) == set(tc.TUNING_FIELDS)
    for f, vals in tune.CANDIDATES.items():
        assert tc.DEFAULT_TUNING[f] in vals
