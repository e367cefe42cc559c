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
