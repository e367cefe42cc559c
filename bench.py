"""Benchmark of the bulk estimator update on one MI355X.

One step = one bulk update (every step of the hot path: Step 1, the arc
grouping sort, the rank directory, Step 2, Step 3) of a bank of r estimators
by one batch of w stream edges, inputs resident in HBM.  The default workload
is the largest single-GPU one: an R-MAT scale-24 stream (2^28 distinct edges,
r = 2^22, w = 2^24), sixteen batches, so the timed steps walk fresh banks
through the stream batch 0, 1, ..., 15, 0, 1, ...  The R-MAT scale-20 stream
(r = 2^20, w = 2^22) is timed beside it as an extra entry.

Prints ONE JSON line (rank 0) with the metric, a roofline entry for the
dominant kernel (HIP-event time per launch on the step's stream) and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("r·m/s (estimator-edge updates/s) + % HBM roofline, "
          "batched vs plain, bit-exact")
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rmat20": "R-MAT scale 20, (a,b,c,d)=(0.57,0.19,0.19,0.05), 16Mi distinct "
              "edges in seeded random order, vertex ids permuted; r=2^20, w=2^22",
    "rmat24": "R-MAT scale 24, same parameters, 2^28 distinct edges; "
              "r=2^22, w=2^24 (stream resident in HBM)",
    "gnm-2k": "G(n=2000, m=20000), r=4096, w=2048",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def radix_passes(bound: int, maxid: int) -> list:
    """Which of the four radix launches move arcs for ids up to maxid under a
    declared vertex bound, as the library chooses them: 10-bit digits (two
    passes) when bound - 1 has 17 to 20 bits, else 8-bit digits; a pass
    whose digit is zero in every id skips on the device."""
    bound_bits = max(1, (bound - 1).bit_length())
    d = 10 if 16 < bound_bits <= 20 else 8
    npass = -(-bound_bits // d)
    bits = max(1, maxid.bit_length())
    return [p < npass and d * p < bits for p in range(4)]


def alg_bytes(kernel: str, w: int, r: int, nontrivial: list) -> float:
    """Bytes the step's algorithm must move per launch of `kernel` (see the
    design notes): streamed inputs/outputs only, no table or gather traffic,
    nothing for the radix bookkeeping (the fold, k_csum, k_cscan)."""
    arcs = 2 * w
    if kernel == "k_hist":
        return 8.0 * w
    if kernel.startswith("k_cnt") or kernel.startswith("k_scat"):
        p = int(kernel[kernel.index("<") + 1])
        if not nontrivial[p]:
            return 0.0
        first = not any(nontrivial[:p])
        if kernel.startswith("k_cnt"):
            return 0.0 if first else arcs * 4.0
        return arcs * ((4.0 if first else 8.0) + 8.0)
    if kernel == "k_dir":
        return arcs * 8.0
    if kernel == "k_fold_step1":
        return r * 4.0
    if kernel == "k_est":
        return r * (20.0 + 4.0 + 12.0 + 12.0)
    # Step 3: the join's partition passes read W and the closing edges,
    # write one 8-byte record per edge and per estimator at most, and the
    # join reads them back
    if kernel == "k_pcnt":
        return 8.0 * w + 8.0 * r
    if kernel == "k_pscat":
        return 16.0 * w + 16.0 * r
    if kernel == "k_pjoin":
        return 8.0 * w + 8.0 * r
    if kernel == "k_small":  # the whole step of a small chunk: W once, the state
        return 8.0 * w + 40.0 * r
    return 0.0


def cpu_baseline(E_host, r, seed, w, budget_s=12.0):
    """The oracle (paper-steps variant, one thread) on the first batches of
    the same stream, until about budget_s seconds of CPU work."""
    import oracle as O
    b = O.Bank(r, seed)
    t0 = time.perf_counter()
    nb = 0
    while nb * w < E_host.shape[0]:
        rc = b.process(E_host[nb * w:(nb + 1) * w])
        if rc != O.OK:
            raise RuntimeError(f"oracle failed: {rc}")
        nb += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return b, nb, dt


def oracle_worker(path, r, seed, w, nb):
    """Child-process mode (no GPU, no torch): the oracle on the first nb
    batches saved at `path`; prints the seconds it took."""
    import numpy as np
    import oracle as O
    E = np.load(path)
    b = O.Bank(r, seed)
    t0 = time.perf_counter()
    for k in range(nb):
        if b.process(E[k * w:(k + 1) * w]) != O.OK:
            raise SystemExit("oracle failed")
    print(json.dumps({"seconds": time.perf_counter() - t0}), flush=True)


def cpu_baseline_all_cores(E_host, r, seed, w, nb, workers):
    """The same oracle, unchanged, on every host core: the bank is split
    into `workers` independent banks of r/workers estimators (own seeds),
    each advanced over the same nb batches by its own process; the rate is
    r * nb * w over the slowest worker's time."""
    import subprocess
    import tempfile
    import numpy as np
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "batches.npy")
        np.save(path, E_host[:nb * w])
        rw = max(1, r // workers)
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                                   path, str(rw), str(seed + 1 + k), str(w), str(nb)],
                                  stdout=subprocess.PIPE, text=True)
                 for k in range(workers)]
        secs = []
        for p in procs:
            o, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError("oracle worker failed")
            secs.append(json.loads(o.strip().splitlines()[-1])["seconds"])
    worst = max(secs)
    return {"value": rw * workers * nb * w / worst, "unit": "estimator-edge updates/s",
            "cores": workers, "kind": "oracle",
            "sample": f"first {nb} batch(es) of the same stream, {workers} processes of "
                      f"r/{workers} = {rw} estimators each (own seeds), paper-steps oracle "
                      f"variant, slowest process {worst:.1f} s"}


def batched_comparison(tc, inputs, nstreams=256, ks=(1, 2, 4, 8, 16, 64), replays=3):
    """Plain (one bank per stream, one launch set per chunk) against batched
    (every stream's chunk in one launch set per step) and graph replay of the
    batched steps, on independent streams of uneven length.  Each stream is
    cut into K batches (w_s = ceil(m_s / K)).  At every K the launch shapes
    of the batched steps are tuned (paper_1308_2166_amd.tune: coordinate
    descent, cached by architecture, w and r buckets and key bits) and the
    plain form is timed too; the K with the best batched rate is the
    reported one.  Returns a dict for the JSON line."""
    import numpy as np
    import torch
    from paper_1308_2166_amd import tune
    log(f"[bench] generating {nstreams} independent streams on the GPU")
    streams = inputs.many_streams(nstreams, device="cuda")
    rs = [s["r"] for s in streams]
    seeds = [s["seed"] for s in streams]
    ms = [s["edges"].shape[0] for s in streams]
    rm_total = float(sum(r * m for r, m in zip(rs, ms)))
    stream = torch.cuda.current_stream()

    def plan(K):
        steps = []
        for k in range(K):
            ids, chunks = [], []
            for b, st in enumerate(streams):
                w = (ms[b] + K - 1) // K
                c = st["edges"][k * w:(k + 1) * w]
                if c.shape[0]:
                    ids.append(b)
                    chunks.append(c)
            steps.append((ids, chunks))
        return steps

    nv = max(st["n"] for st in streams)  # every stream's ids lie below this
    key_bits = (nv - 1).bit_length()
    mb = tc.MultiBank(rs, seeds)
    tc.tc_multi_set_vertex_bound(mb.h, nv)

    def run_batched(steps):
        tc.tc_multi_reset(mb.h, stream)
        for ids, chunks in steps:
            mb.process(ids, chunks, stream)

    def time_plain(steps, K, reps=1):
        banks = []
        for b in range(nstreams):
            bk = tc.Bank(rs[b], seeds[b])
            tc.tc_set_vertex_bound(bk.h, streams[b]["n"])
            tc.tc_reserve(bk.h, (ms[b] + K - 1) // K)
            banks.append(bk)

        def run_plain():
            for bk in banks:
                tc.tc_reset(bk.h, stream)
            for ids, chunks in steps:
                for b, c in zip(ids, chunks):
                    banks[b].process(c, stream)

        run_plain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run_plain()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        return dt, banks

    per_k, cache = {}, {}
    arch = tune.arch()
    for K in ks:
        steps = plan(K)
        tc.tc_multi_reserve(mb.h, steps[0][0], [c.shape[0] for c in steps[0][1]])
        nchunk = sum(len(ids) for ids, _ in steps)
        k_ = tune.key(arch, sum(ms) / nchunk, sum(rs) / nstreams, key_bits)
        best, t_b, trials = tune.tune(lambda: run_batched(steps),
                                      lambda cfg: tc.tc_multi_set_tuning(mb.h, cfg), repeats=1)
        default = trials[json.dumps(dict(tc.DEFAULT_TUNING), sort_keys=True)]
        t_p, banks = time_plain(steps, K)
        for bk in banks:
            bk.close()
        per_k[str(K)] = {"batched_value": rm_total / t_b, "plain_value": rm_total / t_p,
                         "batched_vs_plain": t_p / t_b, "batched_default_shapes_value":
                         rm_total / default, "tuning": best, "key": k_,
                         "configs_timed": len(trials)}
        cache[k_] = {"tuning": best, "ms_per_step": t_b * 1e3 / K}
        log(f"[bench]   K={K}: batched {rm_total / t_b:.3e} (default shapes "
            f"{rm_total / default:.3e}), plain {rm_total / t_p:.3e} r*m/s, tuning {best}")
    try:
        cache_path = tune.save(cache)
    except OSError:
        cache_path = None
    K = int(max(per_k, key=lambda k_: per_k[k_]["batched_value"]))
    steps = plan(K)
    tc.tc_multi_reserve(mb.h, steps[0][0], [c.shape[0] for c in steps[0][1]])
    tc.tc_multi_set_tuning(mb.h, per_k[str(K)]["tuning"])

    # batched (eager launches)
    run_batched(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        run_batched(steps)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / replays
    st_batched = [mb.state(b) for b in range(nstreams)]

    # the same steps captured once into a HIP graph, replayed
    tc.tc_multi_graph_reserve(mb.h, K)
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(stream)
    with torch.cuda.graph(g, stream=cs):
        tc.tc_multi_reset(mb.h, cs)
        for ids, chunks in steps:
            mb.process(ids, chunks, cs)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / replays
    graph_same = all(all(np.array_equal(x, y) for x, y in zip(mb.state(b), st_batched[b]))
                     for b in range(nstreams))

    # plain at the chosen K (default shapes): same states
    t_plain, banks = time_plain(steps, K, reps=replays)
    plain_same = all(all(np.array_equal(x, y) for x, y in zip(banks[b].state(), st_batched[b]))
                     for b in range(nstreams))
    for bk in banks:
        bk.close()
    mb.close()
    return {
        "workload": f"{nstreams} independent streams, lognormal m in [1e4, 1e7] "
                    "(median 3e5), even R-MAT scale 16-22, odd Chung-Lu n=m/8 "
                    "gamma=2.1, r=2^14..2^18 per stream",
        "total_edges": int(sum(ms)), "total_estimators": int(sum(rs)),
        "batches_per_stream": K, "per_k": per_k, "tuning_cache": cache_path,
        "plain_value": rm_total / t_plain, "batched_value": rm_total / t_batched,
        "graph_value": rm_total / t_graph, "unit": "estimator-edge updates/s",
        "batched_vs_plain": t_plain / t_batched, "graph_vs_plain": t_plain / t_graph,
        "identical_results": bool(plain_same and graph_same),
    }


def batched_profile(tc, inputs, K, reps, nstreams=256):
    """The batched form alone, for a profiler: the same streams and banks as
    the batched comparison, each stream cut into K batches; one warm-up pass,
    then `reps` passes of K steps (so a kernel's last reps*K launches are the
    measured ones)."""
    import torch
    streams = inputs.many_streams(nstreams, device="cuda")
    rs = [s_["r"] for s_ in streams]
    ms = [s_["edges"].shape[0] for s_ in streams]
    steps = []
    for k in range(K):
        ids, chunks = [], []
        for b, st in enumerate(streams):
            w = (ms[b] + K - 1) // K
            c = st["edges"][k * w:(k + 1) * w]
            if c.shape[0]:
                ids.append(b)
                chunks.append(c)
        steps.append((ids, chunks))
    mb = tc.MultiBank(rs, [s_["seed"] for s_ in streams])
    tc.tc_multi_set_vertex_bound(mb.h, max(s_["n"] for s_ in streams))
    tc.tc_multi_reserve(mb.h, steps[0][0], [c.shape[0] for c in steps[0][1]])
    stream = torch.cuda.current_stream()
    times = []
    for rep in range(reps + 1):
        tc.tc_multi_reset(mb.h, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for ids, chunks in steps:
            mb.process(ids, chunks, stream)
        torch.cuda.synchronize()
        if rep:
            times.append(time.perf_counter() - t0)
    mb.close()
    rm = float(sum(r * m for r, m in zip(rs, ms)))
    best = min(times)
    return {"form": "batched", "streams": nstreams, "batches_per_stream": K,
            "ms_per_step": round(best * 1e3 / K, 3), "value": rm / best,
            "unit": "estimator-edge updates/s"}


def host_fed(tc, G, r, seed, w, nv, reps=2):
    """The same stream fed from pinned host memory through the library
    (tc_process_host_stream: each batch is copied to one of two device
    staging buffers on the library's copy stream while the previous batch
    is processed).  Returns the PCIe-inclusive rate (never the headline
    value), the copy rate alone, and whether the state equals the resident
    stream's."""
    import numpy as np
    import torch
    m = G.shape[0]
    nb = (m + w - 1) // w
    host = torch.empty(G.shape, dtype=G.dtype, pin_memory=True)
    host.copy_(G)
    stream = torch.cuda.current_stream()
    best, state_fed = None, None
    for _ in range(reps):
        b = tc.Bank(r, seed)
        tc.tc_set_vertex_bound(b.h, nv)
        tc.tc_reserve(b.h, w)
        b.process_host_stream(host[:min(m, w)], w, stream)  # sizes the staging buffers
        tc.tc_reset(b.h, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.process_host_stream(host, w, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        state_fed = b.state()
        b.close()
        best = dt if best is None else min(best, dt)
    ref = tc.Bank(r, seed)
    ref.process_stream(G, w)
    same = all(np.array_equal(x, y) for x, y in zip(ref.state(), state_fed))
    ref.close()
    buf = torch.empty((w, 2), dtype=G.dtype, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nb):
        wk = min(w, m - k * w)
        buf[:wk].copy_(host[k * w:k * w + wk], non_blocking=True)
    torch.cuda.synchronize()
    t_copy = time.perf_counter() - t0
    return {"ms_per_step": best * 1e3 / nb, "value": r * m / best,
            "edges_per_s": m / best, "unit": "estimator-edge updates/s",
            "h2d_GBs": 8.0 * m / t_copy / 1e9, "same_state_as_resident": bool(same),
            "entry_point": "tc_process_host_stream",
            "note": "the whole stream from pinned host memory, copied by the library "
                    "(double-buffered, overlapped with the steps); PCIe-inclusive, "
                    "not the headline"}


def naive_vs_bulk(tc, inputs, shapes=((4096, 2048), (4096, 16384), (65536, 16384),
                                       (16384, 131072), (262144, 65536))):
    """Per-batch time of the per-estimator form (every estimator scans the
    batch, O(r w)) against the bulk step at small r * w, on R-MAT scale-16
    batches, with a check that both leave the same state."""
    import numpy as np
    import torch
    G = inputs.rmat(16, 16 << 16, seed=33, device="cuda")
    out = []
    for r, w in shapes:
        batches = [G[j:j + w] for j in range(0, 4 * w, w)]
        times, states = {}, {}
        for form in ("naive", "bulk"):
            b = tc.Bank(r, 9)
            tc.tc_set_vertex_bound(b.h, 1 << 16)
            tc.tc_reserve(b.h, w)
            (b.process_naive if form == "naive" else b.process)(batches[0])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in batches[1:]:
                (b.process_naive if form == "naive" else b.process)(c)
            torch.cuda.synchronize()
            times[form] = (time.perf_counter() - t0) * 1e6 / (len(batches) - 1)
            states[form] = b.state()
            b.close()
        same = all(np.array_equal(x, y) for x, y in zip(states["naive"], states["bulk"]))
        out.append({"r": r, "w": w, "naive_us": round(times["naive"], 1),
                    "bulk_us": round(times["bulk"], 1), "identical": bool(same)})
        log(f"[bench]   r={r} w={w}: naive {times['naive']:.1f} us, bulk {times['bulk']:.1f} us")
    return out


def parse_rate(tc, inputs, G, reps=3):
    """The stream as a text edge list in device memory, parsed on the device
    (tc_parse_edges, blocking, including its scratch allocation)."""
    import torch
    txt = inputs.edge_list_text(G, header="# synthetic R-MAT edge list\n")
    out = tc.tc_parse_edges(txt)
    same = bool(torch.equal(out, G))
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tc.tc_parse_edges(txt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return {"bytes": int(txt.numel()), "ms": round(best * 1e3, 3),
            "GB_per_s": round(txt.numel() / best / 1e9, 2),
            "edges_per_s": G.shape[0] / best, "round_trip_identical": same}


KERNEL_SRC = os.path.join(ROOT, "paper_1308_2166_amd", "csrc", "tc_kernels.hip")
def traffic_json(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


PROFILE_TITLES = {
    "batched": "C4 (256 streams, one batch per stream)",
    "rmat20": "R-MAT scale 20 (r=2^20, w=2^22)",
    "rmat24": "R-MAT scale 24 (r=2^22, w=2^24)",
    "gnm-2k": "G(2000, 20000) (r=4096, w=2048)",
}


def kernel_source_hash() -> str:
    """Hash of the kernel source's code: comments and blank space removed, so
    that only a change to what is compiled invalidates recorded counters."""
    import hashlib
    import re
    with open(KERNEL_SRC) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


STEP_ORDER = (["k_hist", "k_fold_step1", "k_cscan<0>", "k_scat<0>"]
              + [f"{k}<{p}>" for p in range(1, 4)
                 for k in ("k_cnt", "k_csum", "k_cscan", "k_scat")]
              + ["k_dir", "k_est", "k_pcnt", "k_pscan", "k_pscat", "k_pjoin", "k_small"])


def _short(name: str) -> str:
    """Kernel name as tc_kernel_name gives it: the digit width and the
    single-segment flag are dropped (k_scat<1, 10> is the launch k_scat<1>,
    k_hist<8> is k_hist, k_est<true> is k_est), and the four-wave build of a
    radix pass, k_scat4<P>, is the launch k_scat<P>."""
    import re
    n = re.sub(r"\(.*", "", name).replace("void ", "").replace("tc::", "").strip()
    n = re.sub(r"<(\d+), \d+>$", r"<\1>", n)
    n = re.sub(r"^(k_hist|k_fold_step1|k_est)<.*>$", r"\1", n)
    return n.replace("k_scat4<", "k_scat<")


def summarize(trace_dir, fetch_dir, write_dir, calib_mib, out_dir, command, timed=0,
              workload="rmat20"):
    """Turn rocprofv3 CSV output of this benchmark into the committed
    summaries: per-kernel average duration (kernel trace) and per-kernel HBM
    traffic from FETCH_SIZE / WRITE_SIZE, each scaled by what the counter
    reads for the calibration copy of calib_mib MiB.  timed > 0: the last
    `timed` launches of each step kernel are the benchmark's timed region
    (run with --no-batched --no-served --no-cpu-baseline) and get their own
    average."""
    import csv
    import glob
    import statistics as stt

    def rows(d, pattern):
        f = glob.glob(os.path.join(d, "**", pattern), recursive=True)
        if not f:
            raise FileNotFoundError(f"{pattern} under {d}")
        with open(f[0]) as fh:
            return list(csv.DictReader(fh))

    durs = {}
    for r in rows(trace_dir, "*kernel_trace.csv"):
        durs.setdefault(_short(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    ctr, first_copy = {}, {}
    for d, name in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        for r in rows(d, "*counter_collection.csv"):
            if r["Counter_Name"] == name:
                ctr.setdefault((_short(r["Kernel_Name"]), name), []).append(
                    float(r["Counter_Value"]))
                # the calibration copy is the run's first copy dispatch
                if "copyBuffer" in r["Kernel_Name"]:
                    did = int(r["Dispatch_Id"])
                    if name not in first_copy or did < first_copy[name][0]:
                        first_copy[name] = (did, float(r["Counter_Value"]))
    calib_bytes = calib_mib * 2**20
    fcopy = first_copy["FETCH_SIZE"][1] if "FETCH_SIZE" in first_copy else None
    wcopy = first_copy["WRITE_SIZE"][1] if "WRITE_SIZE" in first_copy else None
    ff = calib_bytes / (fcopy * 1024) if fcopy else None
    fw = calib_bytes / (wcopy * 1024) if wcopy else None
    kernels = [k for k in durs if k.startswith("k_")]
    kernels.sort(key=lambda k: STEP_ORDER.index(k) if k in STEP_ORDER else 99)
    per = {}
    lines = ["| kernel | launches | avg us | min us | max us | avg us, timed region "
             "| FETCH KiB/launch | WRITE KiB/launch | HBM bytes/launch (calibrated) |",
             "|---|---|---|---|---|---|---|---|---|"]
    for k in kernels:
        d = durs[k]
        dt_ = d[-timed:] if timed and len(d) >= timed else []
        tavg = stt.mean(dt_) if dt_ else None
        fk = stt.mean(ctr.get((k, "FETCH_SIZE"), [float("nan")]))
        wk = stt.mean(ctr.get((k, "WRITE_SIZE"), [float("nan")]))
        tb = fk * 1024 * ff + wk * 1024 * fw if ff and fw else None
        per[k] = {"launches": len(d), "avg_us": stt.mean(d), "avg_us_timed": tavg,
                  "fetch_kib": fk, "write_kib": wk, "hbm_bytes": tb}
        lines.append(f"| {k} | {len(d)} | {stt.mean(d):.2f} | {min(d):.2f} | {max(d):.2f} | "
                     + (f"{tavg:.2f}" if tavg else "n/a")
                     + f" | {fk:.0f} | {wk:.0f} | " + (f"{tb:.4g} |" if tb else "n/a |"))
    os.makedirs(out_dir, exist_ok=True)
    rec = {"kernel_source_sha256_16": kernel_source_hash(), "calib_copy_mib": calib_mib,
           "fetch_factor": ff, "write_factor": fw, "per_kernel": per,
           "command": command}
    with open(os.path.join(out_dir, f"traffic_{workload}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    with open(os.path.join(out_dir, f"step_kernels_{workload}.md"), "w") as f:
        form = "batched form" if workload == "batched" else "plain form"
        f.write(f"# Step kernels, {PROFILE_TITLES[workload]}, {form}\n\n")
        f.write("Commands (run from the repository root on one MI355X):\n\n```\n"
                + command + "\n```\n\n")
        f.write(f"Calibration: a {calib_mib} MiB device copy (`__amd_rocclr_copyBuffer`) "
                f"reads FETCH_SIZE {fcopy} KiB and WRITE_SIZE {wcopy} KiB; "
                f"scale factors {ff:.4f} (fetch) and {fw:.4f} (write) convert the "
                "counters to bytes.\n\n" if ff and fw else "No calibration copy found.\n\n")
        f.write("\n".join(lines) + "\n")
    print(json.dumps(rec, indent=1))


def summarize_l2(ctr_dir, out_dir, command, workload="rmat20"):
    """L2 (TCC) hits and misses per step kernel from one rocprofv3 --pmc run
    of TCC_HIT_sum and TCC_MISS_sum: per-launch means and the hit rate."""
    import csv
    import glob
    import statistics as stt
    f = glob.glob(os.path.join(ctr_dir, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise FileNotFoundError(f"counter_collection.csv under {ctr_dir}")
    vals = {}
    with open(f[0]) as fh:
        for r in csv.DictReader(fh):
            k = _short(r["Kernel_Name"])
            if k.startswith("k_"):
                vals.setdefault((k, r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    kernels = sorted({k for k, _ in vals}, key=lambda k: STEP_ORDER.index(k)
                     if k in STEP_ORDER else 99)
    lines = ["| kernel | launches | L2 hits/launch | L2 misses/launch | hit rate |",
             "|---|---|---|---|---|"]
    for k in kernels:
        h = vals.get((k, "TCC_HIT_sum"), [])
        m = vals.get((k, "TCC_MISS_sum"), [])
        if not h or not m:
            continue
        hm, mm = stt.mean(h), stt.mean(m)
        rate = hm / (hm + mm) if hm + mm else float("nan")
        lines.append(f"| {k} | {len(h)} | {hm:.4g} | {mm:.4g} | {rate:.3f} |")
    os.makedirs(out_dir, exist_ok=True)
    rec = {"kernel_source_sha256_16": kernel_source_hash(), "command": command,
           "per_kernel": {k: {"launches": len(vals[(k, "TCC_HIT_sum")]),
                              "hits": stt.mean(vals[(k, "TCC_HIT_sum")]),
                              "misses": stt.mean(vals[(k, "TCC_MISS_sum")])}
                          for k in kernels
                          if (k, "TCC_HIT_sum") in vals and (k, "TCC_MISS_sum") in vals}}
    with open(os.path.join(out_dir, f"l2_hits_{workload}.json"), "w") as fo:
        json.dump(rec, fo, indent=1)
    with open(os.path.join(out_dir, f"l2_hits_{workload}.md"), "w") as fo:
        fo.write(f"# L2 hits and misses of the step kernels, {PROFILE_TITLES[workload]}\n\n")
        fo.write("Commands (run from the repository root on one MI355X):\n\n```\n"
                 + command + "\n```\n\n")
        fo.write("TCC requests that hit or missed the XCD's L2, summed over its channels, "
                 "averaged over the launches of the run.\n\n")
        fo.write("\n".join(lines) + "\n")


def line_rate_ceiling(tc, table_bytes=1 << 30, n=1 << 24):
    """Random 128-byte line reads per second that this GPU serves from a
    table far above its caches (hand-written probe kernel, tc_probe_line_rate):
    one, two and four independent lines per thread and a chain of four
    dependent ones.  The largest is the ceiling of a kernel bound by random
    line reads."""
    import torch
    table = torch.zeros(table_bytes // 4, dtype=torch.int32, device="cuda")
    shapes = [(1, False), (2, False), (4, False), (4, True)]
    rates = {f"{p}{'_dependent' if d else ''}": round(
        tc.tc_probe_line_rate(table, n, p, d, reps=10) / 1e9, 2) for p, d in shapes}
    del table
    torch.cuda.empty_cache()
    return {"table_bytes": table_bytes, "threads": n, "G_lines_per_s": rates,
            "ceiling_G_lines_per_s": max(rates.values())}


def served_comparison(tc, inputs, nstreams=1024, ngraphs=64, r=1 << 16,
                      loads=(0.5, 0.9), budget=200 << 30, tight_budget=3 << 30,
                      max_step_edges=1 << 26, tight_step_edges=1 << 23, plain_group=32):
    """Continuous batching of Poisson-arriving chunks (1K-1M pairs) from
    `nstreams` streams (each replays one of `ngraphs` resident graphs with
    its own estimator seed); banks of r estimators; steps of at most
    max_step_edges edges.  Slots are what the device-byte budget allows
    (banks plus the reserved scratch of the largest step, as the library
    accounts them).  Capacity is measured with every chunk available at
    time 0; then arrivals are paced at each load fraction of it, and once
    under a budget small enough to bind.  Reports ingest latency p50/p99,
    throughput, the device bytes held, and the plain form (one bank per
    stream, one call per chunk, same chunks) for comparison."""
    import numpy as np
    import torch
    from paper_1308_2166_amd import serve
    log(f"[bench] serving: generating {ngraphs} graphs for {nstreams} streams")
    pool = inputs.many_streams(ngraphs, seed=505, device="cuda")
    graphs = [pool[s % ngraphs]["edges"] for s in range(nstreams)]
    nv = max(p["n"] for p in pool)  # every stream's ids lie below this
    seeds = [(0x9E3779B97F4A7C15 * (s + 1)) & ((1 << 63) - 1) for s in range(nstreams)]
    chunks = serve.chunk_streams(graphs, seed=6)
    nchunks = sum(len(c) for c in chunks)
    total_w = sum(int(c.shape[0]) for cs in chunks for c in cs)
    mean_chunk = total_w / nchunks
    servers = {}

    def server(bud, cap_w):
        if bud not in servers:
            servers[bud] = serve.Server(r=r, max_step_edges=cap_w, budget_bytes=bud,
                                        vertex_bound=nv, max_slots=nstreams)
        return servers[bud]

    def run(rate, bud, seed, cap_w=max_step_edges):
        srv = server(bud, cap_w)
        lat, res, el, rw = srv.run(serve.poisson_arrivals(chunks, rate, seed), seeds)
        lat = np.array(lat) * 1e3
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "value": rw / el, "elapsed_s": el, "slots": srv.slots,
                "device_bytes": srv.device_bytes(), "steps": srv.steps,
                "fused_steps": srv.fused_steps}, res

    log("[bench]   capacity run")
    run(0.0, budget, 1)
    cap, res_cap = run(0.0, budget, 1)
    capacity = cap["value"]
    out = {"workload": f"{nstreams} streams replaying {ngraphs} R-MAT/Chung-Lu graphs, "
                       f"chunks log-uniform in [1e3, 1e6] pairs, Poisson arrivals, r={r}, "
                       f"steps of at most {max_step_edges} edges",
           "chunks": nchunks, "edges": total_w, "budget_bytes": budget,
           "slots": cap["slots"], "device_bytes": cap["device_bytes"],
           "capacity": capacity, "unit": "estimator-edge updates/s", "loads": []}
    for f in loads:
        rate = f * capacity / (r * mean_chunk)
        log(f"[bench]   load {f:.0%}")
        d, res = run(rate, budget, 2)
        d["load"] = f
        out["loads"].append(d)
    # the same capacity and first-load runs with the fused small-chunk step
    # switched off (every step then takes the chain of kernels)
    log("[bench]   without the fused step")
    h = server(budget, max_step_edges).bank.h
    tun = tc.tc_multi_get_tuning(h)
    tc.tc_multi_set_tuning(h, dict(tun, fused_edges=0))
    run(0.0, budget, 1)
    cap0, res0 = run(0.0, budget, 1)
    d0, _ = run(loads[0] * capacity / (r * mean_chunk), budget, 2)
    tc.tc_multi_set_tuning(h, tun)
    out["without_fused_step"] = {"capacity": cap0["value"], "load": loads[0],
                                 "p50_ms": d0["p50_ms"], "p99_ms": d0["p99_ms"],
                                 "steps": d0["steps"]}
    log(f"[bench]   tight budget: {tight_budget} bytes")
    run(0.0, tight_budget, 1, tight_step_edges)  # warm-up of this server
    d, res_t = run(0.5 * capacity / (r * mean_chunk), tight_budget, 3, tight_step_edges)
    d["load"], d["budget_bytes"], d["max_step_edges"] = 0.5, tight_budget, tight_step_edges
    out["tight_budget"] = d
    same = all((res_cap[s].S, res_cap[s].m) == (res_t[s].S, res_t[s].m) == (res0[s].S, res0[s].m)
               for s in range(nstreams))
    for srv in servers.values():
        srv.close()
    servers.clear()
    torch.cuda.synchronize()
    # the plain form on the same chunks: one bank per stream, one
    # tc_process_batch per chunk, streams in groups whose banks are made
    # (and their scratch sized) outside the timed region
    log("[bench]   plain form on the same chunks")
    t_plain, rw_plain = 0.0, 0
    stream = torch.cuda.current_stream()
    for g0 in range(0, nstreams, plain_group):
        ids = list(range(g0, min(nstreams, g0 + plain_group)))
        banks = {}
        for s in ids:
            b = tc.Bank(r, seeds[s])
            tc.tc_set_vertex_bound(b.h, nv)
            tc.tc_reserve(b.h, max(int(c.shape[0]) for c in chunks[s]))
            banks[s] = b
        order = [(s, k) for k in range(max(len(chunks[s]) for s in ids))
                 for s in ids if k < len(chunks[s])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, k in order:
            banks[s].process(chunks[s][k], stream)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        for s in ids:
            rw_plain += r * sum(int(c.shape[0]) for c in chunks[s])
            S, m, _ = tc.tc_estimate_ex(banks[s].h)
            same = same and (S, m) == (res_cap[s].S, res_cap[s].m)
            banks[s].close()
    out["plain_value"] = rw_plain / t_plain
    out["served_vs_plain"] = capacity / out["plain_value"]
    out["identical_results"] = bool(same)
    return out


def quick_rate(tc, inputs, name, steps=16):
    """Plain-form rate of another workload: fresh banks walk its stream in
    one tc_process_stream call each (as the timed region of the headline),
    `steps` steps after one warm-up bank; no events."""
    import torch
    G, r, w, seed = inputs.workload(name, device="cuda")
    G = G.contiguous()
    nv = inputs.vertex_count(name)
    m = G.shape[0]
    nb = (m + w - 1) // w
    stream = torch.cuda.current_stream()

    def bank():
        b = tc.Bank(r, seed)
        tc.tc_set_vertex_bound(b.h, nv)
        tc.tc_reserve(b.h, w)
        return b
    warm = bank()
    warm.process_stream(G, w, stream)
    warm.sync()
    warm.close()
    banks = [bank() for _ in range((steps + nb - 1) // nb)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    for b in banks:
        cnt = min(nb, steps - k)
        b.process_stream(G[:min(m, cnt * w)], w, stream)
        k += cnt
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    edges = sum(min(w, m - (j % nb) * w) for j in range(steps))
    for b in banks:
        b.sync()
        b.close()
    b_alg = 8.0 * w + 32.0 * w + 48.0 * r
    del G
    torch.cuda.empty_cache()
    return {"workload": name, "description": WORKLOADS[name], "r": r, "w": w,
            "steps": steps, "ms_per_step": dt * 1e3 / steps, "value": r * edges / dt,
            "unit": "estimator-edge updates/s", "edges_per_s": edges / dt,
            "method_frac": round(b_alg / (dt / steps) / 1e9 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--no-extra-workload", action="store_true",
                    help="skip the extra timing of the R-MAT scale-20 stream")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the steps without events between kernels")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the plain vs batched comparison on many streams")
    ap.add_argument("--streams", type=int, default=256)
    ap.add_argument("--no-naive", action="store_true",
                    help="skip the per-estimator form comparison")
    ap.add_argument("--no-host-fed", action="store_true",
                    help="skip the run fed from pinned host memory")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the continuous-batching serving run")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (profiler calibration)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE", "FETCH", "WRITE"),
                    help="summarize rocprofv3 CSV dirs of this benchmark into profiles/")
    ap.add_argument("--summary-command", default="")
    ap.add_argument("--summary-name", default="", choices=["", "batched"],
                    help="name the profile summary for this form instead of --workload")
    ap.add_argument("--batched-profile", type=int, default=0, metavar="K",
                    help="only run the batched form (K batches per stream), "
                         "one warm-up pass then --steps passes, for a profiler")
    ap.add_argument("--summarize-l2", metavar="PMC_DIR",
                    help="summarize a TCC_HIT_sum/TCC_MISS_sum rocprofv3 run into profiles/")
    ap.add_argument("--oracle-worker", nargs=5, metavar=("NPY", "R", "SEED", "W", "NB"),
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_worker:
        path, rr, sd, ww, nbb = args.oracle_worker
        oracle_worker(path, int(rr), int(sd), int(ww), int(nbb))
        return
    if args.summarize_l2:
        summarize_l2(args.summarize_l2, os.path.join(ROOT, "profiles"),
                     args.summary_command, args.workload)
        return
    if args.summarize:
        summarize(*args.summarize, calib_mib=args.calib_copy_mib,
                  out_dir=os.path.join(ROOT, "profiles"), command=args.summary_command,
                  timed=args.steps, workload=args.summary_name or args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); "
              "the multi-GPU sharding is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1308_2166_amd as tc
    from paper_1308_2166_amd import inputs

    torch.cuda.set_device(0)
    tc.lib()
    if args.calib_copy_mib:
        # a cold source: the copied first quarter was written before three
        # more quarters pushed it out of the 256 MB memory-side cache
        n = args.calib_copy_mib << 20
        big = torch.ones(4 * n, dtype=torch.uint8, device="cuda")
        dst = torch.empty(n, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        dst.copy_(big[:n])
        torch.cuda.synchronize()
        del big, dst
    if args.batched_profile:
        print(json.dumps(batched_profile(tc, inputs, args.batched_profile, args.steps,
                                         args.streams)), flush=True)
        return
    log(f"[bench] generating {args.workload} on the GPU")
    G, r, w, seed = inputs.workload(args.workload, device="cuda")
    G = G.contiguous()
    nv = inputs.vertex_count(args.workload)  # ids lie in [0, nv)
    m = G.shape[0]
    nb = (m + w - 1) // w
    batches = [G[j:j + w] for j in range(0, m, w)]
    steps, warm = args.steps, args.warmup
    stream = torch.cuda.current_stream()

    # fresh banks: every timed step is batch (k mod nb) of a bank's stream
    nbanks = (steps + nb - 1) // nb
    log(f"[bench] m={m} r={r} w={w} batches/stream={nb} timed banks={nbanks}")
    def new_bank():
        b = tc.Bank(r, seed)
        tc.tc_set_vertex_bound(b.h, nv)
        tc.tc_reserve(b.h, w)
        return b

    warm_bank = new_bank()
    for k in range(warm):
        if k % nb == 0 and k:
            warm_bank.close()
            warm_bank = new_bank()
        warm_bank.process(batches[k % nb], stream)
    warm_bank.sync()
    warm_bank.close()

    def fresh_banks(timing, every=1):
        """timing: False, True (every kernel) or a list of kernel names, set
        on every `every`-th bank (each bank walks its stream's batches in
        order, so any subset of banks samples every batch alike)."""
        out = []
        for i in range(nbanks):
            b = new_bank()
            if timing and i % every == 0:
                tc.tc_set_kernel_timing(b.h, timing)
            out.append(b)
        torch.cuda.synchronize()
        return out

    def timed_run(banks, one_call_per_stream):
        """Walk the banks through the steps; returns wall seconds.  With
        one_call_per_stream each bank takes its batches in one
        tc_process_stream call (Step 3 of a batch overlaps the grouping of
        the next), else one tc_process_batch call per batch."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if one_call_per_stream:
            k = 0
            for b in banks:
                cnt = min(nb, steps - k)
                b.process_stream(G[:min(m, cnt * w)], w, stream)
                k += cnt
        else:
            for k in range(steps):
                banks[k // nb].process(batches[k % nb], stream)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t0
        for b in banks:
            b.sync()
        return dt_

    def kernel_totals(banks):
        tot, n = {}, 0
        for b in banks:
            t, s_ = tc.tc_kernel_times(b.h)
            n += s_
            for k_, v in t.items():
                tot[k_] = tot.get(k_, 0.0) + v
        return tot, n

    def close_all(banks):
        for b in banks:
            b.close()

    # 1. per-kernel breakdown: every kernel bracketed by events, one call per
    #    batch (kernels run one at a time, so each time is the kernel's own)
    per_kernel, timed, dom = {}, 0, None
    if not args.no_kernel_timing:
        bk = fresh_banks(True)
        timed_run(bk, False)
        per_kernel, timed = kernel_totals(bk)
        close_all(bk)
        dom = max(per_kernel, key=per_kernel.get)
        log(f"[bench] dominant kernel {dom}")
    # 2. one call per batch, no events (for comparison)
    bk = fresh_banks(False)
    per_batch_ms = timed_run(bk, False) * 1e3 / steps
    close_all(bk)
    # 3. the timed region: one tc_process_stream call per bank, events only
    #    around the dominant kernel, on every other bank (each event pair
    #    costs a few microseconds of the step)
    banks = fresh_banks([dom] if dom else False, every=2)
    log(f"[bench] timing {steps} steps")
    dt = timed_run(banks, True)
    call_forms = {"per_batch_calls": round(per_batch_ms, 4),
                  "stream_call": round(dt * 1e3 / steps, 4)}
    log(f"[bench] ms/step by call form: {call_forms}")
    edges_done = sum(batches[k % nb].shape[0] for k in range(steps))
    value = r * edges_done / dt
    log(f"[bench] {dt * 1e3 / steps:.3f} ms/step, {value:.3e} r*m/s")

    roofline = None
    if dom:
        live, live_n = kernel_totals(banks)
        # non-trivial digit passes of this stream (vertex id width)
        nontrivial = radix_passes(nv, int(G.max().item()))
        avg_ms = live[dom] / live_n
        ab = alg_bytes(dom, w, r, nontrivial)
        achieved = ab / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": dom, "avg_launch_us": round(avg_ms * 1e3, 2),
                    "alg_bytes_per_launch": ab,
                    "avg_launch_us_alone": round(per_kernel[dom] / timed * 1e3, 2)}
        try:
            with open(traffic_json(args.workload)) as f:
                rec = json.load(f)
            if (rec["kernel_source_sha256_16"] == kernel_source_hash()
                    and rec["per_kernel"].get(dom, {}).get("hbm_bytes")):
                roofline["traffic"] = rec["per_kernel"][dom]["hbm_bytes"]
                # the whole step: measured HBM bytes of every kernel it
                # launches, over the timed step time
                step_bytes = sum(v["hbm_bytes"] for k_, v in rec["per_kernel"].items()
                                 if k_ in per_kernel and per_kernel[k_] > 0 and v["hbm_bytes"])
                roofline["step_traffic_bytes"] = step_bytes
                roofline["step_traffic_GBs"] = round(step_bytes / (dt / steps) / 1e9, 1)
                roofline["step_traffic_frac"] = round(
                    step_bytes / (dt / steps) / 1e9 / HBM_PEAK_GBS, 4)
        except (OSError, KeyError, ValueError):
            pass
        # random-line view of the dominant kernel: the lines it reads per
        # second (rocprofv3 FETCH_SIZE counts 64 bytes per line request)
        # against the random-line ceiling of this GPU
        try:
            with open(traffic_json(args.workload)) as f:
                rec = json.load(f)
            if rec["kernel_source_sha256_16"] == kernel_source_hash():
                lines = rec["per_kernel"][dom]["fetch_kib"] * 1024 / 64
                rate = lines / (avg_ms * 1e-3) / 1e9
                ceil = line_rate_ceiling(tc)
                roofline["random_lines"] = {
                    "kernel": dom, "lines_per_launch": round(lines),
                    "lines_per_estimator": round(lines / r, 3),
                    "G_lines_per_s": round(rate, 2), "probe": ceil,
                    "frac_of_ceiling": round(rate / ceil["ceiling_G_lines_per_s"], 3)}
        except (OSError, KeyError, ValueError):
            pass
        step_alg = sum(alg_bytes(k_, w, r, nontrivial) for k_ in per_kernel)
        roofline["step_alg_bytes"] = step_alg
        roofline["step_alg_GBs"] = round(step_alg / (dt / steps) / 1e9, 1)
        # the method's own bytes per step: read W, write and read the 2w
        # 8-byte arcs once, read and write 24 bytes of state per estimator
        b_alg = 8.0 * w + 32.0 * w + 48.0 * r
        roofline["method_bytes_per_step"] = b_alg
        roofline["method_GBs"] = round(b_alg / (dt / steps) / 1e9, 1)
        roofline["method_frac"] = round(b_alg / (dt / steps) / 1e9 / HBM_PEAK_GBS, 4)

    out = {
        "metric": METRIC, "value": value, "unit": "estimator-edge updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": dt * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "r": r, "w": w, "m_stream": m, "vertex_bound": nv, "form": "plain"},
        "edges_per_s": edges_done / dt,
        "ms_per_step_by_call_form": call_forms,
        "roofline": roofline,
        "kernel_ms_per_step_alone": {k_: round(v / timed, 4)
                                     for k_, v in per_kernel.items()} if timed else None,
    }

    if not args.no_naive:
        log("[bench] per-estimator form vs bulk at small r*w")
        out["naive_vs_bulk"] = naive_vs_bulk(tc, inputs)

    if not args.no_host_fed:
        log("[bench] host-fed stream")
        out["host_fed"] = host_fed(tc, G, r, seed, w, nv)
        log("[bench] text edge list parsed on the device")
        # (at most the first 2^26 edges: about 1.2 GB of text)
        out["text_parse"] = parse_rate(tc, inputs, G[:1 << 26])

    if not args.no_extra_workload and args.workload != "rmat20":
        log("[bench] extra: R-MAT scale 20 stream")
        out["extra_workloads"] = {"rmat20": quick_rate(tc, inputs, "rmat20")}

    if not args.no_batched:
        out["batched"] = batched_comparison(tc, inputs, nstreams=args.streams)

    if not args.no_served:
        out["served"] = served_comparison(tc, inputs)

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        E_host = G[:2 * w].cpu().numpy().view(np.uint32)
        ob, nbo, odt = cpu_baseline(E_host, r, seed, w)
        out["cpu_baseline"] = {
            "value": r * nbo * w / odt, "unit": "estimator-edge updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"first {nbo} batch(es) of the same stream (r={r}, w={w}), "
                      f"paper-steps oracle variant, single thread, {odt:.1f} s"}
        workers = max(1, min(16, os.cpu_count() or 1))
        log(f"[bench] CPU oracle on {workers} cores")
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(E_host, r, seed, w, nbo, workers)
        # the same batches on the GPU must give the oracle's state
        chk = new_bank()
        chk.process_stream(G[:min(m, nbo * w)], w, stream)
        same = all(np.array_equal(a, b_) for a, b_ in zip(chk.state(), ob.state()))
        out["bit_exact_vs_oracle"] = bool(same)
        out["parity_sample"] = f"state after {nbo} batch(es), all {r} estimators"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
