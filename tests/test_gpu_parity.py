"""GPU path == CPU oracle, through the C-ABI (needs an MI355X).

Estimator state (f1, f2, chi, closed) must match the oracle bit for bit
after every batch; S = sum chi*closed exactly; tau_hat within 1e-12
relative.  Inputs are the seeded synthetic streams of
``paper_1308_2166_amd.inputs``; expected values come only from ``oracle``.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1308_2166_amd import inputs

pytestmark = pytest.mark.gpu
REL_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_2166_amd as tcm
    tcm.lib()
    return tcm


def to_dev(E: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.uint32).view(np.int32)).cuda()


def assert_same(gpu_state, ora_state, where=""):
    names = ("r1", "r2", "c", "closed")
    for name, g, o in zip(names, gpu_state, ora_state):
        if not np.array_equal(g, o):
            bad = np.nonzero(g != o)[0]
            raise AssertionError(f"{where}: {name} differs at {bad.size} estimators, "
                                 f"first {bad[:5].tolist()}: gpu {g[bad[:5]].tolist()} "
                                 f"oracle {o[bad[:5]].tolist()}")


def run_both(tc, E, r, seed, w, variant="bulk", every=True):
    """Feed E in batches of w to a GPU bank and an oracle bank, comparing."""
    say(f"  run r={r} seed={seed} w={w} m={len(E)}")
    dev = to_dev(E)
    g = tc.Bank(r, seed)
    o = O.Bank(r, seed)
    for k, j in enumerate(range(0, len(E), w)):
        g.process(dev[j:j + w])
        assert o.process(E[j:j + w], variant) == O.OK
        if every or j + w >= len(E):
            assert_same(g.state(), o.state(), f"batch {k}")
    S, m, tau = tc.tc_estimate_ex(g.h)
    assert S == o.sum() and m == o.m == len(E)
    want = o.estimate()
    assert abs(tau - want) <= REL_TOL * max(1.0, abs(want))
    assert g.batch == o.batch
    return g, o


def np_edges(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


# -- the small workload: G(2000, 20000), r = 4096, w = 2048 (ragged tail) ---------

def test_gnm2k_every_batch(tc):
    G, r, w, seed = inputs.workload("gnm-2k")
    E = np_edges(G)
    g, o = run_both(tc, E, r, seed, w)
    d = O.run_stream(E, r, seed, w, variant="def")
    assert_same(g.state(), d.state(), "def variant")


@pytest.mark.parametrize("n,m,r,w", [
    (30, 120, 1, 1), (30, 120, 7, 2), (40, 300, 64, 3), (60, 500, 100, 7),
    (200, 3000, 1000, 4096), (500, 5000, 3000, 1000), (1000, 9000, 257, 2049),
    (80, 2000, 5000, 333),
])
def test_small_graphs(tc, n, m, r, w):
    E = np_edges(inputs.gnm(n, m, seed=n + m))
    run_both(tc, E, r, seed=r + w, w=w, variant="def")


def test_multi_tile_ragged(tc):
    # 2w spans several 4096-arc tiles with a ragged last one
    E = np_edges(inputs.rmat(14, 60000, seed=3))
    run_both(tc, E, r=20000, seed=9, w=9001)


@pytest.mark.parametrize("n,m,w", [(12000, 20000, 3000), (16000, 9000, 4000), (8190, 6000, 2049)])
def test_dense_directory_id_windows(tc, n, m, w):
    # ids spread over up to 4w (still the dense directory) make a tile's id
    # range span several 4096-id windows of the offsets, with gaps of empty
    # ids between the arcs
    E = np_edges(inputs.gnm(n, m, seed=n + w))
    run_both(tc, E, r=5000, seed=n, w=w)


def test_dense_directory_far_apart_ids(tc):
    # a few vertices at both ends of the dense id range: long runs of
    # absent ids inside one tile, and the last tile's run up to the top
    w = 3000
    lo = np.arange(0, 40, dtype=np.uint32)
    hi = np.arange(4 * w - 41, 4 * w - 1, dtype=np.uint32)
    ids = np.concatenate([lo, hi])
    rng = np.random.default_rng(5)
    pairs = {(int(min(a, b)), int(max(a, b))) for a, b in rng.choice(ids, (6000, 2)) if a != b}
    E = np.array(sorted(pairs), dtype=np.uint32)
    E = E[rng.permutation(len(E))]
    run_both(tc, E, r=3000, seed=11, w=w)


def test_star_giant_segment(tc):
    hub = 7
    leaves = np.arange(8, 20008, dtype=np.uint32)
    E = np.stack([np.full_like(leaves, hub), leaves], 1)
    chords = np.stack([leaves[:-1:5], leaves[1::5]], 1)
    E = np.concatenate([E, chords])
    E = E[np.random.default_rng(1).permutation(len(E))]
    run_both(tc, E, r=30000, seed=2, w=6000)


def test_wide_ids_use_the_hashed_directory(tc):
    # ids spread over [0, 2^32): max id far above the dense directory range
    E = np_edges(inputs.gnm(3000, 20000, seed=5)).astype(np.uint64)
    spread = (E * 1431655761 + 977) % (2**32 - 5)
    E = spread.astype(np.uint32)
    assert E.max() > 2**31
    run_both(tc, E, r=4096, seed=4, w=3000)


def test_ids_at_the_top_of_uint32(tc):
    E = np_edges(inputs.gnm(500, 4000, seed=6)).astype(np.uint64)
    E = (np.uint64(2**32 - 1) - E).astype(np.uint32)
    run_both(tc, E, r=2000, seed=8, w=777)


def test_repeated_edges_are_deterministic(tc):
    E = np_edges(inputs.gnm(300, 2000, seed=7))
    E = np.concatenate([E, E[:500], E[100:300]])
    run_both(tc, E, r=3000, seed=5, w=401)


def test_batch_of_one_then_large(tc):
    E = np_edges(inputs.gnm(400, 6000, seed=8))
    dev = to_dev(E)
    g, o = tc.Bank(1500, 3), O.Bank(1500, 3)
    for a, b in [(0, 1), (1, 2), (2, 5000), (5000, 5001), (5001, 6000)]:
        g.process(dev[a:b])
        o.process(E[a:b])
        assert_same(g.state(), o.state(), f"[{a},{b})")


def _random_case(k: int):
    """Configuration k of a seeded sweep: graph family and size, id layout
    (compact, strided, or spread over 32 bits so the directory is hashed),
    bank size, batch size (ragged tails), and whether a vertex bound is
    declared.  Drawn from numpy's seeded generator; nothing here depends on
    the device."""
    rng = np.random.default_rng(1000 + k)
    fam = k % 3
    if fam == 0:
        n = int(rng.integers(3, 3000))
        m = int(min(rng.integers(1, 25000), n * (n - 1) // 2))
        E = np_edges(inputs.gnm(n, m, seed=k + 1))
    elif fam == 1:
        scale = int(rng.integers(6, 14))
        n = 1 << scale
        m = int(min(rng.integers(1, 30000), n * 4))
        E = np_edges(inputs.rmat(scale, m, seed=k + 1))
    else:
        n = int(rng.integers(50, 4000))
        m = int(rng.integers(n, 8 * n))
        E = np_edges(inputs.chung_lu(n, m, seed=k + 1))
        n = int(E.max()) + 1
    layout = int(rng.integers(0, 3))
    bound = None
    if layout == 1:  # strided ids: sparse, still below a declared bound
        stride = int(rng.integers(2, 50))
        E = (E.astype(np.uint64) * stride + int(rng.integers(0, stride))).astype(np.uint32)
        bound = int(E.max()) + 1 + int(rng.integers(0, 1000))
    elif layout == 2:  # spread over [0, 2^32)
        E = ((E.astype(np.uint64) * 2654435761 + 12345) % (2**32 - 7)).astype(np.uint32)
    elif rng.integers(0, 2):
        bound = n
    r = int(rng.integers(1, 6000))
    w = int(rng.integers(1, max(2, len(E) // int(rng.integers(1, 9)) + 1)))
    seed = int(rng.integers(0, 2**63))
    return E, r, w, seed, bound, f"fam={fam} n={n} m={len(E)} layout={layout} r={r} w={w} bound={bound}"


@pytest.mark.parametrize("k", range(24))
def test_random_configurations(tc, k):
    E, r, w, seed, bound, desc = _random_case(k)
    say(f"  case {k}: {desc}")
    dev = to_dev(E)
    g, o = tc.Bank(r, seed), O.Bank(r, seed)
    if bound is not None:
        tc.tc_set_vertex_bound(g.h, bound)
    for j in range(0, len(E), w):
        g.process(dev[j:j + w])
        assert o.process(E[j:j + w]) == O.OK
    assert_same(g.state(), o.state(), desc)
    S, m, _ = tc.tc_estimate_ex(g.h)
    assert S == o.sum() and m == len(E)


# -- boundary behaviour ------------------------------------------------------------

def test_empty_batch_is_a_noop(tc):
    g = tc.Bank(10, 1)
    g.process(torch.zeros((0, 2), dtype=torch.int32, device="cuda"))
    assert g.batch == 0 and g.m == 0
    r1, r2, c, closed = g.state()
    assert np.all(r1 == tc.TC_EMPTY_EDGE) and np.all(r2 == tc.TC_EMPTY_EDGE)
    assert not c.any() and not closed.any()
    assert g.estimate() == 0.0


def test_invalid_arguments(tc):
    with pytest.raises(tc.TcError):
        tc.tc_create(0, 1)
    g = tc.Bank(4, 1)
    with pytest.raises(tc.TcError) as ei:
        tc.tc_process_batch(g.h, None, w=5)
    assert ei.value.code == tc.TC_EINVAL
    assert tc.lib().tc_process_batch(g.h, 1, tc.TC_MAX_BATCH + 1, None) == tc.TC_EINVAL
    assert g.batch == 0


def test_self_loop_is_reported(tc):
    E = np.array([[1, 2], [3, 3], [4, 5]], dtype=np.uint32)
    g = tc.Bank(8, 1)
    g.process(to_dev(E))
    with pytest.raises(tc.TcError) as ei:
        g.sync()
    assert ei.value.code == tc.TC_EBADEDGE
    with pytest.raises(tc.TcError):  # sticky
        g.process(to_dev(E[:1]))


def test_repeat_runs_are_identical(tc):
    E = np_edges(inputs.rmat(16, 200000, seed=11))
    dev = to_dev(E)
    states = []
    for _ in range(2):
        g = tc.Bank(50000, 17)
        for j in range(0, len(E), 65536):
            g.process(dev[j:j + 65536])
        states.append(g.state())
    for a, b in zip(*states):
        assert np.array_equal(a, b)


def test_kernel_timing(tc):
    E = np_edges(inputs.gnm(300, 3000, seed=2))
    g = tc.Bank(1000, 1)
    tc.tc_set_kernel_timing(g.h, True)
    g.process(to_dev(E[:1500]))
    g.process(to_dev(E[1500:]))
    times, steps = tc.tc_kernel_times(g.h)
    assert steps == 2 and len(times) == tc.tc_num_kernels()
    assert all(v >= 0 for v in times.values()) and sum(times.values()) > 0
    tc.tc_set_kernel_timing(g.h, False)
    o = O.run_stream(E, 1000, 1, 1500)
    assert_same(g.state(), o.state(), "timed")


# -- many banks in one launch set ------------------------------------------------------

def test_multi_banks_equal_their_own_streams(tc):
    rs = [1, 100, 4096, 3000, 777, 20000]
    seeds = [11, 12, 13, 14, 15, 16]
    streams = [np_edges(inputs.gnm(200 + 50 * b, 2000 + 1500 * b, seed=30 + b))
               for b in range(len(rs))]
    ws = [97, 1000, 2048, 1, 5000, 3333]
    mb = tc.MultiBank(rs, seeds)
    devs = [to_dev(E) for E in streams]
    pos = [0] * len(rs)
    step = 0
    oracles = [O.Bank(r, s) for r, s in zip(rs, seeds)]
    while any(p < len(E) for p, E in zip(pos, streams)):
        ids, chunks = [], []
        for b in range(len(rs)):
            if pos[b] >= len(streams[b]) or (b + step) % 3 == 0:
                continue  # this bank sits the step out
            w = ws[b] if b != 3 else 1 + (step * 37) % 700
            ids.append(b)
            chunks.append(devs[b][pos[b]:pos[b] + w])
            oracles[b].process(streams[b][pos[b]:pos[b] + w])
            pos[b] += w
        if not ids:
            step += 1
            continue
        mb.process(ids, chunks)
        step += 1
    S, m, tau = mb.estimate()
    for b in range(len(rs)):
        assert_same(mb.state(b), oracles[b].state(), f"bank {b}")
        assert S[b] == oracles[b].sum() and m[b] == len(streams[b])
    say(f"  {step} steps")


def test_bank_alone_equals_bank_in_a_mix(tc):
    E0 = np_edges(inputs.rmat(12, 30000, seed=1))
    E1 = np_edges(inputs.gnm(900, 30000, seed=2))
    d0, d1 = to_dev(E0), to_dev(E1)
    alone = tc.MultiBank([5000], [3])
    mix = tc.MultiBank([5000, 7000], [3, 4])
    for j in range(0, 30000, 4000):
        alone.process([0], [d0[j:j + 4000]])
        mix.process([0, 1], [d0[j:j + 4000], d1[j:j + 2500]])
    for a, b in zip(alone.state(0), mix.state(0)):
        assert np.array_equal(a, b)


def test_generators_identical_on_cpu_and_gpu(tc):
    for make in (lambda d: inputs.rmat(12, 30000, seed=4, device=d),
                 lambda d: inputs.gnm(1000, 20000, seed=5, device=d),
                 lambda d: inputs.chung_lu(5000, 30000, seed=6, device=d)):
        assert torch.equal(make("cpu"), make("cuda").cpu())


# -- the benchmark workloads at full size --------------------------------------------

def test_rmat20_full_stream(tc):
    # R-MAT scale 20, m = 16*2^20, r = 2^20, w = 2^22: every batch, full state
    say("  generating rmat20 on the GPU")
    G, r, w, seed = inputs.workload("rmat20", device="cuda")
    E = np_edges(G)
    run_both(tc, E, r, seed, w)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_rmat24_first_batches(tc):
    # R-MAT scale 24 shape: r = 2^22, w = 2^24, the first four batches (up to
    # |E| = 2^26, so Step 1 draws from bounds m + w up to 2^26), full state
    # after every batch
    say("  generating rmat24 on the GPU")
    G, r, w, seed = inputs.workload("rmat24", device="cuda")
    E = np_edges(G[:4 * w])
    del G
    torch.cuda.empty_cache()
    run_both(tc, E, r, seed, w)


def test_largest_batch_bulk_equals_per_estimator(tc):
    # one batch of TC_MAX_BATCH = 2^28 edges (the whole R-MAT scale-24
    # stream): too large for the CPU oracle, so the bulk step is checked
    # against the per-estimator kernel, an independent route to the same
    # state (itself checked against the oracle at small sizes); then a
    # second batch on top of it
    say("  generating rmat24 on the GPU")
    G, _, _, _ = inputs.workload("rmat24", device="cuda")
    assert G.shape[0] == tc.TC_MAX_BATCH
    r, seed = 256, 99
    n = inputs.vertex_count("rmat24")
    bulk, naive = tc.Bank(r, seed), tc.Bank(r, seed)
    tc.tc_set_vertex_bound(bulk.h, 2 * n)
    bulk.process(G)
    naive.process_naive(G)
    assert_same(bulk.state(), naive.state(), "largest batch")
    # second batch: new edges from existing vertices to fresh ones (none
    # repeats an edge of the first)
    k = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
    tail = torch.stack([G[:1 << 20, 0].to(torch.int64), n + k], 1).to(torch.int32).contiguous()
    bulk.process(tail)
    naive.process_naive(tail)
    assert_same(bulk.state(), naive.state(), "after a second batch")
    assert tc.tc_estimate_ex(bulk.h)[0] == tc.tc_estimate_ex(naive.h)[0]
    bulk.close()
    naive.close()
    del G
    torch.cuda.empty_cache()


# -- reset and HIP-graph replay ---------------------------------------------------------

def test_reset_gives_a_fresh_bank(tc):
    E = np_edges(inputs.gnm(500, 6000, seed=12))
    dev = to_dev(E)
    g = tc.Bank(3000, 21)
    for j in range(0, 6000, 1500):
        g.process(dev[j:j + 1500])
    tc.tc_reset(g.h)
    assert g.m == 0 and g.batch == 0
    for j in range(0, 6000, 2000):
        g.process(dev[j:j + 2000])
    o = O.run_stream(E, 3000, 21, 2000)
    assert_same(g.state(), o.state(), "after reset")


def _graph_workload(tc, nb=5, K=4):
    streams = [np_edges(inputs.rmat(11 + b % 3, 3000 + 2000 * b, seed=60 + b)) for b in range(nb)]
    rs = [500 + 700 * b for b in range(nb)]
    seeds = [70 + b for b in range(nb)]
    devs = [to_dev(E) for E in streams]
    steps = []
    for k in range(K):
        ids, chunks = [], []
        for b, E in enumerate(streams):
            w = (len(E) + K - 1) // K
            if k * w < len(E):
                ids.append(b)
                chunks.append(devs[b][k * w:(k + 1) * w])
        steps.append((ids, chunks))
    return streams, rs, seeds, steps, K


def test_graph_replay_matches_eager(tc):
    streams, rs, seeds, steps, K = _graph_workload(tc)
    mb = tc.MultiBank(rs, seeds)
    tc.tc_multi_reserve(mb.h, steps[0][0], [c.shape[0] for c in steps[0][1]])
    st = torch.cuda.current_stream()
    tc.tc_multi_reset(mb.h, st)
    for ids, chunks in steps:
        mb.process(ids, chunks, st)
    eager = [mb.state(b) for b in range(len(rs))]
    for b, E in enumerate(streams):  # eager == the oracle
        o = O.run_stream(E, rs[b], seeds[b], (len(E) + K - 1) // K)
        assert_same(eager[b], o.state(), f"eager bank {b}")

    tc.tc_multi_graph_reserve(mb.h, K)
    gr = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(st)
    with torch.cuda.graph(gr, stream=cs):
        tc.tc_multi_reset(mb.h, cs)
        for ids, chunks in steps:
            mb.process(ids, chunks, cs)
    other = tc.Bank(900, 5)
    filler = to_dev(np_edges(inputs.gnm(300, 4000, seed=13)))
    for rep in range(3):
        gr.replay()
        torch.cuda.synchronize()
        for b in range(len(rs)):
            assert_same(mb.state(b), eager[b], f"replay {rep} bank {b}")
        # the program's own eager work between replays
        other.process(filler[rep * 1000:(rep + 1) * 1000])
        _ = (filler.float() * 2).sum().item()
        torch.cuda.synchronize()


def test_graph_replay_single_bank(tc):
    E = np_edges(inputs.rmat(13, 20000, seed=14))
    dev = to_dev(E)
    mb = tc.MultiBank([4000], [31])
    tc.tc_multi_reserve(mb.h, [0], [5000])
    tc.tc_multi_graph_reserve(mb.h, 4)
    gr = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(gr, stream=cs):
        tc.tc_multi_reset(mb.h, cs)
        for j in range(0, 20000, 5000):
            mb.process([0], [dev[j:j + 5000]], cs)
    o = O.run_stream(E, 4000, 31, 5000)
    for rep in range(3):
        gr.replay()
        torch.cuda.synchronize()
        assert_same(mb.state(0), o.state(), f"replay {rep}")
        _ = torch.ones(1000, device="cuda").sum().item()


def test_graph_replay_wide_digits_many_partitions(tc):
    # the captured step runs both 10-bit passes with their chunk scans
    # (100 000-edge batches: two radix chunks) and a Step-3 join over 1024
    # partitions (r = 2^20 + 1)
    r, seed, w = (1 << 20) + 1, 41, 100000
    E = _spread_ids(np_edges(inputs.rmat(16, 300000, seed=16)), 1 << 20, 16)
    dev = to_dev(E)
    g = tc.Bank(r, seed)
    tc.tc_set_vertex_bound(g.h, 1 << 20)
    tc.tc_reserve(g.h, w)
    gr = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(gr, stream=cs):
        tc.tc_reset(g.h, cs)
        g.process_stream(dev, w, cs)
    o = O.run_stream(E, r, seed, w)
    for rep in range(3):
        gr.replay()
        torch.cuda.synchronize()
        assert_same(g.state(), o.state(), f"replay {rep}")
        _ = torch.ones(1000, device="cuda").sum().item()


def test_capture_refuses_growth_and_graph_survives_later_growth(tc):
    # (1) a step captured with less scratch reserved than it needs is refused
    # with TC_EINVAL before it synchronises, allocates or enqueues anything;
    # (2) a captured graph keeps replaying correctly after an eager step has
    # grown the bank's scratch (the block it captured is kept, not freed)
    E = np_edges(inputs.rmat(13, 30000, seed=18))
    dev = to_dev(E)
    g = tc.Bank(3000, 23)
    tc.tc_reserve(g.h, 2000)
    x = torch.zeros(16, device="cuda")
    gr = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    rc = None
    with torch.cuda.graph(gr, stream=cs):
        x.add_(1)
        rc = tc.lib().tc_process_batch(g.h, dev[:5000].data_ptr(), 5000, cs.cuda_stream)
    assert rc == tc.TC_EINVAL and g.batch == 0
    torch.cuda.synchronize()
    # (2)
    h = tc.Bank(3000, 23)
    tc.tc_reserve(h.h, 2000)
    gr2 = torch.cuda.CUDAGraph()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(gr2, stream=cs):
        tc.tc_reset(h.h, cs)
        tc.tc_process_batch(h.h, dev[:2000], stream=cs)
    gr2.replay()
    torch.cuda.synchronize()
    o = O.run_stream(E[:2000], 3000, 23, 2000)
    assert_same(h.state(), o.state(), "first replay")
    tc.tc_process_batch(h.h, dev[2000:30000])  # grows the scratch
    h.sync()
    for rep in range(2):
        gr2.replay()
        torch.cuda.synchronize()
        assert_same(h.state(), o.state(), f"replay {rep} after growth")
        _ = torch.ones(1000, device="cuda").sum().item()


# -- continuous batching: each stream's result alone == in the mix -----------------------

def test_served_streams_equal_their_alone_runs(tc):
    from paper_1308_2166_amd import serve
    nstreams, r = 24, 3000
    graphs = [inputs.rmat(10 + s % 4, 4000 + 900 * s, seed=80 + s, device="cuda")
              if s % 2 == 0 else inputs.chung_lu(600 + 50 * s, 3000 + 700 * s, seed=90 + s,
                                                 device="cuda")
              for s in range(nstreams)]
    chunks = serve.chunk_streams(graphs, seed=3, lo=200, hi=5000)
    seeds = [1000 + s for s in range(nstreams)]
    arrivals = serve.poisson_arrivals(chunks, rate_per_s=20000.0, seed=4)
    srv = serve.Server(r=r, max_step_edges=20000, slots=7)  # streams wait for slots
    lat, results, elapsed, rw = srv.run(arrivals, seeds)
    assert 0 < srv.fused_steps < srv.steps  # chunks of 200-5000 edges: both kinds of step
    # the same arrivals with every step on the chain of kernels
    tun = tc.tc_multi_get_tuning(srv.bank.h)
    tc.tc_multi_set_tuning(srv.bank.h, dict(tun, fused_edges=0))
    _, results0, _, _ = srv.run(arrivals, seeds)
    assert srv.fused_steps == 0
    srv.close()
    assert {s: (x.S, x.m) for s, x in results.items()} == {s: (x.S, x.m) for s, x in results0.items()}
    assert len(lat) == sum(len(c) for c in chunks) and len(results) == nstreams
    assert min(lat) > 0
    for s in range(nstreams):
        alone = tc.Bank(r, seeds[s])
        for c in chunks[s]:
            alone.process(c)
        S, m, tau = tc.tc_estimate_ex(alone.h)
        assert (results[s].S, results[s].m) == (S, m), s
        if s < 6:  # and the oracle agrees with the alone run
            o = O.Bank(r, seeds[s])
            for c in chunks[s]:
                o.process(np_edges(c))
            assert_same(alone.state(), o.state(), f"stream {s}")
            assert S == o.sum()


def test_served_under_a_byte_budget(tc):
    # admission by device bytes: the budget fixes the slot count, the
    # library's allocations stay under it, and results equal the alone runs
    from paper_1308_2166_amd import serve
    nstreams, r, cap = 40, 5000, 30000
    graphs = [inputs.rmat(11 + s % 3, 3000 + 400 * s, seed=300 + s, device="cuda")
              for s in range(nstreams)]
    chunks = serve.chunk_streams(graphs, seed=9, lo=300, hi=8000)
    seeds = [7000 + s for s in range(nstreams)]
    budget = serve.server_bytes(9, r, cap) + 12345  # room for 9 slots, not 10
    assert serve.slots_for_budget(budget, r, cap) == 9
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    srv = serve.Server(r=r, max_step_edges=cap, budget_bytes=budget)
    assert srv.slots == 9
    lat, results, _, _ = srv.run(serve.poisson_arrivals(chunks, 5e4, seed=2), seeds)
    torch.cuda.synchronize()
    held = srv.device_bytes()
    used = free0 - torch.cuda.mem_get_info()[0]
    assert held <= budget, (held, budget)
    assert used <= budget + (64 << 20), (used, budget)  # allocator rounding
    srv.close()
    assert len(results) == nstreams
    for s in range(0, nstreams, 5):
        alone = tc.Bank(r, seeds[s])
        for c in chunks[s]:
            alone.process(c)
        S, m, _ = tc.tc_estimate_ex(alone.h)
        assert (results[s].S, results[s].m) == (S, m), s


# -- a resident stream in one call (Step 3 of batch k overlaps batch k+1) -------

@pytest.mark.parametrize("m,w,r", [(20000, 2048, 4096), (60000, 9001, 20000),
                                   (5000, 5000, 3000), (4999, 5000, 3000),
                                   (700, 1, 50), (3001, 1000, 2000)])
def test_process_stream_equals_batches(tc, m, w, r):
    n = max(60, m // 8)
    E = np_edges(inputs.gnm(n, m, seed=m + w))
    say(f"  stream m={m} w={w} r={r}")
    dev = to_dev(E)
    g = tc.Bank(r, 17)
    g.process_stream(dev, w)
    o = O.run_stream(E, r, 17, w)
    assert_same(g.state(), o.state(), "process_stream")
    S, mm, tau = tc.tc_estimate_ex(g.h)
    assert S == o.sum() and mm == m and g.batch == o.batch == -(-m // w)
    # a second call continues the same bank (batch indices carry on)
    E2 = np_edges(inputs.gnm(n + 50, 2 * w + 3, seed=m))
    E2 = E2 + np.uint32(n + 100)  # new vertex ids: no repeated edge
    g.process_stream(to_dev(E2), w)
    for j in range(0, len(E2), w):
        assert o.process(E2[j:j + w], "bulk") == O.OK
    assert_same(g.state(), o.state(), "second call")


def test_process_stream_rmat20_first_batches(tc):
    G, r, w, seed = inputs.workload("rmat20", device="cuda")
    k = 3
    sub = G[:k * w]
    g = tc.Bank(r, seed)
    g.process_stream(sub, w)
    o = O.run_stream(np_edges(sub), r, seed, w)
    assert_same(g.state(), o.state(), "rmat20 3 batches")


def test_process_stream_in_a_graph(tc):
    E = np_edges(inputs.rmat(13, 20000, seed=15))
    dev = to_dev(E)
    g = tc.Bank(4000, 33)
    tc.tc_reserve(g.h, 3000)
    gr = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(gr, stream=cs):
        tc.tc_reset(g.h, cs)
        g.process_stream(dev, 3000, cs)
    o = O.run_stream(E, 4000, 33, 3000)
    for rep in range(3):
        gr.replay()
        torch.cuda.synchronize()
        assert_same(g.state(), o.state(), f"replay {rep}")
        _ = torch.ones(1000, device="cuda").sum().item()


def test_process_stream_arguments(tc):
    g = tc.Bank(100, 1)
    dev = to_dev(np_edges(inputs.gnm(50, 200, seed=1)))
    for w in (0, (1 << 28) + 1):
        with pytest.raises(tc.TcError) as ei:
            g.process_stream(dev, w)
        assert ei.value.code == tc.TC_EINVAL
    g.process_stream(dev[:0], 10)  # empty stream: nothing happens
    assert g.m == 0 and g.batch == 0


# -- a stream in host memory, copied by the library (double-buffered) ------------

@pytest.mark.parametrize("m,w,r,pinned", [(20000, 2048, 4096, True), (60000, 9001, 20000, True),
                                          (4999, 5000, 3000, False), (3001, 1000, 2000, False),
                                          (700, 1, 50, True)])
def test_host_stream_equals_oracle(tc, m, w, r, pinned):
    n = max(60, m // 8)
    E = np_edges(inputs.gnm(n, m, seed=m + 3 * w))
    say(f"  host stream m={m} w={w} r={r} pinned={pinned}")
    host = torch.from_numpy(E.view(np.int32).copy())
    if pinned:
        host = host.pin_memory()
    g = tc.Bank(r, 23)
    g.process_host_stream(host, w)
    o = O.run_stream(E, r, 23, w)
    assert_same(g.state(), o.state(), "host stream")
    S, mm, tau = tc.tc_estimate_ex(g.h)
    assert S == o.sum() and mm == m and g.batch == o.batch == -(-m // w)
    # a second call (from a numpy array) continues the bank with larger batches
    E2 = np_edges(inputs.gnm(n + 50, 3 * w + 5, seed=m + 1)) + np.uint32(n + 100)
    g.process_host_stream(np.ascontiguousarray(E2), 2 * w)
    for j in range(0, len(E2), 2 * w):
        assert o.process(E2[j:j + 2 * w], "bulk") == O.OK
    assert_same(g.state(), o.state(), "second call")


def test_host_stream_rmat20_equals_resident(tc):
    # the R-MAT scale-20 stream (four batches of 2^22) from pinned host
    # memory: the same state as the resident stream, and the oracle's after
    # the first two batches
    G, r, w, seed = inputs.workload("rmat20", device="cuda")
    host = G.cpu().pin_memory()
    g = tc.Bank(r, seed)
    tc.tc_set_vertex_bound(g.h, inputs.vertex_count("rmat20"))
    g.process_host_stream(host[:2 * w], w)
    o = O.run_stream(np_edges(G[:2 * w]), r, seed, w)
    assert_same(g.state(), o.state(), "host stream, two batches")
    g.process_host_stream(host[2 * w:], w)
    ref = tc.Bank(r, seed)
    ref.process_stream(G, w)
    assert_same(g.state(), ref.state(), "host stream vs resident stream")
    assert tc.tc_estimate_ex(g.h) == tc.tc_estimate_ex(ref.h)


def test_host_stream_arguments(tc):
    g = tc.Bank(100, 1)
    host = torch.from_numpy(np_edges(inputs.gnm(50, 200, seed=1)).view(np.int32).copy())
    for w in (0, (1 << 28) + 1):
        with pytest.raises(tc.TcError) as ei:
            g.process_host_stream(host, w)
        assert ei.value.code == tc.TC_EINVAL
    with pytest.raises(TypeError):
        g.process_host_stream(host.cuda(), 10)
    g.process_host_stream(host[:0], 10)  # empty stream: nothing happens
    assert g.m == 0 and g.batch == 0
    # not capturable: refused before anything is enqueued
    tc.tc_reserve(g.h, 64)
    gr = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with pytest.raises(tc.TcError) as ei:
        with torch.cuda.graph(gr, stream=cs):
            g.process_host_stream(host, 64, cs)
    assert ei.value.code == tc.TC_EINVAL
    torch.cuda.synchronize()
    assert g.m == 0
    g.process_host_stream(host, 64)
    assert g.m == 200 and g.batch == 4


# -- device memory accounting ------------------------------------------------------

def test_device_bytes_match_the_allocations(tc):
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    r, w = 1 << 20, 1 << 21
    g = tc.Bank(r, 5)
    tc.tc_reserve(g.h, w)
    torch.cuda.synchronize()
    held = tc.tc_device_bytes(g.h)
    # one bank, the step scratch, and 16 bytes of per-object words
    assert held == tc.tc_bank_bytes(r) + tc.tc_step_bytes([r], [w]) + 16
    # what the device lost: no more than reported, up to the allocator's
    # rounding of each of the ~20 allocations (at most 2 MiB each)
    used = free0 - torch.cuda.mem_get_info()[0]
    assert used <= held + (64 << 20), (held, used)
    # host-ingest staging is counted too
    host = torch.zeros((3000, 2), dtype=torch.int32).pin_memory()
    host[:, 1] = 1
    g.process_host_stream(host, 3000)
    assert tc.tc_device_bytes(g.h) == held + 16 * 3000
    g.close()


# -- declared vertex bound: fewer radix passes, same results ----------------------

@pytest.mark.parametrize("n,m,w,bound", [(200, 3000, 700, 200), (2000, 20000, 2048, 2000),
                                         (3000, 30000, 9001, 1 << 16), (250, 2000, 500, 256),
                                         (200, 3000, 700, 1 << 16)])
def test_vertex_bound_same_results(tc, n, m, w, bound):
    E = np_edges(inputs.gnm(n, m, seed=n + w))
    dev = to_dev(E)
    g = tc.Bank(3000, 21)
    tc.tc_set_vertex_bound(g.h, bound)
    g.process_stream(dev, w)
    o = O.run_stream(E, 3000, 21, w)
    assert_same(g.state(), o.state(), f"bound {bound}")


def test_vertex_bound_rmat20(tc):
    G, r, w, seed = inputs.workload("rmat20", device="cuda")
    sub = G[:2 * w]
    g = tc.Bank(r, seed)
    tc.tc_set_vertex_bound(g.h, inputs.vertex_count("rmat20"))
    for k in range(2):
        g.process(sub[k * w:(k + 1) * w])
    o = O.run_stream(np_edges(sub), r, seed, w)
    assert_same(g.state(), o.state(), "rmat20 with bound")


def test_vertex_bound_violation_is_reported(tc):
    E = np_edges(inputs.gnm(100, 800, seed=2))
    g = tc.Bank(500, 3)
    tc.tc_set_vertex_bound(g.h, 100)
    g.process(to_dev(E))
    g.sync()
    bad = E[:50].copy()
    bad[7] = (5, 150)
    g.process(to_dev(bad))
    with pytest.raises(tc.TcError) as ei:
        g.sync()
    assert ei.value.code == tc.TC_EINVAL
    with pytest.raises(tc.TcError):  # sticky
        g.process(to_dev(E[:10]))
    for n in (0, 1, (1 << 32) + 1):
        with pytest.raises(tc.TcError):
            tc.tc_set_vertex_bound(tc.Bank(10, 1).h, n)


def test_multi_vertex_bound(tc):
    rs, seeds = [700, 1500, 900], [1, 2, 3]
    Es = [np_edges(inputs.gnm(300 + 100 * b, 4000, seed=40 + b)) for b in range(3)]
    mb = tc.MultiBank(rs, seeds)
    tc.tc_multi_set_vertex_bound(mb.h, 600)
    w = 1000
    for k in range(4):
        mb.process([0, 1, 2], [to_dev(E[k * w:(k + 1) * w]) for E in Es])
    for b in range(3):
        assert_same(mb.state(b), O.run_stream(Es[b], rs[b], seeds[b], w).state(), f"bank {b}")


def test_kernel_timing_with_bound(tc):
    # passes above the bound are not launched: their times stay zero; a
    # batch of one radix chunk (8-bit digits) launches no chunk scan (the
    # fused step is switched off, so these small batches take the chain)
    E = to_dev(np_edges(inputs.gnm(200, 3000, seed=9)))
    g = tc.Bank(1000, 2)
    tc.tc_set_vertex_bound(g.h, 200)
    tc.tc_set_tuning(g.h, {"fused_edges": 0})
    tc.tc_set_kernel_timing(g.h, True)
    g.process(E[:1500])
    g.process(E[1500:])
    times, steps = tc.tc_kernel_times(g.h)
    assert steps == 2
    assert times["k_scat<0>"] > 0 and times["k_est"] > 0 and times["k_cscan<0>"] == 0.0
    assert times["k_small"] == 0.0
    for p in (1, 2, 3):
        for k in ("k_cnt", "k_csum", "k_cscan", "k_scat"):
            assert times[f"{k}<{p}>"] == 0.0


def test_kernel_timing_two_chunks(tc):
    # 75000 edges: 150000 arcs, 37 tiles, two radix chunks, so the chunk
    # scans run; a 13-bit bound launches two 8-bit passes
    E = np_edges(inputs.gnm(5000, 150000, seed=10))
    g, o = tc.Bank(3000, 5), O.Bank(3000, 5)
    tc.tc_set_vertex_bound(g.h, 5000)
    tc.tc_set_kernel_timing(g.h, True)
    dev = to_dev(E)
    for j in (0, 75000):
        g.process(dev[j:j + 75000])
        assert o.process(E[j:j + 75000]) == O.OK
    assert_same(g.state(), o.state(), "two chunks, bound 5000")
    times, steps = tc.tc_kernel_times(g.h)
    assert steps == 2
    for k in ("k_cscan<0>", "k_cnt<1>", "k_csum<1>", "k_cscan<1>", "k_scat<1>"):
        assert times[k] > 0, k
    for p in (2, 3):
        for k in ("k_cnt", "k_csum", "k_cscan", "k_scat"):
            assert times[f"{k}<{p}>"] == 0.0


# -- 10-bit digits: a declared bound of 17 to 20 bits sorts in two passes ----------

def _spread_ids(E: np.ndarray, bound: int, seed: int) -> np.ndarray:
    """E's ids (all below `bound`) sent through x -> (A x + B) mod bound with
    gcd(A, bound) = 1: a bijection of [0, bound) that spreads them over the
    whole range, so every digit bit varies."""
    import math
    rng = np.random.default_rng(seed)
    while True:
        A = int(rng.integers(max(2, bound // 16), bound))
        if math.gcd(A, bound) == 1:
            break
    B = int(rng.integers(0, bound))
    return ((E.astype(np.uint64) * A + B) % bound).astype(np.uint32)


@pytest.mark.parametrize("bound,w", [((1 << 16) + 1, 300001), ((1 << 18) + 5, 100003),
                                     (1 << 20, 65537), (1 << 20, 257)])
def test_wide_digit_bounds(tc, bound, w):
    # several radix chunks of 32 tiles (2w > 131072 arcs) with a ragged
    # tail, ids over the whole bound, two passes of 10-bit digits
    n = min(bound, 60000)
    E = _spread_ids(np_edges(inputs.gnm(n, 3 * w + 17, seed=w)), bound, seed=w)
    assert int(E.max()) < bound
    dev = to_dev(E)
    g, o = tc.Bank(5000, 7), O.Bank(5000, 7)
    tc.tc_set_vertex_bound(g.h, bound)
    for k, j in enumerate(range(0, len(E), w)):
        g.process(dev[j:j + w])
        assert o.process(E[j:j + w]) == O.OK
        assert_same(g.state(), o.state(), f"bound {bound} batch {k}")
    assert tc.tc_estimate_ex(g.h)[0] == o.sum()


def test_wide_digit_rmat_skew(tc):
    # R-MAT ids (scale 20, so the bound is 2^20): a few vertices fill whole
    # waves with one digit, which the ballot match groups
    E = np_edges(inputs.rmat(20, 600000, seed=5))
    g = tc.Bank(20000, 3)
    tc.tc_set_vertex_bound(g.h, 1 << 20)
    g.process_stream(to_dev(E), 200000)
    o = O.run_stream(E, 20000, 3, 200000)
    assert_same(g.state(), o.state(), "rmat scale 20, bound 2^20")


@pytest.mark.parametrize("id_bits", [10, 15])
def test_wide_digit_bound_above_the_ids(tc, id_bits):
    # bound 2^20 but every id below 2^10 (the second pass finds its digit
    # zero everywhere and skips on the device) or below 2^15 (its digit has
    # five bits, few enough that the count matches equal digits first)
    E = _spread_ids(np_edges(inputs.gnm(1000, 60000, seed=8)), 1 << id_bits, id_bits)
    g = tc.Bank(3000, 4)
    tc.tc_set_vertex_bound(g.h, 1 << 20)
    g.process_stream(to_dev(E), 20000)
    assert_same(g.state(), O.run_stream(E, 3000, 4, 20000).state(), f"ids below 2^{id_bits}")


def test_wide_digit_multi(tc):
    rs, seeds, w = [900, 4000, 1], [5, 6, 7], 70001
    Es = [_spread_ids(np_edges(inputs.gnm(20000, 2 * w + 99 * b, seed=60 + b)), 1 << 19, b)
          for b in range(3)]
    mb = tc.MultiBank(rs, seeds)
    tc.tc_multi_set_vertex_bound(mb.h, 1 << 19)
    for k in range(3):
        mb.process([0, 1, 2], [to_dev(E[k * w:(k + 1) * w]) for E in Es])
    for b in range(3):
        assert_same(mb.state(b), O.run_stream(Es[b], rs[b], seeds[b], w).state(), f"bank {b}")


def test_wide_digit_kernel_timing(tc):
    # a 20-bit bound launches passes 0 and 1 only
    E = to_dev(_spread_ids(np_edges(inputs.gnm(5000, 40000, seed=9)), 1 << 20, 9))
    g = tc.Bank(1000, 2)
    tc.tc_set_vertex_bound(g.h, 1 << 20)
    tc.tc_set_kernel_timing(g.h, True)
    g.process(E[:20000])
    g.process(E[20000:])
    times, steps = tc.tc_kernel_times(g.h)
    assert steps == 2
    for k in ("k_cnt", "k_csum", "k_cscan", "k_scat"):
        assert times[f"{k}<1>"] > 0
        for p in (2, 3):
            assert times[f"{k}<{p}>"] == 0.0


@pytest.mark.parametrize("bound,bad_id", [((1 << 17) + 1, (1 << 17) + 100),
                                          ((1 << 20) - 3, (1 << 20) + 7)])
def test_wide_digit_bound_violation(tc, bound, bad_id):
    E = _spread_ids(np_edges(inputs.gnm(3000, 20000, seed=3)), bound, 3)
    g = tc.Bank(800, 3)
    tc.tc_set_vertex_bound(g.h, bound)
    g.process(to_dev(E[:10000]))
    g.sync()
    bad = E[10000:].copy()
    bad[123] = (bad[123][0], bad_id)
    g.process(to_dev(bad))
    with pytest.raises(tc.TcError) as ei:
        g.sync()
    assert ei.value.code == tc.TC_EINVAL


# -- large banks: the Step-3 join over many partitions ------------------------------

def test_join_large_bank(tc):
    # r = 2^20 + 1: 1024 partitions of the waiting estimators
    E = np_edges(inputs.rmat(16, 300000, seed=12))
    r, w = (1 << 20) + 1, 100000
    g = tc.Bank(r, 8)
    g.process_stream(to_dev(E), w)
    o = O.run_stream(E, r, 8, w)
    assert_same(g.state(), o.state(), "r = 2^20 + 1")
    assert tc.tc_estimate_ex(g.h)[0] == o.sum()


def test_join_large_bank_batched(tc):
    # banks with 1 to 1024 partitions in one step, the largest at a nonzero
    # partition offset
    rs, seeds, w = [1 << 18, (1 << 20) + 1, 5000, 1 << 18, 1], [21, 22, 23, 24, 25], 30000
    Es = [np_edges(inputs.gnm(3000 + 500 * b, 90000, seed=70 + b)) for b in range(5)]
    mb = tc.MultiBank(rs, seeds)
    for k in range(3):
        mb.process(list(range(5)), [to_dev(E[k * w:(k + 1) * w]) for E in Es])
    for b in range(5):
        assert_same(mb.state(b), O.run_stream(Es[b], rs[b], seeds[b], w).state(), f"bank {b}")


# -- Step 3's partitioned join: crowded partitions, slices, few partitions ---------

def _two_hubs(n: int, seed: int) -> np.ndarray:
    """K_{2,n}: hubs 0 and 1 joined to leaves 2..n+1 in seeded order, then the
    edge between the hubs: every wedge leaf-centred between the hubs waits
    for that one closing edge."""
    rng = np.random.default_rng(seed)
    leaves = np.arange(2, n + 2, dtype=np.uint32)
    E = np.concatenate([np.stack([np.zeros(n, np.uint32), leaves], 1),
                        np.stack([np.ones(n, np.uint32), leaves], 1)])
    E = E[rng.permutation(len(E))]
    return np.concatenate([E, np.array([[1, 0]], np.uint32)])


@pytest.mark.parametrize("n,r,w", [(6000, 40000, 4001), (3000, 9000, 100000), (500, 3, 77)])
def test_join_many_estimators_wait_for_one_edge(tc, n, r, w):
    # thousands of estimators wait for the same closing edge: one partition
    # holds more than a round of the join's LDS table
    E = _two_hubs(n, seed=n)
    g, o = run_both(tc, E, r, seed=n + r, w=w)
    closed = o.state()[3]
    say(f"  closed estimators: {int(closed.sum())}")


def test_join_slices_and_partition_counts(tc):
    # few estimators against large batches (several join slices per
    # partition, one or two partitions), then many estimators against a
    # small batch (many partitions, most slices without edges)
    E = np_edges(inputs.rmat(15, 400000, seed=44))
    for r, w in ((1, 200000), (2049, 150000), (4097, 33333), (300000, 5000)):
        run_both(tc, E[:min(len(E), 2 * w + 17)], r, seed=r, w=w, every=False)


# -- the fused step of small chunks (k_small) against the chain and the oracle ------

@pytest.mark.parametrize("n,m,r,w", [(30, 120, 7, 2), (60, 500, 100, 7), (200, 3000, 1000, 2048),
                                     (1000, 9000, 257, 2047), (80, 2000, 5000, 333),
                                     (3000, 30000, 9000, 1500)])
def test_fused_step_equals_chain_and_oracle(tc, n, m, r, w):
    E = np_edges(inputs.gnm(n, m, seed=n + 7 * m))
    dev = to_dev(E)
    o = O.run_stream(E, r, 55, w)
    for fused in (0, 2048):
        g = tc.Bank(r, 55)
        tc.tc_set_tuning(g.h, {"fused_edges": fused})
        for j in range(0, len(E), w):
            g.process(dev[j:j + w])
        assert_same(g.state(), o.state(), f"fused_edges={fused}")
        assert tc.tc_estimate_ex(g.h)[0] == o.sum()


def test_fused_step_edge_cases(tc):
    # a star (one vertex in every arc), ids at the top of uint32, repeated
    # edges, a bank larger than one block's slice, and fused and chained
    # chunks in one batched step
    hub = 0xFFFFFFFE
    leaves = np.arange(5, 2005, dtype=np.uint32)
    star = np.stack([np.full_like(leaves, hub), leaves], 1)
    star = star[np.random.default_rng(2).permutation(len(star))]
    g, o = run_both(tc, star, r=9000, seed=3, w=2000)
    rep = np_edges(inputs.gnm(40, 300, seed=4))
    rep = np.concatenate([rep, rep[::-1], rep])
    run_both(tc, rep, r=5000, seed=5, w=611)
    top = (np.uint64(2**32 - 1) - np_edges(inputs.gnm(300, 4000, seed=6)).astype(np.uint64))
    run_both(tc, top.astype(np.uint32), r=20000, seed=7, w=1999)
    rs, seeds = [3000, 70000, 5000], [1, 2, 3]
    Es = [np_edges(inputs.gnm(900 + 400 * b, 20000, seed=80 + b)) for b in range(3)]
    # steps of three fused chunks (one launch, descriptors uploaded), then
    # steps mixing small chunks with one that needs the chain (all take it)
    for ws in ([2048, 1024, 700], [2048, 1024, 6000]):
        mb = tc.MultiBank(rs, seeds)
        for t in range(max(-(-len(E) // w) for E, w in zip(Es, ws))):
            ids = [b for b in range(3) if t * ws[b] < len(Es[b])]
            mb.process(ids, [to_dev(Es[b][t * ws[b]:(t + 1) * ws[b]]) for b in ids])
        for b in range(3):
            assert_same(mb.state(b), O.run_stream(Es[b], rs[b], seeds[b], ws[b]).state(),
                        f"bank {b}, chunks {ws}")
        mb.close()


def test_fused_step_errors(tc):
    # a self-loop or an id above the bound in a fused chunk is reported
    g = tc.Bank(100, 1)
    E = np_edges(inputs.gnm(50, 200, seed=1)).copy()
    E[7] = [3, 3]
    g.process(to_dev(E))
    with pytest.raises(tc.TcError) as ei:
        g.sync()
    assert ei.value.code == tc.TC_EBADEDGE
    g = tc.Bank(100, 1)
    tc.tc_set_vertex_bound(g.h, 40)
    g.process(to_dev(np_edges(inputs.gnm(50, 200, seed=1))))
    with pytest.raises(tc.TcError) as ei:
        g.sync()
    assert ei.value.code == tc.TC_EINVAL


def test_fused_kernel_timing(tc):
    E = to_dev(np_edges(inputs.gnm(300, 3000, seed=2)))
    g = tc.Bank(1000, 1)
    tc.tc_set_kernel_timing(g.h, True)
    g.process(E[:1500])
    g.process(E[1500:])
    times, steps = tc.tc_kernel_times(g.h)
    assert steps == 2 and times["k_small"] > 0
    assert all(v == 0.0 for k, v in times.items() if k != "k_small")


# -- launch shapes (tc_tuning): no choice changes a result --------------------------

def _tuning_workload():
    # banks from one to many partitions, batches of one to several radix
    # chunks (ids of up to 18 bits under a declared bound of 2^18, so the
    # digit width is a choice), repeated across three steps
    rs, seeds = [1, 3000, 70000, (1 << 19) + 5, 9000], [31, 32, 33, 34, 35]
    Es = [_spread_ids(np_edges(inputs.gnm(3000 + 900 * b, 90000 + 40000 * b, seed=60 + b)),
                      1 << 18, 60 + b) for b in range(5)]
    return rs, seeds, Es, [1700, 50000, 140000, 63000, 9000]


def test_every_tuning_choice_leaves_identical_state(tc):
    from paper_1308_2166_amd import tune
    rs, seeds, Es, ws = _tuning_workload()
    want = [O.run_stream(Es[b], rs[b], seeds[b], ws[b]).state() for b in range(5)]
    configs = [dict(tc.DEFAULT_TUNING)]
    for field, values in tune.CANDIDATES.items():
        for v in values:
            if v != tc.DEFAULT_TUNING[field]:
                c = dict(tc.DEFAULT_TUNING)
                c[field] = v
                configs.append(c)
    configs.append({"digit_bits": 8, "chunk_tiles": 8, "part_estimators": 512,
                    "join_edges": 1024, "fused_edges": 0})
    configs.append({"digit_bits": 0, "chunk_tiles": 16, "part_estimators": 8192,
                    "join_edges": 65536, "fused_edges": 1024})
    devs = [to_dev(E) for E in Es]
    for cfg in configs:
        say(f"  tuning {cfg}")
        mb = tc.MultiBank(rs, seeds)
        tc.tc_multi_set_vertex_bound(mb.h, 1 << 18)
        tc.tc_multi_set_tuning(mb.h, cfg)
        assert tc.tc_multi_get_tuning(mb.h) == cfg
        for t in range(max(-(-len(E) // w) for E, w in zip(Es, ws))):
            ids = [b for b in range(5) if t * ws[b] < len(Es[b])]
            mb.process(ids, [devs[b][t * ws[b]:(t + 1) * ws[b]] for b in ids])
        for b in range(5):
            assert_same(mb.state(b), want[b], f"bank {b}, tuning {cfg}")
        mb.close()
    # one bank too
    g = tc.Bank(20000, 9)
    tc.tc_set_tuning(g.h, {"chunk_tiles": 8, "part_estimators": 512, "join_edges": 1024})
    E = np_edges(inputs.rmat(15, 300000, seed=9))
    g.process_stream(to_dev(E), 140000)
    assert_same(g.state(), O.run_stream(E, 20000, 9, 140000).state(), "single bank, tuned")


def test_tuning_arguments(tc):
    g = tc.Bank(10, 1)
    for bad in ({"digit_bits": 10}, {"chunk_tiles": 4}, {"chunk_tiles": 24},
                {"chunk_tiles": 64}, {"part_estimators": 256}, {"part_estimators": 3000},
                {"join_edges": 512}, {"join_edges": 1 << 17}):
        with pytest.raises(tc.TcError) as ei:
            tc.tc_set_tuning(g.h, bad)
        assert ei.value.code == tc.TC_EINVAL
    assert tc.tc_get_tuning(g.h) == tc.DEFAULT_TUNING


# -- random mixes of digit widths, chunk counts and table sizes -------------------

def _mix_case(k):
    """A seeded configuration drawn over the choices the step makes by
    itself: 8- or 10-bit digits (bounds of 17 to 20 bits with ids spread
    over them), one or several radix chunks, one to 1024 Step-3 partitions
    (r above 2^20 now and then), dense or hashed directory."""
    rng = np.random.default_rng(9000 + k)
    fam = int(rng.integers(0, 3))
    m = int(rng.integers(1000, 250000))
    if fam == 0:
        n = int(rng.integers(50, 60000))
        E = np_edges(inputs.gnm(n, min(m, n * (n - 1) // 4), seed=k))
    elif fam == 1:
        sc = int(rng.integers(8, 18))
        E = np_edges(inputs.rmat(sc, min(m, (1 << sc) * 8), seed=k))
    else:
        n = int(rng.integers(1000, 60000))
        E = np_edges(inputs.chung_lu(n, min(m, n * 8), seed=k))
    kind = int(rng.integers(0, 4))
    bound = None
    if kind == 1:
        bound = (1 << int(rng.integers(17, 21))) - int(rng.integers(0, 3))
        if int(E.max()) < bound:
            E = _spread_ids(E, bound, seed=k)
        else:
            bound = None
    elif kind == 2:
        bound = int(E.max()) + 1 + int(rng.integers(0, 100))
    elif kind == 3:
        E = ((E.astype(np.uint64) * 2654435761 + 77) % (2**32 - 7)).astype(np.uint32)
    r = (1 << 20) + int(rng.integers(1, 5000)) if rng.integers(0, 6) == 0 else int(rng.integers(1, 70000))
    w = int(rng.integers(1, max(2, len(E) // int(rng.integers(1, 6)) + 1)))
    w = max(w, -(-len(E) // max(1, min(200, int(2e7 // r)))))  # bounded oracle time
    return E, r, w, bound, f"fam={fam} m={len(E)} kind={kind} bound={bound} r={r} w={w}"


@pytest.mark.parametrize("k", range(16))
def test_random_mix(tc, k):
    E, r, w, bound, desc = _mix_case(k)
    say(f"  mix {k}: {desc}")
    g, o = tc.Bank(r, 1000 + k), O.Bank(r, 1000 + k)
    if bound is not None:
        tc.tc_set_vertex_bound(g.h, bound)
    dev = to_dev(E)
    for j in range(0, len(E), w):
        g.process(dev[j:j + w])
        assert o.process(E[j:j + w]) == O.OK
    assert_same(g.state(), o.state(), desc)
    assert tc.tc_estimate_ex(g.h)[0] == o.sum()


@pytest.mark.parametrize("k", range(4))
def test_random_mix_batched(tc, k):
    rng = np.random.default_rng(7000 + k)
    nb = int(rng.integers(2, 7))
    rs = [int(rng.integers(1, 300000)) if rng.integers(0, 4) else (1 << 20) + 3 for _ in range(nb)]
    seeds = [int(rng.integers(0, 2**62)) for _ in range(nb)]
    Es = [np_edges(inputs.gnm(int(rng.integers(100, 20000)), int(rng.integers(500, 120000)),
                              seed=k * 10 + b)) for b in range(nb)]
    bound = None
    if rng.integers(0, 2):
        bound = 1 << int(rng.integers(17, 21))
        Es = [_spread_ids(E, bound, seed=k * 10 + b) for b, E in enumerate(Es)]
    w = int(rng.integers(10000, 70000))
    say(f"  batched mix {k}: nb={nb} rs={rs} w={w} bound={bound}")
    mb = tc.MultiBank(rs, seeds)
    if bound:
        tc.tc_multi_set_vertex_bound(mb.h, bound)
    for t in range(max(-(-len(E) // w) for E in Es)):
        ids = [b for b in range(nb) if t * w < len(Es[b])]
        mb.process(ids, [to_dev(Es[b][t * w:(t + 1) * w]) for b in ids])
    for b in range(nb):
        assert_same(mb.state(b), O.run_stream(Es[b], rs[b], seeds[b], w).state(), f"bank {b}")


# -- median-of-means aggregate -----------------------------------------------------

def _assert_mom(got, want):
    (tg, sg), (to, so) = got, want
    assert list(map(int, sg)) == list(map(int, so))
    assert abs(tg - to) <= REL_TOL * max(1.0, abs(to))


@pytest.mark.parametrize("groups", [1, 2, 7, 64, 4095, 4096])
def test_mom_matches_oracle_gnm2k(tc, groups):
    G, r, w, seed = inputs.workload("gnm-2k")
    E = np_edges(G)
    g = tc.Bank(r, seed)
    g.process_stream(to_dev(E), w)
    o = O.run_stream(E, r, seed, w)
    _assert_mom(tc.tc_estimate_mom(g.h, groups), o.mom(groups))


def test_mom_matches_oracle_rmat20(tc):
    G, r, w, seed = inputs.workload("rmat20", device="cuda")
    sub = G[:2 * w]
    g = tc.Bank(r, seed)
    g.process_stream(sub, w)
    o = O.run_stream(np_edges(sub), r, seed, w)
    for groups in (1, 9, 1024, r):
        _assert_mom(tc.tc_estimate_mom(g.h, groups), o.mom(groups))
    # the plain estimate through the same group-sum kernel
    S, m, tau = tc.tc_estimate_ex(g.h)
    assert S == o.sum() and abs(tau - o.estimate()) <= REL_TOL * o.estimate()


def test_multi_mom_and_arguments(tc):
    rs, seeds = [700, 1500, 333], [1, 2, 3]
    Es = [np_edges(inputs.gnm(300 + 100 * b, 4000, seed=60 + b)) for b in range(3)]
    mb = tc.MultiBank(rs, seeds)
    w = 1000
    for k in range(4):
        mb.process([0, 1, 2], [to_dev(E[k * w:(k + 1) * w]) for E in Es])
    for b in range(3):
        o = O.run_stream(Es[b], rs[b], seeds[b], w)
        for groups in (1, 5, rs[b]):
            _assert_mom(tc.tc_multi_estimate_mom(mb.h, b, groups), o.mom(groups))
    for bad in (0, rs[0] + 1):
        with pytest.raises(tc.TcError) as ei:
            tc.tc_multi_estimate_mom(mb.h, 0, bad)
        assert ei.value.code == tc.TC_EINVAL


# -- the per-estimator (naive) form: an independent path to the same state ---------

@pytest.mark.parametrize("n,m,r,w", [(30, 120, 7, 2), (60, 500, 100, 7), (200, 3000, 1000, 4096),
                                     (1000, 9000, 257, 2049), (2000, 20000, 4096, 2048)])
def test_naive_equals_oracle(tc, n, m, r, w):
    E = np_edges(inputs.gnm(n, m, seed=n + m))
    dev = to_dev(E)
    g = tc.Bank(r, r + w)
    o = O.Bank(r, r + w)
    for k, j in enumerate(range(0, len(E), w)):
        g.process_naive(dev[j:j + w])
        assert o.process(E[j:j + w], "def") == O.OK
        assert_same(g.state(), o.state(), f"batch {k}")
    assert tc.tc_estimate_ex(g.h)[0] == o.sum()


def test_naive_and_bulk_interleave(tc):
    E = np_edges(inputs.rmat(13, 30000, seed=17))
    dev = to_dev(E)
    w, r = 3000, 5000
    banks = [tc.Bank(r, 44) for _ in range(3)]  # naive, alternating, bulk
    for k, j in enumerate(range(0, len(E), w)):
        c = dev[j:j + w]
        banks[0].process_naive(c)
        (banks[1].process_naive if k % 2 else banks[1].process)(c)
        banks[2].process(c)
        ref = banks[2].state()
        assert_same(banks[0].state(), ref, f"naive, batch {k}")
        assert_same(banks[1].state(), ref, f"alternating, batch {k}")


def test_naive_boundary(tc):
    g = tc.Bank(50, 1)
    E = to_dev(np_edges(inputs.gnm(40, 200, seed=3)))
    g.process_naive(E[:0])
    assert g.m == 0 and g.batch == 0
    g.process_naive(E[:100])
    assert g.m == 100 and g.batch == 1
    bad = np_edges(inputs.gnm(40, 50, seed=4)).copy()
    bad[3] = (9, 9)
    g.process_naive(to_dev(bad))
    with pytest.raises(tc.TcError) as ei:
        g.sync()
    assert ei.value.code == tc.TC_EBADEDGE


# -- text edge lists parsed on the device -------------------------------------------

def _ref_parse(text: bytes):
    from oracle.parse import parse_edge_list
    return parse_edge_list(text)


def _dev_bytes(b: bytes) -> torch.Tensor:
    return torch.tensor(list(b), dtype=torch.uint8).cuda()


def test_parse_handmade_texts(tc):
    texts = [
        b"1 2\n3 4\n",
        b"# SNAP header\n# Nodes: 5\n1\t2\r\n3\t4\r\n\n5 6",
        b"% matrix market style\n7,8\n  9   10  \n4294967295 0\n",
        b"",
        b"#only a comment",
        b"12 34\n#c 99 98\n56\t78\n" * 1000,
    ]
    # a long line (under the 4096-byte limit) and tokens across 256-byte thread spans
    texts.append(b" " * 3000 + b"11 22\n" + b"1" * 9 + b" " + b"2" * 9 + b"\n")
    texts.append(b"".join(b"%d %d\n" % (i, i * 7 + 1) for i in range(70000)))
    # text denser than four bytes per id (more ids than a block stages)
    texts.append(b"1 2\n" * 20000 + b"3,4\n" * 20000)
    # ids and comment lines crossing 128-byte thread slices and 32 KB tiles
    texts.append(b"".join((b"#" + b"x" * (i % 300) + b"\n" if i % 7 == 0 else
                           b"%d%s%d\n" % (i * 104729 % 4294967291, b" " * (1 + i % 37),
                                          i * 7919 % 4294967291)) for i in range(9000)))
    for t in texts:
        got = tc.tc_parse_edges(_dev_bytes(t)) if t else tc.tc_parse_edges(
            torch.empty(0, dtype=torch.uint8, device="cuda"))
        want = _ref_parse(t)
        assert got.shape[0] == want.shape[0]
        assert np.array_equal(got.cpu().numpy().view(np.uint32).astype(np.uint64), want)


def test_parse_misaligned_text(tc):
    # a text that does not start on a 16-byte boundary (a view into a larger
    # buffer) is staged byte by byte; the result is the same
    G = inputs.gnm(3000, 40000, seed=44, device="cuda")
    txt = inputs.edge_list_text(G, sep=" ", header="# shifted\n")
    for shift in (1, 3, 8):
        buf = torch.zeros(txt.numel() + 16, dtype=torch.uint8, device="cuda")
        buf[shift:shift + txt.numel()] = txt
        got = tc.tc_parse_edges(buf[shift:shift + txt.numel()])
        assert torch.equal(got, G), f"shift {shift}"


def test_parse_round_trip_and_process(tc):
    G = inputs.rmat(14, 60000, seed=31, device="cuda")
    for sep in ("\t", " ", ", "):
        txt = inputs.edge_list_text(G, sep=sep, header="# R-MAT scale 14\n% second comment\n")
        got = tc.tc_parse_edges(txt)
        assert torch.equal(got, G)
    # the parsed stream through the step, against the oracle on the original
    g = tc.Bank(20000, 5)
    g.process_stream(got, 9001)
    o = O.run_stream(np_edges(G), 20000, 5, 9001)
    assert_same(g.state(), o.state(), "parsed stream")


def test_parse_errors(tc):
    for bad in (b"1 2 3\n", b"4294967296 1\n", b"1 " + b" " * 5000 + b"2\n"):
        with pytest.raises(tc.TcError) as ei:
            tc.tc_parse_edges(_dev_bytes(bad))
        assert ei.value.code == tc.TC_EINVAL
    with pytest.raises(tc.TcError):
        tc.tc_parse_edges(_dev_bytes(b"1 2\n3 4\n5 6\n"), max_edges=2)


def test_probe_line_rate(tc):
    # the diagnostic behind the random-line roofline: a positive, finite
    # rate for every shape, reads only (the table is left as it was)
    table = torch.arange(1 << 22, dtype=torch.int32, device="cuda")  # 16 MB
    before = table.clone()
    for per, dep in ((1, False), (2, False), (4, True), (8, False)):
        rate = tc.tc_probe_line_rate(table, 1 << 16, per, dep, reps=2)
        assert 1e6 < rate < 1e13, (per, dep, rate)
    assert torch.equal(table, before)
    with pytest.raises(tc.TcError):
        tc.tc_probe_line_rate(table[:10], 1 << 10)  # 40 bytes: not whole lines
