"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the expected values come from
the paper's worked example (Figs. 1-3), published test vectors, brute force
on tiny graphs, the exact law of an NBSI estimator (Claim 1, Lemma 1), and
the reduction of the bulk update to the per-edge sampler when w = 1.
"""
import numpy as np
import pytest
from scipy import stats

import brute
import oracle as O
from conftest import golden

A, B, C, D, E, F = range(6)
NAMES = {ch: i for i, ch in enumerate("ABCDEF")}
FIG1_W = [(B, C), (C, D), (E, F), (B, D), (D, F)]  # Fig. 1 solid edges, pos 1..5


# -- random protocol ---------------------------------------------------------

def test_splitmix64_published_stream():
    want = [int(r[0], 16) for r in golden("splitmix64_seed0.txt")]
    got = [O.mix64((k * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)) for k in range(1, 6)]
    assert got == want


def test_lemire_fixed_points():
    assert O.lemire_step(123456789, 1) == (0, False)
    # 2^63*10 = 5*2^64 has low half 0 < 2^64 mod 10 = 6: rejected
    assert O.lemire_step(1 << 63, 10) == (5, True)
    assert O.lemire_step((1 << 63) + (1 << 60), 10) == (5, False)
    # 2^64 mod 3 = 1, so the single low half 0 is rejected
    assert O.lemire_step(0, 3) == (0, True)
    assert O.lemire_step(1, 3) == (0, False)
    top = (1 << 64) - 1
    assert O.lemire_step(top, top) == (top - 1, False)
    rng = np.random.default_rng(0)
    for _ in range(200):
        x = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        n = int(rng.integers(1, 1 << 62))
        v, _ = O.lemire_step(x, n)
        assert v == (x * n) >> 64 and v < n


def test_lemire_rejection_makes_uniform():
    # n = 3*2^62: multiply-shift alone gives v = 0 mod 3 twice the mass of
    # the other residues; the rejection step must remove exactly that excess
    n = 3 << 62
    res = np.array([O.uniform(9, i, 0, 1, n) % 3 for i in range(30000)])
    counts = np.bincount(res, minlength=3)
    assert stats.chisquare(counts).pvalue > 1e-6
    small = np.bincount([O.uniform(4, i, 7, 2, 7) for i in range(14000)], minlength=7)
    assert stats.chisquare(small).pvalue > 1e-6


def test_python_and_c_keyed_draws_agree():
    for est in range(50):
        for batch in (0, 1, 17):
            for purpose in (1, 2):
                n = 1 + est * 7919 + batch
                assert O.uniform(11, est, batch, purpose, n) == \
                    brute.draw(11, est, batch, purpose, n)


# -- worked example, Sec. 4.3 (Figs. 1-3) --------------------------------------

def test_fig2_rankall_output():
    src, dst, rank, pos = O.rank_all(FIG1_W)
    want = golden("fig2_rankall.txt")
    assert [NAMES[r[0]] for r in want] == src.tolist()
    assert [NAMES[r[1]] for r in want] == dst.tolist()
    assert [int(r[2]) - 1 for r in want] == pos.tolist()
    assert [int(r[3]) for r in want] == rank.tolist()


def test_fig1_rank_table():
    for x, y, rk in golden("fig1_ranks.txt"):
        assert O.rank(FIG1_W, NAMES[x], NAMES[y]) == int(rk)


def test_fig3_phi_naming():
    for u, v, phi, edge in golden("fig3_phi.txt"):
        p = O.phi_pos(FIG1_W, NAMES[u], NAMES[v], int(phi))
        assert set(FIG1_W[p]) == {NAMES[edge[0]], NAMES[edge[1]]}


# Hand trace of one batch on the Fig. 1 graph.  Earlier (dashed) edges are
# E = <AC, CE, AD>: the figure shows AC and CE (C->A has rank deg_W(C) = 2;
# f1 = CE appears in Fig. 3); the third dashed edge is not recoverable from
# the text, AD is this test's choice.  Draws are forced per (batch, est,
# purpose); the expected states below are worked out by hand.
E_EARLY = [(A, C), (C, E), (A, D)]
FORCED = {
    0: {1: [0, 0, 0, 0, 1, 0], 2: {0: 0, 1: 0, 2: 0, 3: 0, 5: 1}},
    1: {1: [3, 3, 4, 0, 2, 1], 2: {0: 1, 1: 0, 2: 1, 3: 0, 4: 2, 5: 3}},
}
BOUNDS = {0: {1: 3, 2: {0: 2, 1: 2, 2: 2, 3: 2, 5: 2}},
          1: {1: 8, 2: {0: 2, 1: 2, 2: 2, 3: 4, 4: 3, 5: 4}}}
HAND = [  # (f1, f2, chi, closed) after the batch W
    ((B, C), (C, D), 2, 1),  # phi=1 -> CD at 2; closing BD at 4 > 2
    ((B, C), (B, D), 2, 0),  # phi=0 -> BD at 4; closing CD at 2 < 4
    ((C, D), (B, D), 2, 0),  # u=C,v=D: ld=0, rd=2; phi=1 -> BD; BC at 1 < 4
    ((A, C), (A, D), 4, 1),  # f2 kept (y=0 < 2); closing CD arrives in W
    ((C, E), (E, F), 3, 0),  # Fig. 3 right: phi=2 -> EF; CF never arrives
    ((A, C), (B, C), 4, 0),  # y=3 -> phi=1 -> (C, rank 1) = BC; AB absent
]


@pytest.mark.parametrize("variant", ["def", "bulk"])
def test_hand_traced_batch(variant):
    bank = O.Bank(6, seed=0)
    for b, W in enumerate([E_EARLY, FIG1_W]):
        seen = []

        def hook(ctx, est, purpose, n, b=b, seen=seen):
            if purpose == 1:
                assert n == BOUNDS[b][1]
                return FORCED[b][1][est]
            assert n == BOUNDS[b][2][est]
            seen.append(est)
            return FORCED[b][2][est]

        assert bank.process(W, variant, draw=hook) == O.OK
        assert sorted(seen) == sorted(FORCED[b][2])
    r1, r2, c, closed = bank.state()
    for i, (f1, f2, chi, cl) in enumerate(HAND):
        assert int(r1[i]) == brute.canon(*f1), i
        assert int(r2[i]) == brute.canon(*f2), i
        assert int(c[i]) == chi, i
        assert int(closed[i]) == cl, i
    assert bank.sum() == 2 + 4 and bank.m == 8 and bank.batch == 2


# -- invariants and reductions on random tiny graphs -----------------------------

def _random_graph(n, m, seed):
    from paper_1308_2166_amd import inputs
    return inputs.gnm(n, m, seed).numpy().astype(np.uint32)


@pytest.mark.parametrize("w", [1, 2, 3, 7, 300])
def test_invariants_after_every_batch(w):
    G = _random_graph(40, 150, seed=w)
    codes = brute.stream_codes(G)
    bank = O.Bank(64, seed=100 + w)
    for j in range(0, len(G), w):
        assert bank.process(G[j:j + w], "bulk") == O.OK
        r1, r2, c, closed = bank.state()
        assert brute.check_invariants(codes[:j + w], r1, r2, c, closed) == []


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_w1_reduces_to_per_edge_sampler(seed):
    G = _random_graph(25, 90, seed=seed)
    codes = brute.stream_codes(G)
    bank = O.run_stream(G, r=40, seed=seed, w=1)
    got = bank.state()
    want = brute.per_edge_sampler(codes, 40, seed)
    for g, wv in zip(got, want):
        assert [int(x) for x in g] == list(wv)


@pytest.mark.parametrize("w", [1, 5, 64, 4096])
def test_def_equals_bulk(w):
    G = _random_graph(300, 4000, seed=9)
    a = O.run_stream(G, r=257, seed=5, w=w, variant="def")
    b = O.run_stream(G, r=257, seed=5, w=w, variant="bulk")
    for x, y in zip(a.state(), b.state()):
        np.testing.assert_array_equal(x, y)
    assert a.m == b.m == 4000


def test_def_equals_bulk_star_and_wide_ids():
    # a star (one huge segment) plus ids near 2^32
    hub = 0xFFFFFFF0
    star = np.array([(hub, i) for i in range(1, 400)] +
                    [(i, i + 1) for i in range(1, 399, 3)], dtype=np.uint32)
    rng = np.random.default_rng(3)
    star = star[rng.permutation(len(star))]
    a = O.run_stream(star, r=300, seed=8, w=37, variant="def")
    b = O.run_stream(star, r=300, seed=8, w=37, variant="bulk")
    for x, y in zip(a.state(), b.state()):
        np.testing.assert_array_equal(x, y)
    codes = brute.stream_codes(star)
    assert brute.check_invariants(codes, *b.state()) == []


# -- the exact law of an estimator (Claim 1, Lemma 1) ----------------------------

def test_distribution_matches_claim1():
    G = _random_graph(14, 40, seed=21)
    codes = brute.stream_codes(G)
    m = len(codes)
    r = 40000
    bank = O.run_stream(G, r=r, seed=77, w=7)
    r1, r2, c, closed = bank.state()
    pos = {e: i for i, e in enumerate(codes)}
    # f1 uniform on E
    cnt1 = np.bincount([pos[int(e)] for e in r1], minlength=m)
    assert stats.chisquare(cnt1).pvalue > 1e-6
    # f2 uniform on Gamma(f1): pooled over every (f1, f2) pair
    obs, exp = [], []
    for i in range(m):
        g = brute.gamma(codes, i)
        sel = r1 == codes[i]
        if not g:
            assert np.all(r2[sel] == brute.EMPTY)
            continue
        k = np.bincount([pos[int(e)] for e in r2[sel]], minlength=m)
        for j in g:
            obs.append(k[j])
            exp.append(r / m / len(g))
    obs, exp = np.array(obs, float), np.array(exp)
    assert stats.chisquare(obs, exp * obs.sum() / exp.sum()).pvalue > 1e-6
    # P(closed) = sum over triangles of 1/(m C(t))
    p = sum(1.0 / (m * len(brute.gamma(codes, t[0]))) for t in brute.triangles(codes))
    z = (closed.sum() - r * p) / np.sqrt(r * p * (1 - p))
    assert abs(z) < 5


def test_unbiased_with_exact_variance():
    G = _random_graph(22, 110, seed=5)
    codes = brute.stream_codes(G)
    tau, ex2 = brute.exact_moments(codes)
    assert tau > 10
    var_x = ex2 - tau * tau
    r, S = 2000, 20
    ests = [O.run_stream(G, r=r, seed=1000 + s, w=16).estimate() for s in range(S)]
    z = (np.mean(ests) - tau) / np.sqrt(var_x / (r * S))
    assert abs(z) < 5


def test_small_workload_estimate_near_truth():
    from paper_1308_2166_amd import inputs
    G, r, w, seed = inputs.workload("gnm-2k")
    G = G.numpy().astype(np.uint32)
    codes = brute.stream_codes(G)
    tau = len(brute.triangles(codes))
    bank = O.run_stream(G, r=r, seed=seed, w=w)
    assert bank.m == 20000 and bank.batch == 10
    # generous 6-sigma band from the exact single-estimator variance
    _, ex2 = brute.exact_moments(codes)
    sd = np.sqrt((ex2 - tau * tau) / r)
    assert abs(bank.estimate() - tau) < 6 * sd


# -- boundary behaviour -------------------------------------------------------------

@pytest.mark.parametrize("variant", ["def", "bulk"])
def test_errors_and_empty_batches(variant):
    bank = O.Bank(5, seed=1)
    assert bank.process(np.zeros((0, 2), np.uint32), variant) == O.OK
    assert bank.batch == 0 and bank.m == 0
    assert bank.process([(1, 2), (3, 3)], variant) == O.EBADEDGE
    assert bank.batch == 0 and bank.m == 0
    r1, _, _, _ = bank.state()
    assert np.all(r1 == brute.EMPTY)
    assert bank.process([(1, 2)], variant) == O.OK
    r1, r2, c, closed = bank.state()
    assert np.all(r1 == brute.canon(1, 2)) and np.all(r2 == brute.EMPTY)
    assert np.all(c == 0) and not closed.any() and bank.m == 1


def test_duplicate_edges_are_deterministic():
    G = _random_graph(30, 100, seed=4)
    G = np.concatenate([G, G[:30]])  # caller-contract violation: repeats
    a = O.run_stream(G, r=100, seed=2, w=13, variant="def")
    b = O.run_stream(G, r=100, seed=2, w=13, variant="bulk")
    for x, y in zip(a.state(), b.state()):
        np.testing.assert_array_equal(x, y)


# -- median-of-means aggregate and Theorem 2 sizing -----------------------------------

def _bank_with(c, closed, m):
    """An oracle bank whose (c, closed, |E|) are set directly (test only)."""
    bank = O.Bank(len(c), seed=1)
    st = bank._p.contents
    np.ctypeslib.as_array(st.c, shape=(len(c),))[:] = np.asarray(c, np.uint32)
    np.ctypeslib.as_array(st.closed, shape=(len(c),))[:] = np.asarray(closed, np.uint8)
    st.m = m
    return bank


def test_mom_hand_example():
    # X_i = c_i * closed_i * m = 30, 0, 40, 10, 0, 90 (m = 10)
    bank = _bank_with([3, 1, 4, 1, 5, 9], [1, 0, 1, 1, 0, 1], m=10)
    # g = 3: groups {0,1} {2,3} {4,5}: S = 3, 5, 9; means 15, 25, 45
    tau, sums = bank.mom(3)
    assert list(sums) == [3, 5, 9] and tau == 25.0
    # g = 4: groups {0} {1,2} {3} {4,5}: means 30, 20, 10, 45 -> (20 + 30) / 2
    tau, sums = bank.mom(4)
    assert list(sums) == [3, 4, 1, 9] and tau == 25.0
    # g = r: the median of the single estimators, (10 + 30) / 2
    assert bank.mom(6)[0] == 20.0
    # g = 1 is Lemma 1's mean: 17 * 10 / 6
    assert abs(bank.mom(1)[0] - 170.0 / 6.0) < 1e-12 and bank.mom(1)[0] == bank.estimate()
    for g in (0, 7):
        assert np.isnan(bank.mom(g)[0])


def test_mom_groups_partition_the_bank():
    G = _random_graph(30, 120, seed=4)
    bank = O.run_stream(G, r=1001, seed=8, w=17)
    S = bank.sum()
    _, _, c, closed = bank.state()
    x = c.astype(np.uint64) * closed
    for g in (1, 2, 7, 13, 1000, 1001):
        tau, sums = bank.mom(g)
        assert int(sums.sum()) == S
        bounds = [k * 1001 // g for k in range(g + 1)]
        assert [int(x[bounds[k]:bounds[k + 1]].sum()) for k in range(g)] == [int(v) for v in sums]
        means = sorted(int(s) * bank.m / (bounds[k + 1] - bounds[k]) for k, s in enumerate(sums))
        want = means[g // 2] if g % 2 else 0.5 * (means[g // 2 - 1] + means[g // 2])
        assert abs(tau - want) <= 1e-12 * max(1.0, abs(want))


def test_estimators_needed_is_theorem_2():
    # 96 / 0.25 * 30 * 6 / 10 * ln 10 = 15915.47...
    assert O.estimators_needed(0.5, 0.1, 30, 6, 10.0) == 15916
    assert O.estimators_needed(0.1, 0.01, 1000, 50, 2000.0) == int(np.ceil(
        96 / 0.01 * 1000 * 50 / 2000.0 * np.log(100.0)))
    for bad in ((0.0, 0.1, 30, 6, 10.0), (0.5, 0.0, 30, 6, 10.0), (0.5, 1.0, 30, 6, 10.0),
                (0.5, 0.1, 30, 6, 0.0)):
        assert O.estimators_needed(*bad) == 0


def test_theorem_2_guarantee_holds():
    # with Theorem 2's r, the median-of-means estimate is within eps * tau
    # in (well over) a 1 - delta fraction of independent runs
    G = _random_graph(14, 48, seed=6)
    codes = brute.stream_codes(G)
    tau = len(brute.triangles(codes))
    deg = np.bincount(G.ravel().astype(np.int64))
    eps, delta = 0.5, 0.2
    r = O.estimators_needed(eps, delta, len(G), int(deg.max()), float(tau))
    assert 1000 < r < 200000
    ok = 0
    for s in range(10):
        bank = O.run_stream(G, r=r, seed=700 + s, w=8)
        est, _ = bank.mom(9)
        ok += abs(est - tau) <= eps * tau
    assert ok >= 8


# -- the reference parser of text edge lists ------------------------------------------

def test_reference_parser_pins():
    from oracle.parse import ParseError, parse_edge_list

    def P(t):
        return parse_edge_list(t).tolist()

    assert P(b"1 2\n3 4\n") == [[1, 2], [3, 4]]
    assert P(b"") == [] and P(b"# only a comment") == []
    # comments ('#', '%' first), CRLF, tabs, commas, runs of separators,
    # a missing final newline
    assert P(b"# SNAP\n% mm\n10\t20\r\n 30 ,  40 \n50 60") == [[10, 20], [30, 40], [50, 60]]
    # a '#' later in a line is a separator, not a comment
    assert P(b"7 # 8\n") == [[7, 8]]
    # the largest id
    assert P(b"4294967295 0\n") == [[4294967295, 0]]
    # ids pair up across lines (file order of ids)
    assert P(b"1\n2 3\n4\n") == [[1, 2], [3, 4]]
    for bad in (b"1 2 3\n", b"4294967296 1\n"):
        with pytest.raises(ParseError):
            parse_edge_list(bad)
