"""The no-allocation entry point (tc_process_batch_noalloc) against the
allocating one (tc_process_batch), through the C-ABI (needs an MI355X).

Every per-step buffer of tc_process_batch_noalloc lives in the library's
static device scratch; its results must equal tc_process_batch's bit for
bit: full estimator state (f1, f2, chi, closed) after every call, S exact.
Two calls in a row, the second with a smaller batch; two banks sharing the
scratch on one stream; the hashed directory; a batch too large for the
scratch refused on the host.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1308_2166_amd import inputs

pytestmark = pytest.mark.gpu


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


def np_edges(t):
    return t.cpu().numpy().view(np.uint32)


def to_dev(E):
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.uint32).view(np.int32)).cuda()


def same(a, b, where):
    for name, x, y in zip(("r1", "r2", "c", "closed"), a, b):
        if not np.array_equal(x, y):
            bad = np.nonzero(x != y)[0]
            raise AssertionError(f"{where}: {name} differs at {bad.size} estimators, "
                                 f"first {bad[:5].tolist()}")


@pytest.mark.parametrize("spread", [False, True])
def test_noalloc_equals_process_batch(tc, spread):
    # two calls in a row, the second smaller; dense (ids < 2^14) or hashed
    # (ids spread over 32 bits) directory
    E = np_edges(inputs.rmat(14, 90000, seed=21))
    if spread:
        E = ((E.astype(np.uint64) * 2654435761 + 99) % (2**32 - 5)).astype(np.uint32)
    r, seed = 30000, 77
    say(f"  noalloc vs process_batch r={r} spread={spread}")
    dev = to_dev(E)
    a, b = tc.Bank(r, seed), tc.Bank(r, seed)
    o = O.Bank(r, seed)
    for lo, hi in [(0, 60000), (60000, 67000), (67000, 90000)]:
        tc.tc_process_batch_noalloc(a.h, dev[lo:hi])
        tc.tc_process_batch(b.h, dev[lo:hi])
        assert o.process(E[lo:hi]) == O.OK
        sa = a.state()
        same(sa, b.state(), f"[{lo},{hi}) noalloc vs process_batch")
        same(sa, o.state(), f"[{lo},{hi}) noalloc vs oracle")
    assert tc.tc_estimate_ex(a.h)[:2] == tc.tc_estimate_ex(b.h)[:2]
    assert a.batch == b.batch == 3 and a.m == b.m == 90000


def test_noalloc_two_banks_share_the_scratch(tc):
    # banks of different sizes alternate on one stream, with shrinking and
    # growing batches, mixed with the allocating call on the same bank
    E0 = np_edges(inputs.rmat(13, 40000, seed=5))
    E1 = np_edges(inputs.gnm(3000, 40000, seed=6))
    d0, d1 = to_dev(E0), to_dev(E1)
    x0, x1 = tc.Bank(5000, 1), tc.Bank(20000, 2)
    y0, y1 = tc.Bank(5000, 1), tc.Bank(20000, 2)
    cuts = [0, 9000, 9100, 30000, 31000, 40000]
    for k in range(len(cuts) - 1):
        lo, hi = cuts[k], cuts[k + 1]
        f0 = tc.tc_process_batch if k == 2 else tc.tc_process_batch_noalloc
        f0(x0.h, d0[lo:hi])
        tc.tc_process_batch_noalloc(x1.h, d1[lo:hi])
        tc.tc_process_batch(y0.h, d0[lo:hi])
        tc.tc_process_batch(y1.h, d1[lo:hi])
        same(x0.state(), y0.state(), f"bank 0 batch {k}")
        same(x1.state(), y1.state(), f"bank 1 batch {k}")


def test_noalloc_largest_accepted_and_refused(tc):
    # w = 2^18 with r = 2^18 fits the static scratch; one more edge does not,
    # and is refused on the host with nothing enqueued
    E = np_edges(inputs.rmat(16, (1 << 18) + 1, seed=8))
    dev = to_dev(E)
    r = 1 << 18
    a, b = tc.Bank(r, 3), tc.Bank(r, 3)
    with pytest.raises(tc.TcError) as ei:
        tc.tc_process_batch_noalloc(a.h, dev)
    assert ei.value.code == tc.TC_EINVAL
    assert a.batch == 0 and a.m == 0
    tc.tc_process_batch_noalloc(a.h, dev[:1 << 18])
    tc.tc_process_batch(b.h, dev[:1 << 18])
    same(a.state(), b.state(), "w = r = 2^18")
    tc.tc_process_batch_noalloc(a.h, dev[:1000])
    tc.tc_process_batch(b.h, dev[:1000])
    same(a.state(), b.state(), "then w = 1000")
