"""CPU oracle for the bulk update of neighborhood-sampling estimators.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct reference
the GPU path is checked against (bit-exact estimator state).  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It shares no code with the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc by
``oracle.build.build()``); this module only marshals numpy arrays through
ctypes.  Paper: Tangwongsan, Pavan, Tirthapura, "Parallel Triangle Counting in
Massive Streaming Graphs" -- Sec. 3.1 (NBSI, Lemma 1) and Sec. 4 (bulkUpdateAll).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

EMPTY = (1 << 64) - 1
NONE32 = (1 << 32) - 1
OK, EINVAL, EBADEDGE, EOVERFLOW = 0, -1, -2, -3

DRAW_FN = ctypes.CFUNCTYPE(ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                           ctypes.c_uint32, ctypes.c_uint64)


class _State(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("m", ctypes.c_uint64),
        ("batch", ctypes.c_uint64),
        ("r1", ctypes.POINTER(ctypes.c_uint64)),
        ("r2", ctypes.POINTER(ctypes.c_uint64)),
        ("c", ctypes.POINTER(ctypes.c_uint32)),
        ("closed", ctypes.POINTER(ctypes.c_uint8)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        u32, u64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        P = ctypes.POINTER(_State)
        L.orc_mix64.argtypes, L.orc_mix64.restype = [u64], u64
        L.orc_raw.argtypes, L.orc_raw.restype = [u64, u64, u64, u64, u64], u64
        L.orc_lemire_step.argtypes = [u64, u64, ctypes.POINTER(ctypes.c_int)]
        L.orc_lemire_step.restype = u64
        L.orc_uniform.argtypes, L.orc_uniform.restype = [u64, u64, u64, u64, u64], u64
        L.orc_create.argtypes, L.orc_create.restype = [u32, u64], P
        L.orc_destroy.argtypes, L.orc_destroy.restype = [P], None
        for name in ("orc_batch_def", "orc_batch_bulk"):
            f = getattr(L, name)
            f.argtypes = [P, vp, u32, DRAW_FN, vp]
            f.restype = ctypes.c_int
        L.orc_sum.argtypes, L.orc_sum.restype = [P], u64
        L.orc_estimate.argtypes, L.orc_estimate.restype = [P], ctypes.c_double
        L.orc_mom.argtypes, L.orc_mom.restype = [P, u32, vp], ctypes.c_double
        L.orc_estimators_needed.argtypes = [ctypes.c_double, ctypes.c_double, u64, u64,
                                            ctypes.c_double]
        L.orc_estimators_needed.restype = u64
        L.orc_rank.argtypes, L.orc_rank.restype = [vp, u32, u32, u32], u32
        L.orc_rank_all.argtypes = [vp, u32, vp, vp, vp, vp]
        L.orc_rank_all.restype = None
        L.orc_phi_pos.argtypes, L.orc_phi_pos.restype = [vp, u32, u32, u32, u32], u32
        _lib = L
    return _lib


def _edges(W) -> np.ndarray:
    W = np.ascontiguousarray(np.asarray(W, dtype=np.uint32).reshape(-1, 2))
    return W


def mix64(z: int) -> int:
    return lib().orc_mix64(z)


def raw(seed, est, batch, purpose, attempt) -> int:
    return lib().orc_raw(seed, est, batch, purpose, attempt)


def lemire_step(x: int, n: int) -> tuple[int, bool]:
    rej = ctypes.c_int(0)
    v = lib().orc_lemire_step(x, n, ctypes.byref(rej))
    return v, bool(rej.value)


def uniform(seed, est, batch, purpose, n) -> int:
    return lib().orc_uniform(seed, est, batch, purpose, n)


class Bank:
    """r estimators (f1, f2, closed, chi) advanced batch by batch on the CPU."""

    def __init__(self, r: int, seed: int):
        self._p = lib().orc_create(r, seed)
        if not self._p:
            raise ValueError("orc_create failed (r must be > 0)")
        self.r = r

    def __del__(self):
        p = getattr(self, "_p", None)
        if p and lib is not None:  # (module globals may be gone at exit)
            lib().orc_destroy(p)
            self._p = None

    def process(self, W, variant: str = "bulk", draw=None) -> int:
        """Advance by one batch; returns the oracle's status code."""
        W = _edges(W)
        fn = DRAW_FN(draw) if draw is not None else DRAW_FN()
        f = lib().orc_batch_bulk if variant == "bulk" else lib().orc_batch_def
        return f(self._p, W.ctypes.data if W.size else None, W.shape[0], fn, None)

    @property
    def m(self) -> int:
        return self._p.contents.m

    @property
    def batch(self) -> int:
        return self._p.contents.batch

    def state(self):
        s = self._p.contents
        r = s.r
        r1 = np.ctypeslib.as_array(s.r1, shape=(r,)).copy()
        r2 = np.ctypeslib.as_array(s.r2, shape=(r,)).copy()
        c = np.ctypeslib.as_array(s.c, shape=(r,)).copy()
        closed = np.ctypeslib.as_array(s.closed, shape=(r,)).copy()
        return r1, r2, c, closed

    def sum(self) -> int:
        return lib().orc_sum(self._p)

    def estimate(self) -> float:
        return lib().orc_estimate(self._p)

    def mom(self, g: int):
        """(median-of-means estimate, exact group sums S_k)."""
        sums = np.zeros(max(g, 1), np.uint64)
        tau = lib().orc_mom(self._p, g, sums.ctypes.data)
        return tau, sums[:g]


def estimators_needed(eps: float, delta: float, m: int, maxdeg: int, tau: float) -> int:
    """Theorem 2's r for an (eps, delta)-approximation (0 if out of range)."""
    return lib().orc_estimators_needed(eps, delta, m, maxdeg, tau)


def rank(W, x: int, y: int) -> int:
    W = _edges(W)
    return lib().orc_rank(W.ctypes.data, W.shape[0], x, y)


def rank_all(W):
    W = _edges(W)
    n = 2 * W.shape[0]
    out = [np.zeros(n, dtype=np.uint32) for _ in range(4)]
    lib().orc_rank_all(W.ctypes.data, W.shape[0], *(a.ctypes.data for a in out))
    return tuple(out)  # src, dst, rank, pos (0-based)


def phi_pos(W, u: int, v: int, phi: int) -> int:
    W = _edges(W)
    return lib().orc_phi_pos(W.ctypes.data, W.shape[0], u, v, phi)


def run_stream(edges, r: int, seed: int, w: int, variant: str = "bulk"):
    """Feed `edges` (k x 2) in batches of w; returns the final Bank."""
    E = _edges(edges)
    b = Bank(r, seed)
    for j in range(0, E.shape[0], w):
        rc = b.process(E[j:j + w], variant)
        if rc != OK:
            raise RuntimeError(f"oracle batch failed with {rc}")
    return b
