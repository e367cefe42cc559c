"""Seeded synthetic edge streams (shared by the tests and the benchmark).

Every generator is a pure function of its arguments and seed: the same call
gives bit-identical edges on the CPU and on a GPU, because it uses only
integer tensor arithmetic (wrapping int64), exact int->float conversions,
sorting and searchsorted.  The module contains no part of the estimator
arithmetic; it only makes inputs.

Edge streams are ``int64``-free ``torch.uint32``-compatible ``(m, 2)`` int32
views of uint32 pairs; helpers return ``torch.int32`` tensors holding the
uint32 bit pattern (vertex ids are below 2^31 for every shape used here) so
they can be handed to the GPU library as ``uint32[2w]`` buffers.

Shapes follow the paper's workloads (Sec. 5, Table 1): simple undirected
graphs, each edge once, stream order random, heavy-tailed degrees.  The
paper's SNAP/Friendster graphs are not available, so R-MAT and Chung-Lu
power-law graphs of the same density stand in for them.
"""
from __future__ import annotations

import math

import torch

_M64 = (1 << 64) - 1


def _s64(x: int) -> int:
    """uint64 constant -> the int64 with the same bit pattern."""
    x &= _M64
    return x - (1 << 64) if x >> 63 else x


_C1 = _s64(0xFF51AFD7ED558CCD)  # murmur3 fmix64 constants
_C2 = _s64(0xC4CEB9FE1A85EC53)
_STEP = _s64(0xD1B54A32D192ED03)


def _lsr(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor (bit pattern as uint64)."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def hash64(x: torch.Tensor) -> torch.Tensor:
    """murmur3's fmix64 finalizer, a bijection on 64-bit words."""
    x = x ^ _lsr(x, 33)
    x = x * _C1
    x = x ^ _lsr(x, 33)
    x = x * _C2
    x = x ^ _lsr(x, 33)
    return x


def hash64_int(x: int) -> int:
    """Python-int twin of hash64 (for tests of the generator itself)."""
    x &= _M64
    x ^= x >> 33
    x = (x * 0xFF51AFD7ED558CCD) & _M64
    x ^= x >> 33
    x = (x * 0xC4CEB9FE1A85EC53) & _M64
    x ^= x >> 33
    return x


def _stream(seed: int, tag: int, start: int, n: int, device) -> torch.Tensor:
    """n pseudo-random 64-bit words for counters start..start+n-1."""
    key = hash64_int((seed * 0x9E3779B97F4A7C15 + tag) & _M64)
    ctr = torch.arange(start, start + n, dtype=torch.int64, device=device)
    return hash64(ctr * _STEP + _s64(key))


def _below(h32: torch.Tensor, n: int) -> torch.Tensor:
    """Map 32 random bits to [0, n) by multiply-shift (n < 2^31)."""
    return (h32 * n) >> 32


def _dedup_keys(keys: torch.Tensor) -> torch.Tensor:
    return torch.unique(keys, sorted=True)


def _take_shuffled(keys: torch.Tensor, m: int, seed: int) -> torch.Tensor:
    """A seeded uniform-looking order of the distinct keys, first m kept."""
    pri = hash64(keys ^ _s64(hash64_int(seed ^ 0x5EED)))
    order = torch.argsort(pri, stable=True)
    return keys[order[:m]]


def _orient(keys: torch.Tensor, seed: int) -> torch.Tensor:
    """(m,) canonical keys -> (m,2) int32 pairs with seeded orientation."""
    lo = _lsr(keys, 32)
    hi = keys & 0xFFFFFFFF
    flip = (hash64(keys ^ _s64(hash64_int(seed ^ 0x0F1E))) & 1).bool()
    a = torch.where(flip, hi, lo)
    b = torch.where(flip, lo, hi)
    return torch.stack([a, b], dim=1).to(torch.int32)


def _collect(sample, m: int, seed: int, device, max_rounds: int = 64):
    """Draw candidate canonical keys in rounds until m distinct ones exist."""
    have = torch.empty(0, dtype=torch.int64, device=device)
    ctr = 0
    for _ in range(max_rounds):
        need = m - have.numel()
        if need <= 0:
            break
        k = int(need * 1.35) + 4096
        cand = sample(ctr, k)
        ctr += k
        have = _dedup_keys(torch.cat([have, cand]))
    if have.numel() < m:
        raise ValueError("graph too dense for the requested number of edges")
    return _take_shuffled(have, m, seed)


def _canon_keys(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    keep = a != b
    a, b = a[keep], b[keep]
    lo = torch.minimum(a, b)
    hi = torch.maximum(a, b)
    return (lo << 32) | hi


def gnm(n: int, m: int, seed: int, device="cpu") -> torch.Tensor:
    """Uniform simple graph G(n, m) as a random-order stream of m edges."""
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of vertex pairs")

    def sample(start, k):
        h = _stream(seed, 1, start, k, device)
        a = _below(_lsr(h, 32), n)
        b = _below(h & 0xFFFFFFFF, n)
        return _canon_keys(a, b)

    return _orient(_collect(sample, m, seed, device), seed)


def _scale_bijection(x: torch.Tensor, scale: int, seed: int) -> torch.Tensor:
    """A seeded permutation of [0, 2^scale) (odd multiply, xorshift, add)."""
    mask = (1 << scale) - 1
    k = hash64_int(seed ^ 0xB1EC)
    mul1 = (k | 1) & mask
    mul2 = ((k >> 20) | 1) & mask
    add = (k >> 40) & mask
    sh = max(1, scale // 2)
    x = (x * mul1) & mask
    x = x ^ (x >> sh)
    x = (x * mul2 + add) & mask
    x = x ^ (x >> sh)
    return x


def rmat(scale: int, m: int, seed: int, abcd=(0.57, 0.19, 0.19, 0.05),
         device="cpu", permute: bool = True) -> torch.Tensor:
    """R-MAT graph (recursive quadrant descent, no noise) with exactly m
    distinct loop-free edges, vertex ids permuted by a seeded bijection of
    [0, 2^scale), in a seeded random stream order."""
    if scale > 30:
        raise ValueError("scale must be <= 30")
    a, b, c, _ = abcd
    # 32-bit fixed-point cumulative thresholds for the four quadrants
    ta = int(round(a * 2**32))
    tb = int(round((a + b) * 2**32))
    tc = int(round((a + b + c) * 2**32))

    def sample(start, k):
        src = torch.zeros(k, dtype=torch.int64, device=device)
        dst = torch.zeros(k, dtype=torch.int64, device=device)
        for lvl in range(0, scale, 2):
            h = _stream(seed, 100 + lvl, start, k, device)
            for half in range(2):
                if lvl + half >= scale:
                    break
                u = _lsr(h, 32) if half == 0 else (h & 0xFFFFFFFF)
                sbit = (u >= tb).to(torch.int64)
                dbit = (((u >= ta) & (u < tb)) | (u >= tc)).to(torch.int64)
                src = (src << 1) | sbit
                dst = (dst << 1) | dbit
        if permute:
            src = _scale_bijection(src, scale, seed)
            dst = _scale_bijection(dst, scale, seed)
        return _canon_keys(src, dst)

    return _orient(_collect(sample, m, seed, device), seed)


def chung_lu(n: int, m: int, seed: int, gamma: float = 2.1,
             device="cpu") -> torch.Tensor:
    """Chung-Lu power-law graph: endpoints drawn independently with weight
    proportional to (i+1)^(-1/(gamma-1)); exactly m distinct edges."""
    wts = torch.arange(1, n + 1, dtype=torch.float64) ** (-1.0 / (gamma - 1.0))
    cdf = torch.cumsum(wts, 0)
    cdf = (cdf / cdf[-1]).to(device)  # computed on the CPU: same bits everywhere
    perm = torch.argsort(_stream(seed, 7, 0, n, "cpu"), stable=True).to(device)

    def pick(h):
        u = _lsr(h, 11).to(torch.float64) * (1.0 / 2**53)
        idx = torch.searchsorted(cdf, u, right=True).clamp_(max=n - 1)
        return perm[idx]

    def sample(start, k):
        a = pick(_stream(seed, 8, start, k, device))
        b = pick(_stream(seed, 9, start, k, device))
        return _canon_keys(a, b)

    return _orient(_collect(sample, m, seed, device), seed)


def batches(edges: torch.Tensor, w: int):
    """Split a stream into consecutive batches of w edges (last one ragged)."""
    for j in range(0, edges.shape[0], w):
        yield edges[j:j + w]


# --- named workloads (the paper's shapes at GPU scale) -----------------------

def workload(name: str, device="cpu"):
    """Return (edges, r, w, seed) for a named workload."""
    if name == "gnm-2k":  # G(n=2000, m=20000), r=4096, w=2048
        return gnm(2000, 20000, seed=1, device=device), 4096, 2048, 3
    if name == "rmat20":  # R-MAT scale 20, m=16*2^20, r=2^20, w=2^22
        return rmat(20, 16 << 20, seed=20, device=device), 1 << 20, 1 << 22, 5
    if name == "rmat24":  # R-MAT scale 24, m=2^28, r=2^22, w=2^24
        return rmat(24, 1 << 28, seed=24, device=device), 1 << 22, 1 << 24, 7
    raise KeyError(name)


def vertex_count(name: str) -> int:
    """Vertex ids of a named workload lie in [0, vertex_count)."""
    return {"gnm-2k": 2000, "rmat20": 1 << 20, "rmat24": 1 << 24}[name]


def lognormal_sizes(k: int, seed: int, median: float = 3e5, sigma: float = 1.2,
                    lo: float = 1e4, hi: float = 1e7):
    """k stream lengths, ln m ~ N(ln median, sigma^2), clipped to [lo, hi]."""
    h = _stream(seed, 11, 0, 2 * k, "cpu")
    u1 = (_lsr(h[:k], 11).to(torch.float64) + 0.5) * (1.0 / 2**53)
    u2 = _lsr(h[k:], 11).to(torch.float64) * (1.0 / 2**53)
    z = torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)
    return [int(v) for v in torch.clamp(torch.exp(math.log(median) + sigma * z),
                                        lo, hi).round().tolist()]


def _uniform_ints(seed: int, tag: int, k: int, lo: int, hi: int):
    """k seeded integers uniform on [lo, hi]."""
    h = _stream(seed, tag, 0, k, "cpu")
    return [lo + int(v) for v in _below(_lsr(h, 32), hi - lo + 1).tolist()]


def many_streams(nstreams: int = 256, seed: int = 404, device="cpu",
                 size_scale: float = 1.0):
    """Independent streams of uneven length for the batched form.

    Stream lengths are lognormal (median 3e5, sigma 1.2, clipped to
    [1e4, 1e7]; `size_scale` shrinks them for tests).  Each entry also
    gives n, a bound on its vertex ids.  Even-indexed streams
    are R-MAT with scale ~ U{16..22} (raised until m/n <= 16), odd-indexed
    ones Chung-Lu with n = m/8 and degree exponent 2.1.  Each stream has its
    own bank of r = 2^U{14..18} estimators and its own seed.
    """
    sizes = lognormal_sizes(nstreams, seed)
    scales = _uniform_ints(seed, 12, nstreams, 16, 22)
    rlog = _uniform_ints(seed, 13, nstreams, 14, 18)
    out = []
    for s in range(nstreams):
        m = max(64, int(sizes[s] * size_scale))
        gseed = hash64_int(seed * 1000003 + s) & 0x7FFFFFFF
        if s % 2 == 0:
            sc = scales[s]
            while m > 16 * (1 << sc):
                sc += 1
            e = rmat(sc, m, seed=gseed, device=device)
            kind = f"rmat{sc}"
            nv = 1 << sc
        else:
            n = max(64, m // 8)
            e = chung_lu(n, m, seed=gseed, device=device)
            kind = f"chunglu{n}"
            nv = n
        r = 1 << rlog[s]
        if size_scale < 1.0:
            r = max(16, int(r * size_scale))
        out.append({"edges": e, "r": r, "seed": gseed ^ 0x5A5A, "kind": kind, "n": nv})
    return out


def edge_list_text(edges: torch.Tensor, sep: str = "\t", header: str = "") -> torch.Tensor:
    """A stream as a text edge list ("a<sep>b\\n" per edge, variable-width
    decimal ids, optional comment header) in a uint8 tensor on the edges'
    device: the input form of the text parser."""
    dev = edges.device
    e = edges.to(torch.int64) & 0xFFFFFFFF
    m = e.shape[0]
    if m == 0:
        return torch.tensor(list(header.encode()), dtype=torch.uint8, device=dev)
    pw = torch.tensor([10 ** k for k in range(11)], dtype=torch.int64, device=dev)

    def ndig(v):
        return (v.unsqueeze(1) >= pw[1:].unsqueeze(0)).sum(1) + 1

    na, nb = ndig(e[:, 0]), ndig(e[:, 1])
    s = sep.encode()
    length = na + nb + len(s) + 1
    hb = header.encode()
    off = torch.cumsum(length, 0) - length + len(hb)
    out = torch.empty(int(length.sum()) + len(hb), dtype=torch.uint8, device=dev)
    if hb:
        out[:len(hb)] = torch.tensor(list(hb), dtype=torch.uint8, device=dev)

    def put(v, nd, base):
        for k in range(10):
            live = nd > k
            d = (v // pw[(nd - 1 - k).clamp(min=0)]) % 10
            out[(base + k)[live]] = (48 + d[live]).to(torch.uint8)

    put(e[:, 0], na, off)
    for i, ch in enumerate(s):
        out[off + na + i] = ch
    put(e[:, 1], nb, off + na + len(s))
    out[off + length - 1] = 10
    return out
