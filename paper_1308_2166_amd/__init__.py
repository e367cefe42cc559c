"""Python binding of libtc: the bulk update of neighborhood-sampling triangle
estimators on MI355X (gfx950).

Argument marshalling only.  Every step of the update runs in the HIP kernels
of ``libtc.so``; there is no CPU fallback, and using the binding without the
built library raises.  Function names match the C-ABI in ``include/tc.h``.
Device buffers are torch tensors (torch supplies device memory and streams).

Paper: Tangwongsan, Pavan, Tirthapura, "Parallel Triangle Counting in
Massive Streaming Graphs", Sec. 4 (bulkUpdateAll).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch  # loaded first: libtc must bind to the HIP runtime torch uses

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK, TC_EINVAL, TC_EBADEDGE, TC_EOVERFLOW, TC_ENOMEM, TC_EHIP = 0, -1, -2, -3, -4, -5
TC_EMPTY_EDGE = (1 << 64) - 1
TC_MAX_BATCH = 1 << 28
TC_TIME_ALL = 0xFFFFFFFF

_NAMES = {TC_EINVAL: "TC_EINVAL", TC_EBADEDGE: "TC_EBADEDGE",
          TC_EOVERFLOW: "TC_EOVERFLOW", TC_ENOMEM: "TC_ENOMEM", TC_EHIP: "TC_EHIP"}


class TcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class TcTuning(ctypes.Structure):
    """tc_tuning: launch shapes that do not change results."""
    _fields_ = [("digit_bits", ctypes.c_uint32), ("chunk_tiles", ctypes.c_uint32),
                ("part_estimators", ctypes.c_uint32), ("join_edges", ctypes.c_uint32),
                ("fused_edges", ctypes.c_uint32)]


TUNING_FIELDS = tuple(f for f, _ in TcTuning._fields_)
DEFAULT_TUNING = {"digit_bits": 0, "chunk_tiles": 32, "part_estimators": 2048,
                  "join_edges": 8192, "fused_edges": 2048}

_lib = None


def lib():
    """The loaded libtc (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    maps = open("/proc/self/maps").read()
    hips = set(re.findall(r"\S*libamdhip64\S*", maps))
    if len(hips) > 1:
        raise ImportError(f"two HIP runtimes are mapped: {sorted(hips)}")
    u32, u64, i32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
    P64, P32, P8 = (ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                    ctypes.POINTER(ctypes.c_uint8))
    sig = {
        "tc_create": ([u32, u64], vp),
        "tc_process_batch": ([vp, vp, u32, vp], i32),
        "tc_process_stream": ([vp, vp, u64, u32, vp], i32),
        "tc_process_host_stream": ([vp, vp, u64, u32, vp], i32),
        "tc_bank_bytes": ([u32], u64),
        "tc_set_tuning": ([vp, ctypes.POINTER(TcTuning)], i32),
        "tc_get_tuning": ([vp, ctypes.POINTER(TcTuning)], i32),
        "tc_multi_set_tuning": ([vp, ctypes.POINTER(TcTuning)], i32),
        "tc_multi_get_tuning": ([vp, ctypes.POINTER(TcTuning)], i32),
        "tc_step_bytes_max": ([u32, u32, u64], u64),
        "tc_multi_reserve_max": ([vp, u32, u64], i32),
        "tc_step_bytes": ([u32, vp, vp], u64),
        "tc_device_bytes": ([vp, P64], i32),
        "tc_multi_device_bytes": ([vp, P64], i32),
        "tc_process_batch_naive": ([vp, vp, u32, vp], i32),
        "tc_process_batch_noalloc": ([vp, vp, u32, vp], i32),
        "tc_parse_edges": ([vp, u64, vp, u64, P64, vp], i32),
        "tc_probe_line_rate": ([vp, u64, u32, u32, u32, u32, vp,
                                ctypes.POINTER(ctypes.c_double), vp], i32),
        "tc_set_vertex_bound": ([vp, u64], i32),
        "tc_estimate_mom": ([vp, u32, ctypes.POINTER(ctypes.c_double), P64], i32),
        "tc_multi_estimate_mom": ([vp, u32, u32, ctypes.POINTER(ctypes.c_double), P64], i32),
        "tc_estimators_needed": ([ctypes.c_double, ctypes.c_double, u64, u64, ctypes.c_double],
                                 u64),
        "tc_multi_set_vertex_bound": ([vp, u64], i32),
        "tc_estimate": ([vp], ctypes.c_double),
        "tc_estimate_ex": ([vp, P64, P64, ctypes.POINTER(ctypes.c_double)], i32),
        "tc_read_state": ([vp, vp, vp, vp, vp], i32),
        "tc_sync": ([vp], i32),
        "tc_num_estimators": ([vp], u32),
        "tc_edges_seen": ([vp], u64),
        "tc_batches_seen": ([vp], u64),
        "tc_destroy": ([vp], None),
        "tc_last_error": ([], ctypes.c_char_p),
        "tc_multi_create": ([u32, vp, vp], vp),
        "tc_multi_process": ([vp, u32, vp, vp, vp, vp], i32),
        "tc_multi_estimate": ([vp, vp, vp, vp], i32),
        "tc_multi_read_state": ([vp, u32, vp, vp, vp, vp], i32),
        "tc_multi_sync": ([vp], i32),
        "tc_multi_num_banks": ([vp], u32),
        "tc_multi_destroy": ([vp], None),
        "tc_reserve": ([vp, u32], i32),
        "tc_reset": ([vp, vp], i32),
        "tc_multi_reset": ([vp, vp], i32),
        "tc_multi_graph_reserve": ([vp, u32], i32),
        "tc_multi_assign": ([vp, u32, u64, vp], i32),
        "tc_multi_reserve": ([vp, u32, vp, vp], i32),
        "tc_set_kernel_timing": ([vp, u32], i32),
        "tc_kernel_times": ([vp, vp, P64], i32),
        "tc_multi_set_kernel_timing": ([vp, u32], i32),
        "tc_multi_kernel_times": ([vp, vp, P64], i32),
        "tc_num_kernels": ([], i32),
        "tc_kernel_name": ([i32], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes, f.restype = args, res
    _lib = L
    return L


EXPORTS = ("tc_create", "tc_process_batch", "tc_process_stream", "tc_estimate", "tc_estimate_ex",
           "tc_read_state", "tc_sync", "tc_num_estimators", "tc_edges_seen",
           "tc_batches_seen", "tc_destroy", "tc_last_error", "tc_multi_create",
           "tc_multi_process", "tc_multi_estimate", "tc_multi_read_state",
           "tc_multi_sync", "tc_multi_num_banks", "tc_multi_destroy",
           "tc_set_kernel_timing", "tc_kernel_times", "tc_multi_set_kernel_timing",
           "tc_multi_kernel_times", "tc_num_kernels", "tc_kernel_name",
           "tc_reserve", "tc_multi_reserve", "tc_reset", "tc_multi_reset",
           "tc_multi_graph_reserve", "tc_multi_assign", "tc_set_vertex_bound",
           "tc_multi_set_vertex_bound", "tc_estimate_mom", "tc_multi_estimate_mom",
           "tc_estimators_needed", "tc_process_batch_naive", "tc_parse_edges",
           "tc_probe_line_rate",
           "tc_process_batch_noalloc", "tc_process_host_stream", "tc_bank_bytes",
           "tc_step_bytes", "tc_device_bytes", "tc_multi_device_bytes",
           "tc_step_bytes_max", "tc_multi_reserve_max", "tc_set_tuning", "tc_get_tuning",
           "tc_multi_set_tuning", "tc_multi_get_tuning")


def _check(rc: int):
    if rc != TC_OK:
        raise TcError(rc, tc_last_error())


def _stream_handle(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _edge_ptr(edges) -> tuple[int, int]:
    """(device address, w) of an (w, 2) int32/uint32 CUDA tensor."""
    if not isinstance(edges, torch.Tensor) or not edges.is_cuda:
        raise TypeError("edges must be a CUDA tensor of shape (w, 2)")
    if edges.dtype not in (torch.int32, torch.uint32) or edges.dim() != 2 \
            or edges.shape[1] != 2 or not edges.is_contiguous():
        raise TypeError("edges must be a contiguous (w, 2) int32/uint32 tensor")
    return edges.data_ptr(), edges.shape[0]


# ---- C-ABI, same names ------------------------------------------------------

def tc_last_error() -> str:
    return lib().tc_last_error().decode()


def tc_create(r: int, seed: int) -> int:
    h = lib().tc_create(r, seed & ((1 << 64) - 1))
    if not h:
        raise TcError(TC_EINVAL, tc_last_error())
    return h


def _batch_args(edges, w):
    """(device address or None, w) of a batch; w defaults to the tensor's
    rows and may not exceed them (the kernels would read past its end)."""
    if edges is not None and w is not None and hasattr(edges, "shape") \
            and len(edges.shape) >= 1 and w > edges.shape[0]:
        raise ValueError(f"w = {w} exceeds the {edges.shape[0]} edges of the tensor")
    ptr, n = _edge_ptr(edges) if edges is not None else (0, 0)
    return ptr or None, n if w is None else w


def tc_process_batch(state: int, edges, w: int | None = None, stream=None) -> None:
    ptr, w = _batch_args(edges, w)
    _check(lib().tc_process_batch(state, ptr, w, _stream_handle(stream)))


def tc_process_batch_noalloc(state: int, edges, w: int | None = None, stream=None) -> None:
    ptr, w = _batch_args(edges, w)
    _check(lib().tc_process_batch_noalloc(state, ptr, w, _stream_handle(stream)))


def tc_process_batch_naive(state: int, edges, w: int | None = None, stream=None) -> None:
    ptr, w = _batch_args(edges, w)
    _check(lib().tc_process_batch_naive(state, ptr, w, _stream_handle(stream)))


def tc_parse_edges(text: torch.Tensor, max_edges: int | None = None, stream=None):
    """Parse a text edge list held in a uint8 CUDA tensor; returns an
    (m, 2) int32 CUDA tensor of the edges (uint32 ids as bit patterns)."""
    if not isinstance(text, torch.Tensor) or not text.is_cuda or text.dtype != torch.uint8:
        raise TypeError("text must be a uint8 CUDA tensor")
    n = text.numel()
    if max_edges is None:
        max_edges = n // 4 + 1  # an edge takes at least four bytes ("1 2\n")
    out = torch.empty((max(max_edges, 1), 2), dtype=torch.int32, device=text.device)
    cnt = ctypes.c_uint64()
    _check(lib().tc_parse_edges(text.data_ptr() if n else None, n, out.data_ptr(), max_edges,
                                ctypes.byref(cnt), _stream_handle(stream)))
    return out[:cnt.value]


def tc_probe_line_rate(table: torch.Tensor, n: int, per_thread: int = 1,
                       dependent: bool = False, reps: int = 10, stream=None) -> float:
    """Random 128-byte line reads per second from `table` (a CUDA tensor
    whose byte size is a multiple of 128): a diagnostic of the device, not
    part of the method."""
    if not isinstance(table, torch.Tensor) or not table.is_cuda or not table.is_contiguous():
        raise TypeError("table must be a contiguous CUDA tensor")
    nbytes = table.numel() * table.element_size()
    sink = torch.empty(max(n, 1), dtype=torch.int32, device=table.device)
    rate = ctypes.c_double()
    _check(lib().tc_probe_line_rate(table.data_ptr(), nbytes, n, per_thread, int(dependent),
                                    reps, sink.data_ptr(), ctypes.byref(rate),
                                    _stream_handle(stream)))
    return rate.value


def tc_process_stream(state: int, edges, w: int, stream=None) -> None:
    """All of `edges` ((m, 2) device tensor) as consecutive batches of w."""
    if edges is None or edges.shape[0] == 0:
        ptr, m = 0, 0
    else:
        ptr, m = _edge_ptr(edges)
    _check(lib().tc_process_stream(state, ptr or None, m, w, _stream_handle(stream)))


def tc_process_host_stream(state: int, host_edges, w: int, stream=None) -> None:
    """All of `host_edges` (an (m, 2) int32/uint32 CPU tensor, ideally
    pinned, or a numpy array) as consecutive batches of w, copied to the
    device by the library.  The array must stay alive until `stream` has
    passed this work."""
    if isinstance(host_edges, torch.Tensor):
        if host_edges.is_cuda:
            raise TypeError("host_edges must be in host memory (use tc_process_stream)")
        if host_edges.dtype not in (torch.int32, torch.uint32) or host_edges.dim() != 2 \
                or host_edges.shape[1] != 2 or not host_edges.is_contiguous():
            raise TypeError("host_edges must be a contiguous (m, 2) int32/uint32 tensor")
        ptr, m = host_edges.data_ptr(), host_edges.shape[0]
    else:
        a = np.asarray(host_edges)
        if a.dtype not in (np.int32, np.uint32) or a.ndim != 2 or a.shape[1] != 2 \
                or not a.flags.c_contiguous:
            raise TypeError("host_edges must be a C-contiguous (m, 2) int32/uint32 array")
        ptr, m = a.ctypes.data, a.shape[0]
    _check(lib().tc_process_host_stream(state, (ptr if m else None), m, w,
                                        _stream_handle(stream)))


def _tuning(t: dict) -> TcTuning:
    unknown = set(t) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    full = dict(DEFAULT_TUNING)
    full.update(t)
    return TcTuning(*(int(full[f]) for f in TUNING_FIELDS))


def tc_set_tuning(state: int, tuning: dict) -> None:
    """Set launch shapes (fields of tc_tuning; missing ones take defaults)."""
    _check(lib().tc_set_tuning(state, ctypes.byref(_tuning(tuning))))


def tc_get_tuning(state: int) -> dict:
    t = TcTuning()
    _check(lib().tc_get_tuning(state, ctypes.byref(t)))
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def tc_multi_set_tuning(multi: int, tuning: dict) -> None:
    _check(lib().tc_multi_set_tuning(multi, ctypes.byref(_tuning(tuning))))


def tc_multi_get_tuning(multi: int) -> dict:
    t = TcTuning()
    _check(lib().tc_multi_get_tuning(multi, ctypes.byref(t)))
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def tc_bank_bytes(r: int) -> int:
    return lib().tc_bank_bytes(r)


def tc_step_bytes(rs, ws) -> int:
    r = np.ascontiguousarray(rs, dtype=np.uint32)
    w = np.ascontiguousarray(ws, dtype=np.uint32)
    if r.shape != w.shape:
        raise ValueError("one r and one w per chunk")
    return lib().tc_step_bytes(len(r), r.ctypes.data, w.ctypes.data)


def tc_step_bytes_max(nchunks: int, r_max: int, total_w: int) -> int:
    return lib().tc_step_bytes_max(nchunks, r_max, total_w)


def tc_multi_reserve_max(multi: int, nchunks: int, total_w: int) -> None:
    _check(lib().tc_multi_reserve_max(multi, nchunks, total_w))


def tc_device_bytes(state: int) -> int:
    b = ctypes.c_uint64()
    _check(lib().tc_device_bytes(state, ctypes.byref(b)))
    return b.value


def tc_multi_device_bytes(multi: int) -> int:
    b = ctypes.c_uint64()
    _check(lib().tc_multi_device_bytes(multi, ctypes.byref(b)))
    return b.value


def tc_estimate_mom(state: int, groups: int):
    """(median-of-means estimate, group sums S_k as a uint64 array)."""
    tau = ctypes.c_double()
    sums = np.zeros(max(groups, 1), np.uint64)
    _check(lib().tc_estimate_mom(state, groups, ctypes.byref(tau),
                                 sums.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return tau.value, sums[:groups]


def tc_multi_estimate_mom(multi: int, bank: int, groups: int):
    tau = ctypes.c_double()
    sums = np.zeros(max(groups, 1), np.uint64)
    _check(lib().tc_multi_estimate_mom(multi, bank, groups, ctypes.byref(tau),
                                       sums.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return tau.value, sums[:groups]


def tc_estimators_needed(eps: float, delta: float, m: int, maxdeg: int, tau: float) -> int:
    return lib().tc_estimators_needed(eps, delta, m, maxdeg, tau)


def tc_set_vertex_bound(state: int, n: int) -> None:
    _check(lib().tc_set_vertex_bound(state, n))


def tc_multi_set_vertex_bound(multi: int, n: int) -> None:
    _check(lib().tc_multi_set_vertex_bound(multi, n))


def tc_reserve(state: int, max_w: int) -> None:
    _check(lib().tc_reserve(state, max_w))


def tc_reset(state: int, stream=None) -> None:
    _check(lib().tc_reset(state, _stream_handle(stream)))


def tc_estimate(state: int) -> float:
    return lib().tc_estimate(state)


def tc_estimate_ex(state: int) -> tuple[int, int, float]:
    S, m, tau = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
    _check(lib().tc_estimate_ex(state, ctypes.byref(S), ctypes.byref(m), ctypes.byref(tau)))
    return S.value, m.value, tau.value


def tc_read_state(state: int):
    r = lib().tc_num_estimators(state)
    r1 = np.empty(r, np.uint64)
    r2 = np.empty(r, np.uint64)
    c = np.empty(r, np.uint32)
    closed = np.empty(r, np.uint8)
    _check(lib().tc_read_state(state, r1.ctypes.data, r2.ctypes.data,
                               c.ctypes.data, closed.ctypes.data))
    return r1, r2, c, closed


def tc_sync(state: int) -> None:
    _check(lib().tc_sync(state))


def tc_destroy(state: int) -> None:
    lib().tc_destroy(state)


def tc_num_estimators(state: int) -> int:
    return lib().tc_num_estimators(state)


def tc_edges_seen(state: int) -> int:
    return lib().tc_edges_seen(state)


def tc_batches_seen(state: int) -> int:
    return lib().tc_batches_seen(state)


def tc_multi_num_banks(multi: int) -> int:
    return lib().tc_multi_num_banks(multi)


def tc_num_kernels() -> int:
    return lib().tc_num_kernels()


def tc_kernel_name(k: int) -> str:
    return lib().tc_kernel_name(k).decode()


def _mask(enable) -> int:
    """True -> every kernel, False -> off, an int -> that kernel mask,
    a collection of kernel names -> their bits."""
    if isinstance(enable, bool):
        return TC_TIME_ALL if enable else 0
    if isinstance(enable, int):
        return enable & TC_TIME_ALL
    names = [tc_kernel_name(k) for k in range(tc_num_kernels())]
    return sum(1 << names.index(n) for n in enable)


def tc_set_kernel_timing(state: int, enable) -> None:
    _check(lib().tc_set_kernel_timing(state, _mask(enable)))


def tc_kernel_times(state: int):
    """({kernel name: total ms}, timed steps)."""
    n = tc_num_kernels()
    ms = np.zeros(n, np.float64)
    steps = ctypes.c_uint64()
    _check(lib().tc_kernel_times(state, ms.ctypes.data, ctypes.byref(steps)))
    return {tc_kernel_name(k): float(ms[k]) for k in range(n)}, steps.value


def tc_multi_set_kernel_timing(multi: int, enable) -> None:
    _check(lib().tc_multi_set_kernel_timing(multi, _mask(enable)))


def tc_multi_kernel_times(multi: int):
    n = tc_num_kernels()
    ms = np.zeros(n, np.float64)
    steps = ctypes.c_uint64()
    _check(lib().tc_multi_kernel_times(multi, ms.ctypes.data, ctypes.byref(steps)))
    return {tc_kernel_name(k): float(ms[k]) for k in range(n)}, steps.value


def tc_multi_create(r, seeds) -> int:
    r = np.ascontiguousarray(r, dtype=np.uint32)
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    h = lib().tc_multi_create(len(r), r.ctypes.data, seeds.ctypes.data)
    if not h:
        raise TcError(TC_EINVAL, tc_last_error())
    return h


def tc_multi_process(multi: int, bank_ids, edges_list, stream=None) -> None:
    """One step: chunk k = (bank_ids[k], edges_list[k]) for every k."""
    n = len(bank_ids)
    ids = np.ascontiguousarray(bank_ids, dtype=np.uint32)
    ptrs = np.zeros(n, dtype=np.uint64)
    ws = np.zeros(n, dtype=np.uint32)
    for k, e in enumerate(edges_list):
        if e is None or e.shape[0] == 0:
            continue
        ptrs[k], ws[k] = _edge_ptr(e)
    _check(lib().tc_multi_process(multi, n, ids.ctypes.data, ptrs.ctypes.data,
                                  ws.ctypes.data, _stream_handle(stream)))


def tc_multi_reserve(multi: int, bank_ids, ws) -> None:
    ids = np.ascontiguousarray(bank_ids, dtype=np.uint32)
    w = np.ascontiguousarray(ws, dtype=np.uint32)
    _check(lib().tc_multi_reserve(multi, len(ids), ids.ctypes.data, w.ctypes.data))


def tc_multi_reset(multi: int, stream=None) -> None:
    _check(lib().tc_multi_reset(multi, _stream_handle(stream)))


def tc_multi_assign(multi: int, bank: int, seed: int, stream=None) -> None:
    _check(lib().tc_multi_assign(multi, bank, seed & ((1 << 64) - 1), _stream_handle(stream)))


def tc_multi_graph_reserve(multi: int, nsteps: int) -> None:
    _check(lib().tc_multi_graph_reserve(multi, nsteps))


def tc_multi_estimate(multi: int):
    nb = lib().tc_multi_num_banks(multi)
    S = np.zeros(nb, np.uint64)
    m = np.zeros(nb, np.uint64)
    tau = np.zeros(nb, np.float64)
    _check(lib().tc_multi_estimate(multi, S.ctypes.data, m.ctypes.data, tau.ctypes.data))
    return S, m, tau


def tc_multi_read_state(multi: int, bank: int, r: int):
    r1 = np.empty(r, np.uint64)
    r2 = np.empty(r, np.uint64)
    c = np.empty(r, np.uint32)
    closed = np.empty(r, np.uint8)
    _check(lib().tc_multi_read_state(multi, bank, r1.ctypes.data, r2.ctypes.data,
                                     c.ctypes.data, closed.ctypes.data))
    return r1, r2, c, closed


def tc_multi_sync(multi: int) -> None:
    _check(lib().tc_multi_sync(multi))


def tc_multi_destroy(multi: int) -> None:
    lib().tc_multi_destroy(multi)


# ---- small owning wrappers ------------------------------------------------------

class Bank:
    """One bank of r estimators on the current GPU (owns a tc_state)."""

    def __init__(self, r: int, seed: int):
        self.r = r
        self.h = tc_create(r, seed)

    def process(self, edges, stream=None):
        tc_process_batch(self.h, edges, stream=stream)

    def process_naive(self, edges, stream=None):
        tc_process_batch_naive(self.h, edges, stream=stream)

    def process_stream(self, edges, w: int, stream=None):
        tc_process_stream(self.h, edges, w, stream=stream)

    def process_host_stream(self, host_edges, w: int, stream=None):
        tc_process_host_stream(self.h, host_edges, w, stream=stream)

    def estimate(self) -> float:
        return tc_estimate_ex(self.h)[2]

    def sum(self) -> int:
        return tc_estimate_ex(self.h)[0]

    def state(self):
        return tc_read_state(self.h)

    def sync(self):
        tc_sync(self.h)

    @property
    def m(self) -> int:
        return lib().tc_edges_seen(self.h)

    @property
    def batch(self) -> int:
        return lib().tc_batches_seen(self.h)

    def close(self):
        if self.h:
            tc_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiBank:
    """Many independent banks advanced together (owns a tc_multi)."""

    def __init__(self, rs, seeds):
        self.rs = [int(x) for x in rs]
        self.h = tc_multi_create(self.rs, seeds)

    def process(self, bank_ids, edges_list, stream=None):
        tc_multi_process(self.h, bank_ids, edges_list, stream=stream)

    def estimate(self):
        return tc_multi_estimate(self.h)

    def state(self, bank: int):
        return tc_multi_read_state(self.h, bank, self.rs[bank])

    def sync(self):
        tc_multi_sync(self.h)

    def close(self):
        if self.h:
            tc_multi_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
