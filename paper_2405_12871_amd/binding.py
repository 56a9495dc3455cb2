"""Thin Python binding of the C ABI in ``include/imin.h``.

Argument marshalling only: every step of the estimator runs in the HIP
library.  PyTorch provides device memory and the stream.  There is no
fallback: a missing library or a missing GPU raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import re
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libimin.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "imin.h")

IMIN_OK = 0
STATUS_NAMES = {0: "IMIN_OK", 1: "IMIN_ERR_INVALID", 2: "IMIN_ERR_DATA", 3: "IMIN_ERR_DEVICE",
                4: "IMIN_ERR_NOMEM", 5: "IMIN_ERR_INTERNAL", 6: "IMIN_ERR_WORKSPACE"}

_lib = None


class Query(ctypes.Structure):
    """One entry of imin_solve_many and of the server (imin_query_t)."""
    _fields_ = [("graph", ctypes.c_void_p), ("seeds", ctypes.c_void_p), ("n_seeds", ctypes.c_int32),
                ("k", ctypes.c_int32),
                ("theta", ctypes.c_int64), ("rng_seed", ctypes.c_uint64), ("blockers", ctypes.c_void_p),
                ("gains", ctypes.c_void_p), ("spread_totals", ctypes.c_void_p), ("n_selected", ctypes.c_void_p),
                ("status", ctypes.c_int32), ("device_flags", ctypes.c_uint32)]


class EvalQuery(ctypes.Structure):
    """One entry of imin_evaluate_batch (imin_eval_query_t)."""
    _fields_ = [("seeds", ctypes.c_void_p), ("n_seeds", ctypes.c_int32), ("blocked", ctypes.c_void_p),
                ("n_blocked", ctypes.c_int32), ("w_begin", ctypes.c_int64), ("w_count", ctypes.c_int64),
                ("rng_seed", ctypes.c_uint64), ("gain", ctypes.c_void_p), ("total", ctypes.c_void_p),
                ("world_size", ctypes.c_void_p)]


class LsbmInfo(ctypes.Structure):
    """imin_lsbm_info_t: every intermediate quantity of an LSBM call."""
    _fields_ = [("returned_on", ctypes.c_int32), ("on_size", ctypes.c_int32),
                ("reach_bound", ctypes.c_int64), ("sra_worlds", ctypes.c_int64),
                ("i_hat", ctypes.c_double), ("opt_l", ctypes.c_double),
                ("theta_max", ctypes.c_double), ("theta_0", ctypes.c_double),
                ("i_max", ctypes.c_int32), ("iterations", ctypes.c_int32), ("theta", ctypes.c_int64),
                ("cov1", ctypes.c_int64), ("cov2", ctypes.c_int64), ("cov_upper", ctypes.c_int64),
                ("sigma_l", ctypes.c_double), ("sigma_u", ctypes.c_double), ("a1", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class GsbmInfo(ctypes.Structure):
    """imin_gsbm_info_t."""
    _fields_ = [("returned_on", ctypes.c_int32), ("on_size", ctypes.c_int32), ("nvp", ctypes.c_int64),
                ("sra_worlds", ctypes.c_int64), ("opt_l", ctypes.c_double), ("theta_max", ctypes.c_double),
                ("theta_0", ctypes.c_double), ("i_max", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("theta", ctypes.c_int64), ("cov1", ctypes.c_int64), ("cov2", ctypes.c_int64),
                ("cov_upper", ctypes.c_int64), ("sigma_l", ctypes.c_double), ("sigma_u", ctypes.c_double),
                ("a1", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class SandiminInfo(ctypes.Structure):
    """imin_sandimin_info_t."""
    _fields_ = [("choice", ctypes.c_int32), ("n_blockers", ctypes.c_int32 * 3), ("estimate", ctypes.c_double * 3),
                ("eval_worlds", ctypes.c_int64 * 3), ("lsbm", LsbmInfo), ("gsbm", GsbmInfo)]

    def as_dict(self) -> dict:
        return dict(choice=self.choice, n_blockers=list(self.n_blockers), estimate=list(self.estimate),
                    eval_worlds=list(self.eval_worlds), lsbm=self.lsbm.as_dict(), gsbm=self.gsbm.as_dict())


class IminError(RuntimeError):
    def __init__(self, status: int, message: str, flags: int = 0):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message} (device flags 0x{flags:x})")
        self.status = status
        self.flags = flags


def header_functions() -> list[str]:
    """Names of the functions declared in include/imin.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(imin_[a-z_]+)\s*\(", text)))


def load():
    """Load libimin.so (built by ``paper_2405_12871_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2405_12871_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    st = ctypes.c_int
    lib.imin_graph_create.argtypes = [i32, i64, P, P, P, P, ctypes.POINTER(P)]
    lib.imin_graph_create.restype = st
    lib.imin_graph_destroy.argtypes = [P]
    lib.imin_graph_destroy.restype = st
    lib.imin_graph_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.imin_graph_info.restype = st
    lib.imin_solve.argtypes = [P, P, i32, i32, i64, u64, P, ctypes.c_size_t, P, P, P, P, P, P]
    lib.imin_solve.restype = st
    lib.imin_solve_workspace_size.argtypes = [P, i32, i32, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.imin_solve_workspace_size.restype = st
    lib.imin_solve_static.argtypes = [P, P, i32, i32, i64, u64, P, P, P, P, P, P]
    lib.imin_solve_static.restype = st
    lib.imin_solve_many.argtypes = [P, ctypes.POINTER(Query), i32, ctypes.POINTER(P), i32, ctypes.c_size_t]
    lib.imin_solve_many.restype = st
    lib.imin_server_create.argtypes = [P, ctypes.POINTER(P), i32, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.imin_server_create.restype = st
    lib.imin_server_submit.argtypes = [P, ctypes.POINTER(Query)]
    lib.imin_server_submit.restype = st
    lib.imin_server_next.argtypes = [P, ctypes.POINTER(ctypes.POINTER(Query))]
    lib.imin_server_next.restype = st
    lib.imin_server_destroy.argtypes = [P]
    lib.imin_server_destroy.restype = st
    lib.imin_evaluate.argtypes = [P, P, i32, P, i32, i64, i64, u64, P, P, P, P, P, P]
    lib.imin_evaluate.restype = st
    lib.imin_evaluate_batch.argtypes = [P, ctypes.POINTER(EvalQuery), i32, P]
    lib.imin_evaluate_batch.restype = st
    lib.imin_status_string.argtypes = [st]
    lib.imin_status_string.restype = ctypes.c_char_p
    lib.imin_last_device_flags.argtypes = []
    lib.imin_last_device_flags.restype = ctypes.c_uint32
    lib.imin_timing_enable.argtypes = [ctypes.c_int]
    lib.imin_timing_enable.restype = st
    lib.imin_timing_mask.argtypes = [ctypes.c_uint32]
    lib.imin_timing_mask.restype = st
    lib.imin_timing_sample.argtypes = [ctypes.c_int]
    lib.imin_timing_sample.restype = st
    lib.imin_timing_tallies.argtypes = [ctypes.c_int]
    lib.imin_timing_tallies.restype = st
    lib.imin_timing_launches.argtypes = [ctypes.c_int, ctypes.POINTER(i64)]
    lib.imin_timing_launches.restype = st
    lib.imin_cache_release.argtypes = []
    lib.imin_cache_release.restype = st
    lib.imin_timing_reset.argtypes = []
    lib.imin_timing_reset.restype = st
    lib.imin_timing_read.argtypes = [ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    lib.imin_timing_read.restype = st
    lib.imin_timing_work.argtypes = [ctypes.c_int] + [ctypes.POINTER(i64)] * 5
    lib.imin_timing_work.restype = st
    lib.imin_probe_philox.argtypes = [i64, i32, u64, P, i64, i32, P, ctypes.POINTER(ctypes.c_float)]
    lib.imin_probe_philox.restype = st
    lib.imin_probe_copy.argtypes = [P, P, ctypes.c_size_t, i32, P, ctypes.POINTER(ctypes.c_float)]
    lib.imin_probe_copy.restype = st
    lib.imin_graph_export.argtypes = [P, P, P, P]
    lib.imin_graph_export.restype = st
    lib.imin_max_coverage.argtypes = [P, P, i32, i32, i64, u64, P, P, P, P, P, P]
    lib.imin_max_coverage.restype = st
    lib.imin_coverage.argtypes = [P, P, i32, P, i32, i64, u64, P, P]
    lib.imin_coverage.restype = st
    lib.imin_reach_counts.argtypes = [P, P, i32, i64, i64, u64, P, P, P]
    lib.imin_reach_counts.restype = st
    lib.imin_lsbm.argtypes = [P, P, i32, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, u64, P, P, P,
                              ctypes.POINTER(LsbmInfo)]
    lib.imin_lsbm.restype = st
    lib.imin_autotune.argtypes = [P, P, i32, i64, u64, P, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    lib.imin_autotune.restype = st
    lib.imin_set_launch_shape.argtypes = [P, i32]
    lib.imin_set_launch_shape.restype = st
    lib.imin_last_solve_incremental.argtypes = []
    lib.imin_last_solve_incremental.restype = i32
    lib.imin_world_sizes.argtypes = [P, P, i32, P, i32, i64, i64, u64, P, P]
    lib.imin_world_sizes.restype = st
    lib.imin_vprime.argtypes = [P, P, i32, P, P, ctypes.POINTER(i32)]
    lib.imin_vprime.restype = st
    lib.imin_lrr_max_coverage.argtypes = [P, P, i32, i32, i64, u64, P, P, P, P, P, P]
    lib.imin_lrr_max_coverage.restype = st
    lib.imin_lrr_coverage.argtypes = [P, P, i32, P, i32, i64, u64, P, P]
    lib.imin_lrr_coverage.restype = st
    lib.imin_gsbm.argtypes = [P, P, i32, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, u64, P, P, P,
                              ctypes.POINTER(GsbmInfo)]
    lib.imin_gsbm.restype = st
    lib.imin_lhga.argtypes = [P, P, i32, i32, ctypes.c_double, ctypes.c_double, u64, P, P, P]
    lib.imin_lhga.restype = st
    lib.imin_sandimin.argtypes = [P, P, i32, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, u64, P, P, P, P, ctypes.POINTER(SandiminInfo)]
    lib.imin_sandimin.restype = st
    _lib = lib
    return lib


def _check(status: int):
    if status != IMIN_OK:
        lib = load()
        raise IminError(status, lib.imin_status_string(status).decode(), int(lib.imin_last_device_flags()))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the IMIN library runs on the device only")
    return torch


def _dev(a, dtype, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dtype).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Graph:
    """A graph resident on the GPU (imin_graph_create / imin_graph_destroy)."""

    def __init__(self, n: int, row_ptr, col, p, device="cuda:0"):
        torch = _torch()
        lib = load()
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            rp = _dev(row_ptr, torch.int64, self.device)
            cl = _dev(col, torch.int32, self.device)
            pp = _dev(p, torch.float32, self.device)
            m = int(cl.numel())
            h = ctypes.c_void_p()
            _check(lib.imin_graph_create(int(n), m, _ptr(rp), _ptr(cl) if m else None,
                                         _ptr(pp) if m else None, _stream(self.device), ctypes.byref(h)))
        self._h = h
        self.n = int(n)
        self.m = m

    @classmethod
    def from_synth(cls, g, device="cuda:0"):
        return cls(g.n, g.row_ptr, g.col, g.p, device=device)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("graph already destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            load().imin_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


@dataclasses.dataclass
class SolveResult:
    blockers: np.ndarray
    gains: np.ndarray
    spread_totals: np.ndarray
    n_selected: int
    theta: int

    @property
    def est_spread(self) -> float:
        """Estimated expected spread after blocking: T_final / theta."""
        return float(self.spread_totals[self.n_selected]) / float(self.theta)

    @property
    def est_decrease(self) -> float:
        return float(self.spread_totals[0] - self.spread_totals[self.n_selected]) / float(self.theta)


def _solve_outputs(k: int, dev):
    torch = _torch()
    return (torch.zeros(max(k, 1), dtype=torch.int32, device=dev),
            torch.zeros(max(k, 1), dtype=torch.int64, device=dev),
            torch.zeros(k + 1, dtype=torch.int64, device=dev),
            torch.zeros(1, dtype=torch.int32, device=dev))


def solve_device(graph: Graph, seeds_dev, k: int, theta: int, rng_seed: int, out=None):
    """imin_solve on device tensors, scratch from the library's cache (the
    call waits for its work); returns the device output tensors."""
    torch = _torch()
    lib = load()
    dev = graph.device
    if out is None:
        out = _solve_outputs(k, dev)
    b, g, t, ns = out
    with torch.cuda.device(dev):
        _check(lib.imin_solve(graph.handle, _ptr(seeds_dev), int(seeds_dev.numel()), int(k), int(theta),
                              int(rng_seed) & 0xFFFFFFFFFFFFFFFF, None, 0, _stream(dev), _ptr(b), _ptr(g), _ptr(t),
                              _ptr(ns), None))
    return out


def workspace_size(graph: Graph, n_seeds: int, k: int, theta: int) -> int:
    """Bytes of workspace an enqueued solve needs (imin_solve_workspace_size)."""
    nbytes = ctypes.c_size_t()
    _check(load().imin_solve_workspace_size(graph.handle, int(n_seeds), int(k), int(theta), ctypes.byref(nbytes)))
    return int(nbytes.value)


def solve_enqueue(graph: Graph, seeds_dev, k: int, theta: int, rng_seed: int, workspace, out=None, status=None,
                  stream=None):
    """imin_solve with a workspace (a uint8 device tensor): only enqueues on
    ``stream`` (default: the current stream).  Returns (outputs, status
    tensor); the status (0 = ok, else an imin_status_t) is valid once the
    stream has reached the end of the solve."""
    torch = _torch()
    lib = load()
    dev = graph.device
    if out is None:
        out = _solve_outputs(k, dev)
    if status is None:
        status = torch.full((1,), -1, dtype=torch.int32, device=dev)
    b, g, t, ns = out
    st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(dev)
    with torch.cuda.device(dev):
        _check(lib.imin_solve(graph.handle, _ptr(seeds_dev), int(seeds_dev.numel()), int(k), int(theta),
                              int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _ptr(workspace), workspace.numel(), st, _ptr(b),
                              _ptr(g), _ptr(t), _ptr(ns), _ptr(status)))
    return out, status


def solve_static(graph: Graph, seeds, k: int, theta: int, rng_seed: int) -> "SolveResult":
    """imin_solve_static (the workspace is the library's fixed device array),
    waited for; raises on a non-zero device status."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    out = _solve_outputs(k, dev)
    status = torch.full((1,), -1, dtype=torch.int32, device=dev)
    b, g, t, ns = out
    with torch.cuda.device(dev):
        _check(lib.imin_solve_static(graph.handle, _ptr(s), int(s.numel()), int(k), int(theta),
                                     int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(b), _ptr(g), _ptr(t),
                                     _ptr(ns), _ptr(status)))
    torch.cuda.synchronize(dev)
    code = int(status.cpu()[0])
    if code != IMIN_OK:
        raise IminError(code, lib.imin_status_string(code).decode(), 0)
    return result_of(out, theta)


def result_of(out, theta: int) -> "SolveResult":
    """The host copy of a solve's device outputs."""
    b, g, t, ns = out
    r = int(ns.cpu()[0])
    return SolveResult(blockers=b.cpu().numpy()[:r].copy(), gains=g.cpu().numpy()[:r].copy(),
                       spread_totals=t.cpu().numpy()[:r + 1].copy(), n_selected=r, theta=int(theta))


def solve_ws(graph: Graph, seeds, k: int, theta: int, rng_seed: int, workspace=None) -> "SolveResult":
    """An enqueued solve in a workspace of imin_solve_workspace_size bytes
    (allocated here unless given), waited for; raises on a non-zero device
    status."""
    torch = _torch()
    s = _dev(seeds, torch.int32, graph.device)
    if workspace is None:
        workspace = torch.empty(workspace_size(graph, s.numel(), k, theta), dtype=torch.uint8, device=graph.device)
    out, status = solve_enqueue(graph, s, k, theta, rng_seed, workspace)
    torch.cuda.synchronize(graph.device)
    code = int(status.cpu()[0])
    if code != IMIN_OK:
        raise IminError(code, load().imin_status_string(code).decode(), 0)
    return result_of(out, theta)


def solve(graph: Graph, seeds, k: int, theta: int, rng_seed: int) -> SolveResult:
    """Greedy selection of up to k blockers (imin_solve)."""
    torch = _torch()
    s = _dev(seeds, torch.int32, graph.device)
    b, g, t, ns = solve_device(graph, s, k, theta, rng_seed)
    r = int(ns.cpu()[0])
    return SolveResult(blockers=b.cpu().numpy()[:r].copy(), gains=g.cpu().numpy()[:r].copy(),
                       spread_totals=t.cpu().numpy()[:r + 1].copy(), n_selected=r, theta=int(theta))


def _query_entry(graph, default, seeds, k, theta, rng_seed):
    """A Query entry with its device tensors (kept alive by the caller)."""
    torch = _torch()
    g = graph if graph is not None else default
    s = _dev(seeds, torch.int32, g.device)
    out = _solve_outputs(k, g.device)
    q = Query(g.handle.value if graph is not None else None, s.data_ptr(), int(s.numel()), int(k), int(theta),
              int(rng_seed) & 0xFFFFFFFFFFFFFFFF, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
              out[3].data_ptr(), 0, 0)
    return q, (s, out)


def _split_query(item):
    """(graph or None, seeds, k, theta, rng_seed) from a 4- or 5-tuple."""
    if len(item) == 5:
        return item
    return (None,) + tuple(item)


def solve_many(graph: Graph, queries, n_streams: int = 4, raise_on_error: bool = True, hbm_budget: int = 0):
    """Many selections side by side (imin_solve_many).

    ``queries`` is a sequence of (seeds, k, theta, rng_seed) on ``graph`` or
    (graph, seeds, k, theta, rng_seed) on another resident graph.  Returns one
    SolveResult per query, each equal to solve() of that query alone.  A
    failing query raises IminError (naming the query) or, with
    ``raise_on_error=False``, takes an IminError in its place in the list.
    ``hbm_budget`` is the byte size of the workspace pool (0: the library's
    default).
    """
    torch = _torch()
    lib = load()
    dev = graph.device
    n = len(queries)
    arr = (Query * max(n, 1))()
    keep = []
    for i, item in enumerate(queries):
        gq, seeds, k, theta, rng_seed = _split_query(item)
        arr[i], tensors = _query_entry(gq, graph, seeds, k, theta, rng_seed)
        keep.append((tensors, int(theta)))
    streams = [torch.cuda.Stream(device=dev) for _ in range(max(1, min(int(n_streams), max(n, 1))))]
    handles = (ctypes.c_void_p * len(streams))(*[st.cuda_stream for st in streams])
    torch.cuda.synchronize(dev)  # inputs and zeroed outputs are ready for every stream
    with torch.cuda.device(dev):
        lib.imin_solve_many(graph.handle, arr, n, handles, len(streams), int(hbm_budget))
    results = []
    for i, ((s, out), theta) in enumerate(keep):
        r = _query_result(lib, arr[i], out, theta, f"query {i}")
        if isinstance(r, IminError) and raise_on_error:
            raise r
        results.append(r)
    return results


def _query_result(lib, q: Query, out, theta: int, label: str):
    """SolveResult of a finished query, or the IminError it ended with."""
    status = int(q.status)
    if status != IMIN_OK:
        return IminError(status, f"{label}: " + lib.imin_status_string(status).decode(), int(q.device_flags))
    b, g, t, ns = out
    r = int(ns.cpu()[0])
    return SolveResult(blockers=b.cpu().numpy()[:r].copy(), gains=g.cpu().numpy()[:r].copy(),
                       spread_totals=t.cpu().numpy()[:r + 1].copy(), n_selected=r, theta=int(theta))


class Server:
    """Queries solved as they arrive, admitted by workspace size into a pool
    of device memory and run side by side on several streams
    (imin_server_create / submit / next / destroy)."""

    def __init__(self, graph: Graph, n_streams: int = 4, hbm_budget: int = 0):
        torch = _torch()
        lib = load()
        self.graph = graph
        self._streams = [torch.cuda.Stream(device=graph.device) for _ in range(max(1, int(n_streams)))]
        handles = (ctypes.c_void_p * len(self._streams))(*[st.cuda_stream for st in self._streams])
        h = ctypes.c_void_p()
        with torch.cuda.device(graph.device):
            _check(lib.imin_server_create(graph.handle, handles, len(self._streams), int(hbm_budget),
                                          ctypes.byref(h)))
        self._h = h
        # address of a query entry -> (ticket, entry, its tensors, theta); an
        # address is unique among outstanding queries, tickets for ever
        self._pending = {}
        self._tickets = 0
        self._lock = threading.Lock()

    def submit(self, seeds, k: int, theta: int, rng_seed: int, graph: "Graph" = None) -> int:
        """Queue one query (on ``graph``, default the server's); returns its
        ticket (a serial number) at once."""
        torch = _torch()
        lib = load()
        q, tensors = _query_entry(graph, self.graph, seeds, k, theta, rng_seed)
        torch.cuda.current_stream(self.graph.device).synchronize()  # inputs and zeroed outputs ready
        addr = ctypes.addressof(q)
        with self._lock:
            ticket = self._tickets
            self._tickets += 1
            self._pending[addr] = (ticket, q, tensors, int(theta))
        status = lib.imin_server_submit(self._h, ctypes.byref(q))
        if status != IMIN_OK:
            with self._lock:
                del self._pending[addr]
            _check(status)
        return ticket

    def next(self):
        """(ticket, SolveResult or IminError) of the next query to finish;
        blocks until one has."""
        lib = load()
        p = ctypes.POINTER(Query)()
        _check(lib.imin_server_next(self._h, ctypes.byref(p)))
        with self._lock:
            ticket, q, (s, out), theta = self._pending.pop(ctypes.addressof(p.contents))
        return ticket, _query_result(lib, q, out, theta, f"query {ticket}")

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().imin_server_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def evaluate(graph: Graph, seeds, w_begin: int, w_count: int, rng_seed: int, blocked=(),
             per_world: bool = False, edges: bool = False):
    """One estimator pass over worlds [w_begin, w_begin + w_count) (imin_evaluate).

    Returns (gain int64[n], total) or, with ``per_world``,
    (gain, total, world_size int32[w_count], world_sum int64[w_count]); with
    ``edges`` the per-world scanned-edge counts int64[w_count] are appended.
    """
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    blk = list(blocked) if not isinstance(blocked, torch.Tensor) else blocked
    b = _dev(np.asarray(blk, dtype=np.int32), torch.int32, dev) if len(blk) else None
    gain = torch.empty(graph.n, dtype=torch.int64, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(w_count, dtype=torch.int32, device=dev) if per_world else None
    wsum = torch.empty(w_count, dtype=torch.int64, device=dev) if per_world else None
    wedge = torch.empty(w_count, dtype=torch.int64, device=dev) if edges else None
    with torch.cuda.device(dev):
        _check(lib.imin_evaluate(graph.handle, _ptr(s), int(s.numel()), _ptr(b),
                                 int(b.numel()) if b is not None else 0, int(w_begin), int(w_count),
                                 int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(gain), _ptr(total),
                                 _ptr(ws), _ptr(wsum), _ptr(wedge)))
    res = [gain.cpu().numpy(), int(total.cpu()[0])]
    if per_world:
        res += [ws.cpu().numpy(), wsum.cpu().numpy()]
    if edges:
        res.append(wedge.cpu().numpy())
    return tuple(res)


def evaluate_device(graph: Graph, seeds_dev, w_begin: int, w_count: int, rng_seed: int, gain, total):
    """imin_evaluate on device tensors with no blocked set and no per-world
    outputs: gain (int64[n]) and total (int64[1]) are written in place."""
    torch = _torch()
    lib = load()
    dev = graph.device
    with torch.cuda.device(dev):
        _check(lib.imin_evaluate(graph.handle, _ptr(seeds_dev), int(seeds_dev.numel()), None, 0, int(w_begin),
                                 int(w_count), int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(gain),
                                 _ptr(total), None, None, None))


def evaluate_batch(graph: Graph, queries, per_world: bool = False):
    """imin_evaluate_batch: one estimator pass per query, the tier-0 world
    launches packed.  queries: a list of dicts with seeds, w_begin, w_count,
    rng_seed and optionally blocked.  Returns a list of (gain, total) or, with
    ``per_world``, (gain, total, world_size)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    keep, out = [], []
    arr = (EvalQuery * max(len(queries), 1))()
    for j, qd in enumerate(queries):
        s = _dev(qd["seeds"], torch.int32, dev)
        blk = qd.get("blocked", ())
        blk = list(blk) if not isinstance(blk, torch.Tensor) else blk
        b = _dev(np.asarray(blk, dtype=np.int32), torch.int32, dev) if len(blk) else None
        gain = torch.empty(graph.n, dtype=torch.int64, device=dev)
        total = torch.empty(1, dtype=torch.int64, device=dev)
        ws = torch.empty(int(qd["w_count"]), dtype=torch.int32, device=dev) if per_world else None
        keep += [s, b]
        out.append((gain, total, ws))
        arr[j] = EvalQuery(_ptr(s), int(s.numel()), _ptr(b), int(b.numel()) if b is not None else 0,
                           int(qd["w_begin"]), int(qd["w_count"]), int(qd["rng_seed"]) & 0xFFFFFFFFFFFFFFFF,
                           _ptr(gain), _ptr(total), _ptr(ws))
    with torch.cuda.device(dev):
        _check(lib.imin_evaluate_batch(graph.handle, arr, len(queries), _stream(dev)))
    res = []
    for gain, total, ws in out:
        r = [gain.cpu().numpy(), int(total.cpu()[0])]
        if per_world:
            r.append(ws.cpu().numpy())
        res.append(tuple(r))
    return res


def evaluate_batch_device(graph: Graph, entries):
    """imin_evaluate_batch on device tensors: entries is a list of (seeds_dev,
    w_begin, w_count, rng_seed, gain, total), gain and total written in place."""
    torch = _torch()
    lib = load()
    dev = graph.device
    arr = (EvalQuery * max(len(entries), 1))()
    for j, (sd, wb, wc, seed, gain, total) in enumerate(entries):
        arr[j] = EvalQuery(_ptr(sd), int(sd.numel()), None, 0, int(wb), int(wc), int(seed) & 0xFFFFFFFFFFFFFFFF,
                           _ptr(gain), _ptr(total), None)
    with torch.cuda.device(dev):
        _check(lib.imin_evaluate_batch(graph.handle, arr, len(entries), _stream(dev)))


def cache_release():
    """Free the device blocks the library keeps cached between calls."""
    _check(load().imin_cache_release())


def timing_enable(on: bool = True):
    _check(load().imin_timing_enable(1 if on else 0))


def timing_tallies(on: bool = True):
    """Keep the work tallies of timed calls (imin_timing_tallies)."""
    _check(load().imin_timing_tallies(1 if on else 0))


def timing_mask(kernel_ids=None):
    """Bracket only these kernel ids with events (None: all)."""
    mask = 0xFFFFFFFF if kernel_ids is None else sum(1 << int(i) for i in kernel_ids)
    _check(load().imin_timing_mask(mask))


def timing_sample(every: int = 1):
    """Time one launch in ``every`` of each selected kernel."""
    _check(load().imin_timing_sample(int(every)))


def timing_launches(kernel_id: int) -> int:
    """Launches of a selected kernel since the last reset, timed or not."""
    n = ctypes.c_int64()
    _check(load().imin_timing_launches(int(kernel_id), ctypes.byref(n)))
    return int(n.value)


def timing_reset():
    _check(load().imin_timing_reset())


def timing_read(kernel_id: int):
    """(launches, total milliseconds) of one library kernel since the last reset."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().imin_timing_read(int(kernel_id), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def timing_work(tier: int):
    """(worlds, edges walked, algorithmic bytes, reached nodes, live edges) of
    one world tier (0-2 sampled tiers, 3 replay, 4 label rule by the
    label-rule workgroups, 5 label rule by the replay workgroups) since the
    last reset; reached nodes and live edges for tiers 0-2 only."""
    v = [ctypes.c_int64() for _ in range(5)]
    _check(load().imin_timing_work(int(tier), *[ctypes.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


def probe_philox(worlds: int, groups_per_world: int, key: int, grid: int, device="cuda:0") -> float:
    """Milliseconds of one launch drawing worlds * groups_per_world Philox
    blocks (4 coins each) with the world kernels' coin layout."""
    torch = _torch()
    out = torch.empty(grid * 256, dtype=torch.int32, device=device)
    ms = ctypes.c_float()
    _check(load().imin_probe_philox(int(worlds), int(groups_per_world), int(key), _ptr(out), out.numel(), int(grid),
                                    _stream(device), ctypes.byref(ms)))
    return float(ms.value)


def probe_copy(dst, src, grid: int) -> float:
    """Milliseconds of one device copy of src into dst (torch tensors of the
    same byte size, a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    ms = ctypes.c_float()
    _check(load().imin_probe_copy(_ptr(dst), _ptr(src), nbytes, int(grid), _stream(src.device), ctypes.byref(ms)))
    return float(ms.value)


# ------------------------------------------------------ lower-bound coverage
def graph_export(graph: Graph):
    """(row_ptr int64[n+1], col int32[m], thr uint32[m]) of the handle (imin_graph_export)."""
    lib = load()
    row_ptr = np.zeros(graph.n + 1, dtype=np.int64)
    col = np.zeros(max(graph.m, 1), dtype=np.int32)
    thr = np.zeros(max(graph.m, 1), dtype=np.uint32)
    _check(lib.imin_graph_export(graph.handle, row_ptr.ctypes.data_as(ctypes.c_void_p),
                                 col.ctypes.data_as(ctypes.c_void_p), thr.ctypes.data_as(ctypes.c_void_p)))
    return row_ptr, col[:graph.m], thr[:graph.m]


def max_coverage(graph: Graph, seeds, k: int, theta: int, rng_seed: int) -> dict:
    """Max-Coverage over the CP sequences of worlds [0, theta) (imin_max_coverage):
    dict(blockers, gains, cov, cov_upper, n_selected), cov and cov_upper over
    the prefixes B_0 .. B_{n_selected}."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    blockers = torch.zeros(max(k, 1), dtype=torch.int32, device=dev)
    gains = torch.zeros(max(k, 1), dtype=torch.int64, device=dev)
    cov = torch.zeros(k + 1, dtype=torch.int64, device=dev)
    cu = torch.zeros(k + 1, dtype=torch.int64, device=dev)
    nsel = torch.zeros(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(lib.imin_max_coverage(graph.handle, _ptr(s), int(s.numel()), int(k), int(theta),
                                     int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(blockers), _ptr(gains),
                                     _ptr(cov), _ptr(cu), _ptr(nsel)))
    r = int(nsel.cpu()[0])
    return dict(blockers=blockers.cpu().numpy()[:r], gains=gains.cpu().numpy()[:r],
                cov=cov.cpu().numpy()[:r + 1], cov_upper=cu.cpu().numpy()[:r + 1], n_selected=r)


def coverage(graph: Graph, seeds, blockers, theta: int, rng_seed: int) -> int:
    """Cov(blockers) over the CP sequences of worlds [0, theta) (imin_coverage)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    b = np.asarray(blockers, dtype=np.int32)
    bd = _dev(b, torch.int32, dev) if b.size else None
    out = torch.zeros(1, dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        _check(lib.imin_coverage(graph.handle, _ptr(s), int(s.numel()), _ptr(bd), int(b.size), int(theta),
                                 int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(out)))
    return int(out.cpu()[0])


def reach_counts(graph: Graph, seeds, w_begin: int, w_count: int, rng_seed: int, per_world: bool = False):
    """Per-node reach counts over worlds [w_begin, w_begin + w_count)
    (imin_reach_counts); with per_world also |R_w| per world."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    counts = torch.zeros(graph.n, dtype=torch.int64, device=dev)
    ws = torch.zeros(w_count, dtype=torch.int32, device=dev) if per_world else None
    with torch.cuda.device(dev):
        _check(lib.imin_reach_counts(graph.handle, _ptr(s), int(s.numel()), int(w_begin), int(w_count),
                                     int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(counts), _ptr(ws)))
    if per_world:
        return counts.cpu().numpy(), ws.cpu().numpy()
    return counts.cpu().numpy()


def lsbm(graph: Graph, seeds, k: int, eps: float = 0.2, beta: float = 0.1, delta: float | None = None,
         rng_seed: int = 0) -> dict:
    """LSBM, Algorithm 4 (imin_lsbm): dict(blockers, n_selected, info)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    if delta is None:
        delta = 1.0 / graph.n
    blockers = torch.zeros(max(k, 1), dtype=torch.int32, device=dev)
    nsel = torch.zeros(1, dtype=torch.int32, device=dev)
    info = LsbmInfo()
    with torch.cuda.device(dev):
        _check(lib.imin_lsbm(graph.handle, _ptr(s), int(s.numel()), int(k), float(eps), float(beta), float(delta),
                             int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(blockers), _ptr(nsel),
                             ctypes.byref(info)))
    r = int(nsel.cpu()[0])
    return dict(blockers=blockers.cpu().numpy()[:r], n_selected=r, info=info.as_dict())


def world_sizes(graph: Graph, seeds, w_begin: int, w_count: int, rng_seed: int, blocked=()) -> np.ndarray:
    """|R_w(B)| of worlds [w_begin, w_begin + w_count) (imin_world_sizes)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    b = np.asarray(list(blocked), dtype=np.int32)
    bd = _dev(b, torch.int32, dev) if b.size else None
    out = torch.zeros(w_count, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(lib.imin_world_sizes(graph.handle, _ptr(s), int(s.numel()), _ptr(bd), int(b.size), int(w_begin),
                                    int(w_count), int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(out)))
    return out.cpu().numpy()


def vprime(graph: Graph, seeds) -> np.ndarray:
    """V'_s (imin_vprime)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    cnt = ctypes.c_int32(0)
    with torch.cuda.device(dev):
        _check(lib.imin_vprime(graph.handle, _ptr(s), int(s.numel()), _stream(dev), None, ctypes.byref(cnt)))
        out = torch.zeros(max(cnt.value, 1), dtype=torch.int32, device=dev)
        _check(lib.imin_vprime(graph.handle, _ptr(s), int(s.numel()), _stream(dev), _ptr(out), ctypes.byref(cnt)))
    return out.cpu().numpy()[:cnt.value]


def lrr_max_coverage(graph: Graph, seeds, k: int, theta: int, key: int) -> dict:
    """Max-Coverage over the LRR sets of samples [0, theta) (imin_lrr_max_coverage)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    blockers = torch.zeros(max(k, 1), dtype=torch.int32, device=dev)
    gains = torch.zeros(max(k, 1), dtype=torch.int64, device=dev)
    cov = torch.zeros(k + 1, dtype=torch.int64, device=dev)
    cu = torch.zeros(k + 1, dtype=torch.int64, device=dev)
    nsel = torch.zeros(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(lib.imin_lrr_max_coverage(graph.handle, _ptr(s), int(s.numel()), int(k), int(theta),
                                         int(key) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(blockers), _ptr(gains),
                                         _ptr(cov), _ptr(cu), _ptr(nsel)))
    r = int(nsel.cpu()[0])
    return dict(blockers=blockers.cpu().numpy()[:r], gains=gains.cpu().numpy()[:r],
                cov=cov.cpu().numpy()[:r + 1], cov_upper=cu.cpu().numpy()[:r + 1], n_selected=r)


def lrr_coverage(graph: Graph, seeds, blockers, theta: int, key: int) -> int:
    """Cov(blockers) over the LRR sets of samples [0, theta) (imin_lrr_coverage)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    b = np.asarray(blockers, dtype=np.int32)
    bd = _dev(b, torch.int32, dev) if b.size else None
    out = torch.zeros(1, dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        _check(lib.imin_lrr_coverage(graph.handle, _ptr(s), int(s.numel()), _ptr(bd), int(b.size), int(theta),
                                     int(key) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(out)))
    return int(out.cpu()[0])


def gsbm(graph: Graph, seeds, k: int, eps: float = 0.2, beta: float = 0.1, delta: float | None = None,
         rng_seed: int = 0) -> dict:
    """GSBM (imin_gsbm): dict(blockers, n_selected, info)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    if delta is None:
        delta = 1.0 / graph.n
    blockers = torch.zeros(max(k, 1), dtype=torch.int32, device=dev)
    nsel = torch.zeros(1, dtype=torch.int32, device=dev)
    info = GsbmInfo()
    with torch.cuda.device(dev):
        _check(lib.imin_gsbm(graph.handle, _ptr(s), int(s.numel()), int(k), float(eps), float(beta), float(delta),
                             int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(blockers), _ptr(nsel),
                             ctypes.byref(info)))
    r = int(nsel.cpu()[0])
    return dict(blockers=blockers.cpu().numpy()[:r], n_selected=r, info=info.as_dict())


def lhga(graph: Graph, seeds, k: int, beta: float = 0.1, delta: float | None = None, rng_seed: int = 0):
    """LHGA (imin_lhga): the blockers in decreasing score order."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    if delta is None:
        delta = 1.0 / graph.n
    blockers = torch.zeros(max(k, 1), dtype=torch.int32, device=dev)
    nsel = torch.zeros(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(lib.imin_lhga(graph.handle, _ptr(s), int(s.numel()), int(k), float(beta), float(delta),
                             int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), _ptr(blockers), _ptr(nsel)))
    return blockers.cpu().numpy()[:int(nsel.cpu()[0])]


def sandimin(graph: Graph, seeds, k: int, eps: float = 0.2, beta: float = 0.1, gamma: float = 0.1,
             delta: float | None = None, rng_seed: int = 0) -> dict:
    """SandIMIN, Algorithm 1 (imin_sandimin): dict(blockers, choice, B_L, B_U, B_R, info)."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    if delta is None:
        delta = 1.0 / graph.n
    blockers = torch.zeros(max(k, 1), dtype=torch.int32, device=dev)
    nsel = torch.zeros(1, dtype=torch.int32, device=dev)
    cand = torch.zeros(3 * max(k, 1), dtype=torch.int32, device=dev)
    info = SandiminInfo()
    with torch.cuda.device(dev):
        _check(lib.imin_sandimin(graph.handle, _ptr(s), int(s.numel()), int(k), float(eps), float(beta),
                                 float(gamma), float(delta), int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev),
                                 _ptr(blockers), _ptr(nsel), _ptr(cand), ctypes.byref(info)))
    d = info.as_dict()
    c = cand.cpu().numpy()
    sets = [c[i * k:i * k + d["n_blockers"][i]] for i in range(3)]
    return dict(blockers=blockers.cpu().numpy()[:int(nsel.cpu()[0])], choice="LUR"[d["choice"]], B_L=sets[0],
                B_U=sets[1], B_R=sets[2], info=d)


def last_solve_incremental() -> int:
    """1 when this thread's last blocking solve ran incremental rounds, 0 plain, -1 none."""
    return int(load().imin_last_solve_incremental())


def autotune(graph: Graph, seeds, theta: int, rng_seed: int = 0):
    """(grid0_pct, pass_ms): the tier-0 launch shape imin_autotune keeps for the graph."""
    torch = _torch()
    lib = load()
    dev = graph.device
    s = _dev(seeds, torch.int32, dev)
    pct = ctypes.c_int32(0)
    ms = ctypes.c_float(0.0)
    with torch.cuda.device(dev):
        _check(lib.imin_autotune(graph.handle, _ptr(s), int(s.numel()), int(theta),
                                 int(rng_seed) & 0xFFFFFFFFFFFFFFFF, _stream(dev), ctypes.byref(pct), ctypes.byref(ms)))
    return int(pct.value), float(ms.value)


def set_launch_shape(graph: Graph, grid0_pct: int):
    """imin_set_launch_shape: 0 restores the default shape."""
    _check(load().imin_set_launch_shape(graph.handle, int(grid0_pct)))
