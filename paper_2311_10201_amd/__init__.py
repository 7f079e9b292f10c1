"""Python binding of libbpt: fused breadth-first probabilistic traversals that
sample RRR sets on an AMD MI355X (gfx950).

Argument marshalling only.  Every step of the sampling runs in the HIP
library ``libbpt.so`` (built by ``paper_2311_10201_amd.build``); calls raise
``RuntimeError`` if the library is missing.  Function names follow the C ABI
declared in ``include/bpt.h``.  PyTorch tensors may be passed wherever a
device buffer or stream is expected (``bpt_sample_rrr_device``).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "BPT_OK", "BPT_EINVAL", "BPT_ENOMEM", "BPT_EDEVICE", "BPT_ERANGE", "BPT_EINTERNAL",
    "BPT_PROB_UNIFORM", "BPT_PROB_ROW", "BPT_PROB_EDGE", "BPT_FLAG_UNFUSED", "BPT_FLAG_SORTED_STARTS",
    "BptError", "Counters", "Graph", "Job", "RRRResult", "Request", "Server", "BPT_REQ_SAMPLE", "BPT_REQ_SEEDS",
    "bpt_create_graph", "bpt_sample_rrr", "bpt_free", "bpt_sample_rrr_device", "bpt_sample_rrr_jobs",
    "bpt_sample_rrr_noalloc",
    "bpt_max_cover", "Plan", "bpt_plan_create", "bpt_plan_enqueue", "bpt_jobs_plan_create",
    "bpt_jobs_plan_enqueue",
    "bpt_graph_info", "bpt_graph_set_vertex_order",
    "bpt_graph_release_cache",
    "bpt_default_colors", "bpt_tune_colors", "bpt_thr32", "bpt_coin_word", "bpt_start_vertex", "bpt_version",
    "bpt_last_status", "bpt_last_error", "library_path", "load_library",
]

BPT_OK = 0
BPT_EINVAL = -1
BPT_ENOMEM = -2
BPT_EDEVICE = -3
BPT_ERANGE = -4
BPT_EINTERNAL = -5
BPT_PROB_UNIFORM = 0
BPT_PROB_ROW = 1
BPT_PROB_EDGE = 2
BPT_FLAG_UNFUSED = 1
BPT_FLAG_SORTED_STARTS = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbpt.so")
_lib = None

# every symbol include/bpt.h declares
EXPORTED_SYMBOLS = (
    "bpt_create_graph", "bpt_sample_rrr", "bpt_free", "bpt_rrr_num_samples", "bpt_rrr_num_members",
    "bpt_rrr_offsets", "bpt_rrr_vertices", "bpt_last_status", "bpt_last_error", "bpt_sample_rrr_device",
    "bpt_graph_info", "bpt_graph_release_cache", "bpt_default_colors", "bpt_tune_colors", "bpt_thr32",
    "bpt_coin_word", "bpt_start_vertex", "bpt_version", "bpt_sample_rrr_jobs", "bpt_max_cover",
    "bpt_server_create", "bpt_server_submit", "bpt_server_wait", "bpt_server_now", "bpt_server_stats",
    "bpt_server_destroy", "bpt_graph_set_vertex_order", "bpt_plan_create", "bpt_plan_enqueue",
    "bpt_sample_rrr_noalloc", "bpt_jobs_plan_create", "bpt_jobs_plan_enqueue",
)


class _Counters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "samples", "members", "sample_edges", "edge_accesses", "frontier_entries", "philox_blocks",
        "live_coins", "levels", "max_levels", "batches", "traversal_ns", "finalize_ns", "workgroup_size",
        "workgroups")]


class _Job(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("first_sample", ctypes.c_uint64), ("n_samples", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("colors_per_batch", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("d_offsets", ctypes.c_void_p), ("d_vertices", ctypes.c_void_p), ("capacity", ctypes.c_uint64),
                ("total", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved2", ctypes.c_uint32)]


@dataclass
class Job:
    """One request of bpt_sample_rrr_jobs (device buffers: torch tensors or addresses)."""
    graph: "Graph"
    first_sample: int
    n_samples: int
    seed: int
    d_offsets: object
    d_vertices: object
    capacity: int
    colors_per_batch: int = 0
    total: int = 0
    status: int = BPT_OK


class _Request(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("graph", ctypes.c_void_p), ("first_sample", ctypes.c_uint64),
                ("n_samples", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("kind", ctypes.c_uint32),
                ("k", ctypes.c_uint32), ("d_offsets", ctypes.c_void_p), ("d_vertices", ctypes.c_void_p),
                ("capacity", ctypes.c_uint64), ("seeds", ctypes.c_void_p), ("gains", ctypes.c_void_p),
                ("total", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class _ServerInfo(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("served", ctypes.c_uint64), ("busy_s", ctypes.c_double),
                ("sample_s", ctypes.c_double), ("cover_s", ctypes.c_double), ("alloc_s", ctypes.c_double),
                ("resampled", ctypes.c_uint64), ("batch_s", ctypes.c_double), ("lane_slots", ctypes.c_uint32)]


BPT_REQ_SAMPLE = 0
BPT_REQ_SEEDS = 1


class Request:
    """A queued request of a Server; keeps its C struct and output arrays alive."""

    def __init__(self, kind, graph, first_sample, n_samples, seed, k=0, d_offsets=None, d_vertices=None,
                 capacity=0, tag=0):
        self.graph = graph
        self.d_offsets, self.d_vertices = d_offsets, d_vertices
        self.seeds = np.zeros(max(k, 1), dtype=np.uint32)
        self.gains = np.zeros(max(k, 1), dtype=np.uint64)
        self.k = k
        self.c = _Request(tag, graph.handle, first_sample, n_samples, seed, kind, k, _addr(d_offsets),
                          _addr(d_vertices), capacity, self.seeds.ctypes.data, self.gains.ctypes.data,
                          0, 0, 0, 0.0, 0.0, 0.0)

    tag = property(lambda self: int(self.c.tag))
    kind = property(lambda self: int(self.c.kind))
    n_samples = property(lambda self: int(self.c.n_samples))
    status = property(lambda self: int(self.c.status))
    total = property(lambda self: int(self.c.total))
    t_submit = property(lambda self: float(self.c.t_submit))
    t_start = property(lambda self: float(self.c.t_start))
    t_done = property(lambda self: float(self.c.t_done))


class Server:
    """The library's serving loop (bpt_server_*): submit from any thread,
    collect completed requests with wait()."""

    def __init__(self, memory_budget: int = 0, max_jobs_per_launch: int = 0):
        lib = load_library()
        self.handle = lib.bpt_server_create(memory_budget, max_jobs_per_launch)
        if not self.handle:
            raise BptError(BPT_ENOMEM, "bpt_server_create failed")
        self._live = {}

    def submit(self, req: Request) -> Request:
        addr = ctypes.addressof(req.c)
        self._live[addr] = req
        if load_library().bpt_server_submit(self.handle, ctypes.byref(req.c)) != BPT_OK:
            del self._live[addr]
            raise BptError(BPT_EINVAL, "bpt_server_submit rejected the request")
        return req

    def wait(self, timeout: float = 1.0):
        p = load_library().bpt_server_wait(self.handle, timeout)
        return self._live.pop(p, None) if p else None

    def now(self) -> float:
        return float(load_library().bpt_server_now(self.handle))

    def stats(self) -> dict:
        info = _ServerInfo()
        load_library().bpt_server_stats(self.handle, ctypes.byref(info))
        return {name: getattr(info, name) for name, _ in _ServerInfo._fields_}

    def close(self):
        if self.handle:
            load_library().bpt_server_destroy(self.handle)
            self.handle = None


@dataclass
class Counters:
    samples: int = 0
    members: int = 0
    sample_edges: int = 0
    edge_accesses: int = 0
    frontier_entries: int = 0
    philox_blocks: int = 0
    live_coins: int = 0
    levels: int = 0
    max_levels: int = 0
    batches: int = 0
    traversal_ns: int = 0
    finalize_ns: int = 0
    workgroup_size: int = 0
    workgroups: int = 0


class BptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libbpt error {status}: {message}")
        self.status = status


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Loads libbpt.so; raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_2311_10201_amd.build` (there is no CPU fallback)")
    # PyTorch ships its own HIP runtime.  Loading torch first lets libbpt's
    # dependency on libamdhip64.so.7 bind to that same runtime, so device
    # buffers and streams from torch are valid inside libbpt; two runtimes in
    # one process would each try to own the GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    _check_single_hip_runtime()
    u32, u64, i32, vp, cp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_char_p
    sig = {
        "bpt_create_graph": (vp, [u32, u64, vp, vp, vp]),
        "bpt_sample_rrr": (vp, [vp, u64, u32, u64]),
        "bpt_free": (None, [vp]),
        "bpt_rrr_num_samples": (u64, [vp]),
        "bpt_rrr_num_members": (u64, [vp]),
        "bpt_rrr_offsets": (vp, [vp]),
        "bpt_rrr_vertices": (vp, [vp]),
        "bpt_last_status": (i32, []),
        "bpt_last_error": (cp, []),
        "bpt_sample_rrr_device": (i32, [vp, u64, u64, u32, u64, u32, vp, vp, vp, u64,
                                        ctypes.POINTER(u64), ctypes.POINTER(_Counters)]),
        "bpt_sample_rrr_noalloc": (i32, [vp, u64, u64, u32, u64, vp, vp, vp, u64, ctypes.POINTER(u64)]),
        "bpt_sample_rrr_jobs": (i32, [ctypes.POINTER(_Job), u32, vp, ctypes.POINTER(_Counters)]),
        "bpt_plan_create": (vp, [vp, u64, u32, u64]),
        "bpt_plan_enqueue": (i32, [vp, u64, u64, u64, vp, vp, vp, vp, u64, vp]),
        "bpt_jobs_plan_create": (vp, [ctypes.POINTER(_Job), u32, u64]),
        "bpt_jobs_plan_enqueue": (i32, [vp, vp, vp, vp]),
        "bpt_max_cover": (i32, [vp, vp, u64, u32, u32, vp, vp, vp]),
        "bpt_server_create": (vp, [u64, u32]),
        "bpt_server_submit": (i32, [vp, ctypes.POINTER(_Request)]),
        "bpt_server_wait": (vp, [vp, ctypes.c_double]),
        "bpt_server_now": (ctypes.c_double, [vp]),
        "bpt_server_stats": (i32, [vp, ctypes.POINTER(_ServerInfo)]),
        "bpt_server_destroy": (i32, [vp]),
        "bpt_graph_set_vertex_order": (i32, [vp, vp]),
        "bpt_graph_info": (i32, [vp, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u32)]),
        "bpt_graph_release_cache": (i32, [vp]),
        "bpt_default_colors": (u32, [vp, u64]),
        "bpt_tune_colors": (u32, [vp, u64, u64]),
        "bpt_thr32": (u32, [ctypes.c_float]),
        "bpt_coin_word": (u32, [u64, u64, u64]),
        "bpt_start_vertex": (u32, [u64, u64, u32]),
        "bpt_version": (cp, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check_single_hip_runtime():
    try:
        with open("/proc/self/maps") as f:
            paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return
    if len(paths) > 1:
        raise RuntimeError(f"two HIP runtimes are loaded in this process: {sorted(paths)}")


def _raise_last():
    lib = load_library()
    raise BptError(int(lib.bpt_last_status()), lib.bpt_last_error().decode(errors="replace"))


def _addr(x) -> int | None:
    """Device or host address of a torch tensor, numpy array or integer."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    raise TypeError(f"not a stream: {type(s)}")


class Graph:
    """Owns a bpt_graph handle."""

    def __init__(self, handle: int, n: int, m: int):
        self.handle = handle
        self.n = n
        self.m = m

    def close(self):
        if self.handle:
            load_library().bpt_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class RRRResult:
    offsets: np.ndarray   # uint64[n_samples + 1]
    vertices: np.ndarray  # uint32[offsets[-1]]

    def set_of(self, i: int) -> np.ndarray:
        return self.vertices[self.offsets[i]:self.offsets[i + 1]]

    def __len__(self) -> int:
        return len(self.offsets) - 1


def bpt_create_graph(n: int, src, dst, prob) -> Graph:
    lib = load_library()
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    prob = np.ascontiguousarray(prob, dtype=np.float32)
    m = len(src)
    if len(dst) != m or len(prob) != m:
        raise ValueError("src, dst and prob must have equal length")
    h = lib.bpt_create_graph(n, m, _addr(src) if m else None, _addr(dst) if m else None,
                             _addr(prob) if m else None)
    if not h:
        _raise_last()
    return Graph(h, n, m)


def bpt_free(obj) -> None:
    if isinstance(obj, Graph):
        obj.close()
    else:
        load_library().bpt_free(obj)


def bpt_sample_rrr(graph: Graph, n_samples: int, colors_per_batch: int, seed: int) -> RRRResult:
    """Host-resident RRR sets of samples 0 .. n_samples-1 (copied out of the handle)."""
    lib = load_library()
    r = lib.bpt_sample_rrr(graph.handle, n_samples, colors_per_batch, seed)
    if not r:
        _raise_last()
    try:
        ns = int(lib.bpt_rrr_num_samples(r))
        total = int(lib.bpt_rrr_num_members(r))
        off = np.ctypeslib.as_array(ctypes.cast(lib.bpt_rrr_offsets(r), ctypes.POINTER(ctypes.c_uint64)),
                                    shape=(ns + 1,)).copy()
        if total:
            ver = np.ctypeslib.as_array(ctypes.cast(lib.bpt_rrr_vertices(r), ctypes.POINTER(ctypes.c_uint32)),
                                        shape=(total,)).copy()
        else:
            ver = np.zeros(0, dtype=np.uint32)
    finally:
        lib.bpt_free(r)
    return RRRResult(off, ver)


def bpt_sample_rrr_device(graph: Graph, first_sample: int, n_samples: int, colors_per_batch: int, seed: int,
                          flags: int, stream, d_offsets, d_vertices, capacity: int):
    """Samples into caller-owned device buffers.  Returns (status, total, Counters);
    status is BPT_OK or BPT_ERANGE (buffer too small, total reports the need)."""
    lib = load_library()
    total = ctypes.c_uint64(0)
    cnt = _Counters()
    st = lib.bpt_sample_rrr_device(graph.handle, first_sample, n_samples, colors_per_batch, seed, flags,
                                   _stream(stream), _addr(d_offsets), _addr(d_vertices), capacity,
                                   ctypes.byref(total), ctypes.byref(cnt))
    if st not in (BPT_OK, BPT_ERANGE):
        _raise_last()
    return st, int(total.value), Counters(**{k: int(getattr(cnt, k)) for k, _ in _Counters._fields_})


def bpt_sample_rrr_noalloc(graph: Graph, first_sample: int, n_samples: int, colors_per_batch: int, seed: int,
                           stream, d_offsets, d_vertices, capacity: int):
    """bpt_sample_rrr_device without allocation (fused, no flags, no counters):
    the library's fixed per-GPU scratch holds all working memory.  Returns
    (status, total); status is BPT_OK or BPT_ERANGE."""
    lib = load_library()
    total = ctypes.c_uint64(0)
    st = lib.bpt_sample_rrr_noalloc(graph.handle, first_sample, n_samples, colors_per_batch, seed,
                                    _stream(stream), _addr(d_offsets), _addr(d_vertices), capacity,
                                    ctypes.byref(total))
    if st not in (BPT_OK, BPT_ERANGE):
        _raise_last()
    return st, int(total.value)


def bpt_sample_rrr_jobs(jobs, stream=None):
    """Runs all jobs in one fused launch; fills each Job's total and status.
    Returns (status, Counters); status is BPT_OK or BPT_ERANGE (some job's
    capacity below its total)."""
    lib = load_library()
    arr = (_Job * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        arr[i] = _Job(j.graph.handle, j.first_sample, j.n_samples, j.seed, j.colors_per_batch, 0,
                      _addr(j.d_offsets), _addr(j.d_vertices), j.capacity, 0, 0, 0)
    cnt = _Counters()
    st = lib.bpt_sample_rrr_jobs(arr, len(jobs), _stream(stream), ctypes.byref(cnt))
    if st not in (BPT_OK, BPT_ERANGE):
        _raise_last()
    for i, j in enumerate(jobs):
        j.total = int(arr[i].total)
        j.status = int(arr[i].status)
    return st, Counters(**{k: int(getattr(cnt, k)) for k, _ in _Counters._fields_})


class Plan:
    """Owns a bpt_plan handle (a capturable sampling setup of one graph)."""

    def __init__(self, handle: int, graph: Graph, max_samples: int):
        self.handle = handle
        self.graph = graph  # the graph must outlive the plan
        self.max_samples = max_samples

    def close(self):
        if self.handle:
            load_library().bpt_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bpt_plan_create(graph: Graph, max_samples: int, colors_per_batch: int = 0, pool_capacity: int = 0) -> Plan:
    lib = load_library()
    h = lib.bpt_plan_create(graph.handle, max_samples, colors_per_batch, pool_capacity)
    if not h:
        _raise_last()
    return Plan(h, graph, max_samples)


def bpt_plan_enqueue(plan: Plan, first_sample: int, n_samples: int, seed: int, d_params, stream, d_offsets,
                     d_vertices, capacity: int, d_result) -> None:
    """Enqueues one sampling call on `stream` (kernels only; capturable).  The
    outcome {status, members} lands in the int64 device buffer d_result."""
    st = load_library().bpt_plan_enqueue(plan.handle, first_sample, n_samples, seed, _addr(d_params),
                                         _stream(stream), _addr(d_offsets), _addr(d_vertices), capacity,
                                         _addr(d_result))
    if st != BPT_OK:
        _raise_last()


def bpt_jobs_plan_create(jobs, pool_capacity: int = 0) -> Plan:
    """A capturable plan for a fixed list of Jobs (their graphs, sample counts,
    colours and device buffers are fixed; ranges and seeds can change per call)."""
    lib = load_library()
    arr = (_Job * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        arr[i] = _Job(j.graph.handle, j.first_sample, j.n_samples, j.seed, j.colors_per_batch, 0,
                      _addr(j.d_offsets), _addr(j.d_vertices), j.capacity, 0, 0, 0)
    h = lib.bpt_jobs_plan_create(arr, len(jobs), pool_capacity)
    if not h:
        _raise_last()
    plan = Plan(h, jobs[0].graph, 0)
    plan.jobs = list(jobs)  # the buffers must outlive the plan
    return plan


def bpt_jobs_plan_enqueue(plan: Plan, d_params, stream, d_results) -> None:
    """Enqueues one sampling of every job of a multi-job plan (kernels only;
    capturable); {status, members} of job i land in d_results[2i], [2i+1]."""
    st = load_library().bpt_jobs_plan_enqueue(plan.handle, _addr(d_params), _stream(stream), _addr(d_results))
    if st != BPT_OK:
        _raise_last()


def bpt_max_cover(d_offsets, d_vertices, n_sets: int, n: int, k: int, stream=None):
    """Greedy k seeds over device-resident sets.  Returns (seeds, gains) as
    numpy arrays (uint32, uint64)."""
    lib = load_library()
    seeds = np.zeros(max(k, 1), dtype=np.uint32)
    gains = np.zeros(max(k, 1), dtype=np.uint64)
    if lib.bpt_max_cover(_addr(d_offsets), _addr(d_vertices), n_sets, n, k, _stream(stream),
                         seeds.ctypes.data, gains.ctypes.data) != BPT_OK:
        _raise_last()
    return seeds[:k], gains[:k]


def bpt_graph_info(graph: Graph):
    lib = load_library()
    n, m, lay = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
    if lib.bpt_graph_info(graph.handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(lay)) != BPT_OK:
        _raise_last()
    return int(n.value), int(m.value), int(lay.value)


def bpt_graph_set_vertex_order(graph: Graph, rank) -> None:
    """Vertex order for sorted starts (a permutation of 0..n-1), or None."""
    arr = None if rank is None else np.ascontiguousarray(rank, dtype=np.uint32)
    if load_library().bpt_graph_set_vertex_order(graph.handle, None if arr is None else arr.ctypes.data) != BPT_OK:
        _raise_last()


def bpt_graph_release_cache(graph: Graph) -> None:
    if load_library().bpt_graph_release_cache(graph.handle) != BPT_OK:
        _raise_last()


def bpt_default_colors(graph: Graph, n_samples: int) -> int:
    c = int(load_library().bpt_default_colors(graph.handle, n_samples))
    if c == 0:
        _raise_last()
    return c


def bpt_tune_colors(graph: Graph, n_samples: int, seed: int) -> int:
    c = int(load_library().bpt_tune_colors(graph.handle, n_samples, seed))
    if c == 0:
        _raise_last()
    return c


def bpt_thr32(p: float) -> int:
    return int(load_library().bpt_thr32(float(np.float32(p))))


def bpt_coin_word(seed: int, sample: int, edge: int) -> int:
    return int(load_library().bpt_coin_word(seed, sample, edge))


def bpt_start_vertex(seed: int, sample: int, n: int) -> int:
    return int(load_library().bpt_start_vertex(seed, sample, n))


def bpt_version() -> str:
    return load_library().bpt_version().decode()


def bpt_last_status() -> int:
    return int(load_library().bpt_last_status())


def bpt_last_error() -> str:
    return load_library().bpt_last_error().decode(errors="replace")
