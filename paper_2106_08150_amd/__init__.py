"""MI355X-native minhash metagenomic classifier (MetaCache-GPU method).

Thin Python binding of the C ABI in ``include/mc.h``: argument marshalling
only; every compute step runs in the HIP kernels of ``libmc.so``. PyTorch is
used by callers for device memory and streams (``tensor.data_ptr()``,
``torch.cuda.current_stream().cuda_stream``).

The library is loaded on first use and an error is raised if it has not been
built (``python -m paper_2106_08150_amd.build`` or ``__graft_entry__.build()``);
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmc.so")

MC_OK = 0
MC_ERR_INVALID_ARG = -1
MC_ERR_CAPACITY = -2
MC_ERR_OOM = -3
MC_ERR_TABLE_FULL = -4
MC_ERR_STATE = -5
MC_ERR_HIP = -6
MC_ERR_LIST = -7
MC_UNCLASSIFIED = 0xFFFFFFFF
MC_MAX_TARGETS = 16383
MC_MAX_WINDOWS = 1 << 18
MC_SUBMIT_PINNED = 1

EXPORTS = [
    "mc_last_error", "mc_db_create", "mc_db_destroy", "mc_db_reserve", "mc_db_add_targets",
    "mc_db_add_targets_device", "mc_db_set_taxonomy", "mc_classify", "mc_classify_ex",
    "mc_db_query_status", "mc_db_get_stats", "mc_db_dump", "mc_db_sketch",
    "mc_db_set_profiling", "mc_db_kernel_times",
    "mc_server_create", "mc_server_submit", "mc_server_add_targets", "mc_server_wait",
    "mc_server_wait_times",
    "mc_server_get_stats", "mc_server_destroy",
    "mc_db_set_launch_config", "mc_db_get_launch_config", "mc_db_autotune",
    "mc_classify_graph_create", "mc_classify_graph_launch", "mc_classify_graph_destroy",
    "mc_release_cached_memory", "mc_set_cached_memory_limit", "mc_db_set_insert_path",
    "mc_db_condense", "mc_db_set_routing", "mc_db_get_routing", "mc_classify_noalloc",
]
NOALLOC_MAX_RECORDS = 1 << 20   # MC_NOALLOC_MAX_RECORDS


class MCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class QueryOpts(C.Structure):
    _fields_ = [("top_m", C.c_uint32), ("min_hits", C.c_uint32), ("hit_diff", C.c_uint32),
                ("insert_size", C.c_uint32), ("paired", C.c_uint32)]


class DbStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "n_targets", "n_windows", "n_pairs_inserted", "n_pairs_stored", "n_buckets",
        "table_bytes", "n_cap_candidates", "probe_sum", "n_rehash", "q_features",
        "q_locations", "q_probes", "n_features", "n_tombstones")] + [
        ("load_factor", C.c_double), ("condensed_bytes", C.c_uint64),
        ("q_large_records", C.c_uint64), ("q_hbm_records", C.c_uint64)]

    def as_dict(self) -> dict:
        return {n: (float(getattr(self, n)) if t is C.c_double else int(getattr(self, n)))
                for n, t in self._fields_}


class InsertPath(C.Structure):
    _fields_ = [("global_insert", C.c_uint32), ("part_mb", C.c_uint32),
                ("slice_shift", C.c_uint32), ("fine_bits", C.c_uint32),
                ("stage_entries", C.c_uint32), ("direct", C.c_uint32),
                ("chunk_slots", C.c_uint64), ("fail_after", C.c_uint32),
                ("reserved", C.c_uint32)]


class LaunchConfig(C.Structure):
    _fields_ = [("list_capacity", C.c_uint32), ("waves_per_block", C.c_uint32),
                ("max_blocks", C.c_uint32)]

    def as_tuple(self):
        return (self.list_capacity, self.waves_per_block, self.max_blocks)


class RouteConfig(C.Structure):
    _fields_ = [("n_classes", C.c_uint32), ("max_windows", C.c_uint32 * 4),
                ("shape", LaunchConfig * 4)]


class ServerOpts(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("memory_budget", C.c_uint64),
                ("staging_bytes", C.c_uint64)]


class BatchTimes(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("admit_ms", "copy_ms", "launch_ms", "finish_ms",
                                          "total_ms", "gpu_kernels_ms", "gpu_copy_back_ms")]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("batches", C.c_uint64), ("records", C.c_uint64), ("bases", C.c_uint64),
                ("additions", C.c_uint64), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("max_ms", C.c_double), ("span_s", C.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    """The loaded libmc.so (raises if it has not been built).

    torch is imported first: its HIP runtime then serves libmc.so too (the
    library's libamdhip64.so.7 dependency resolves to the copy torch loaded).
    Loaded the other way round, the process would hold two HIP runtimes, and
    device pointers and streams from torch would not be valid in the library.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_2106_08150_amd.build)")
        import torch  # noqa: F401  (one HIP runtime: torch's)
        L = C.CDLL(LIB_PATH)
        u32, u64, vp, i32 = C.c_uint32, C.c_uint64, C.c_void_p, C.c_int
        L.mc_last_error.restype = C.c_char_p
        L.mc_last_error.argtypes = []
        L.mc_db_create.restype = vp
        L.mc_db_create.argtypes = [u32, u32, u32, u32]
        L.mc_db_destroy.restype, L.mc_db_destroy.argtypes = i32, [vp]
        L.mc_release_cached_memory.restype, L.mc_release_cached_memory.argtypes = i32, []
        L.mc_set_cached_memory_limit.restype = i32
        L.mc_set_cached_memory_limit.argtypes = [u64]
        L.mc_db_condense.restype, L.mc_db_condense.argtypes = i32, [vp, i32]
        L.mc_db_set_routing.restype = i32
        L.mc_db_set_routing.argtypes = [vp, C.POINTER(RouteConfig)]
        L.mc_db_get_routing.restype = i32
        L.mc_db_get_routing.argtypes = [vp, C.POINTER(RouteConfig)]
        L.mc_db_set_insert_path.restype = i32
        L.mc_db_set_insert_path.argtypes = [vp, C.POINTER(InsertPath)]
        L.mc_db_reserve.restype, L.mc_db_reserve.argtypes = i32, [vp, u64, C.c_double]
        L.mc_db_add_targets.restype = i32
        L.mc_db_add_targets.argtypes = [vp, vp, vp, vp, u32]
        L.mc_db_add_targets_device.restype = i32
        L.mc_db_add_targets_device.argtypes = [vp, vp, vp, vp, u32, vp]
        L.mc_db_set_taxonomy.restype, L.mc_db_set_taxonomy.argtypes = i32, [vp, vp, u32]
        L.mc_classify.restype = i32
        L.mc_classify.argtypes = [vp, vp, vp, u32, vp, vp]
        L.mc_classify_ex.restype = i32
        L.mc_classify_ex.argtypes = [vp, vp, vp, u32, C.POINTER(QueryOpts), vp, vp, vp]
        L.mc_classify_noalloc.restype = i32
        L.mc_classify_noalloc.argtypes = [vp, vp, vp, u32, C.POINTER(QueryOpts), vp, vp, vp]
        L.mc_db_query_status.restype = i32
        L.mc_db_query_status.argtypes = [vp, vp, C.POINTER(u64)]
        L.mc_db_get_stats.restype = i32
        L.mc_db_get_stats.argtypes = [vp, C.POINTER(DbStats)]
        L.mc_db_dump.restype = i32
        L.mc_db_dump.argtypes = [vp, u32, u32, vp, vp, u64, C.POINTER(u64)]
        L.mc_db_sketch.restype = i32
        L.mc_db_sketch.argtypes = [vp, vp, vp, u32, vp, vp, vp]
        L.mc_db_set_profiling.restype, L.mc_db_set_profiling.argtypes = i32, [vp, i32]
        L.mc_db_kernel_times.restype = i32
        L.mc_db_kernel_times.argtypes = [vp, vp, vp]
        L.mc_server_create.restype = vp
        L.mc_server_create.argtypes = [vp, C.POINTER(ServerOpts)]
        L.mc_server_submit.restype = i32
        L.mc_server_submit.argtypes = [vp, vp, vp, u32, C.POINTER(QueryOpts), vp, vp, u32,
                                       C.POINTER(u64)]
        L.mc_server_add_targets.restype = i32
        L.mc_server_add_targets.argtypes = [vp, vp, vp, vp, u32, vp, u32, C.POINTER(u64)]
        L.mc_server_wait.restype = i32
        L.mc_server_wait.argtypes = [vp, u64, C.POINTER(C.c_double)]
        L.mc_server_wait_times.restype = i32
        L.mc_server_wait_times.argtypes = [vp, u64, C.POINTER(BatchTimes)]
        L.mc_server_get_stats.restype = i32
        L.mc_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.mc_server_destroy.restype, L.mc_server_destroy.argtypes = i32, [vp]
        L.mc_db_set_launch_config.restype = i32
        L.mc_db_set_launch_config.argtypes = [vp, C.POINTER(LaunchConfig)]
        L.mc_db_get_launch_config.restype = i32
        L.mc_db_get_launch_config.argtypes = [vp, C.POINTER(LaunchConfig)]
        L.mc_db_autotune.restype = i32
        L.mc_db_autotune.argtypes = [vp, vp, vp, u32, C.POINTER(QueryOpts), vp, vp,
                                     C.POINTER(LaunchConfig), C.POINTER(C.c_double)]
        L.mc_classify_graph_create.restype = vp
        L.mc_classify_graph_create.argtypes = [vp, vp, vp, u32, C.POINTER(QueryOpts), vp, vp, vp]
        L.mc_classify_graph_launch.restype, L.mc_classify_graph_launch.argtypes = i32, [vp, vp]
        L.mc_classify_graph_destroy.restype = i32
        L.mc_classify_graph_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != MC_OK:
        raise MCError(rc, lib().mc_last_error().decode(errors="replace"))
    return rc


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t) -> int:
    """Device address of a torch tensor (must live on a HIP device)."""
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- C ABI ----
def mc_db_create(k: int = 16, window: int = 128, sketch_size: int = 16,
                 max_locations: int = 254) -> int:
    h = lib().mc_db_create(k, window, sketch_size, max_locations)
    if not h:
        raise MCError(MC_ERR_INVALID_ARG, lib().mc_last_error().decode(errors="replace"))
    return h


def mc_db_destroy(db: int) -> None:
    _check(lib().mc_db_destroy(db))


def mc_release_cached_memory() -> None:
    _check(lib().mc_release_cached_memory())


def mc_set_cached_memory_limit(bytes_per_device: int) -> None:
    _check(lib().mc_set_cached_memory_limit(int(bytes_per_device)))


def mc_db_set_insert_path(db: int, **fields) -> None:
    """Test entry point: force the insert path (no fields = automatic)."""
    if not fields:
        _check(lib().mc_db_set_insert_path(db, None))
        return
    p = InsertPath(**fields)
    _check(lib().mc_db_set_insert_path(db, C.byref(p)))


def mc_db_condense(db: int, release_table: bool = False) -> None:
    _check(lib().mc_db_condense(db, int(release_table)))


def mc_db_reserve(db: int, n_pairs: int, load_factor: float = 0.0) -> None:
    _check(lib().mc_db_reserve(db, n_pairs, load_factor))


def mc_db_add_targets(db: int, genomes, lengths, taxon_ids) -> None:
    g = np.ascontiguousarray(genomes, dtype=np.uint8)
    L = np.ascontiguousarray(lengths, dtype=np.uint64)
    t = np.ascontiguousarray(taxon_ids, dtype=np.uint32)
    if L.size != t.size or int(L.sum()) > g.size:
        raise ValueError("lengths/taxon_ids/genomes sizes disagree")
    _check(lib().mc_db_add_targets(db, _np_ptr(g), _np_ptr(L), _np_ptr(t), L.size))


def mc_db_add_targets_device(db: int, genomes_dev, lengths, taxon_ids, stream=None) -> None:
    L = np.ascontiguousarray(lengths, dtype=np.uint64)
    t = np.ascontiguousarray(taxon_ids, dtype=np.uint32)
    if L.size != t.size or int(L.sum()) > genomes_dev.numel():
        raise ValueError("lengths/taxon_ids/genomes sizes disagree")
    _check(lib().mc_db_add_targets_device(db, _dev_ptr(genomes_dev), _np_ptr(L), _np_ptr(t),
                                          L.size, _stream(stream)))


def mc_db_set_taxonomy(db: int, parents) -> None:
    p = np.ascontiguousarray(parents, dtype=np.uint32)
    _check(lib().mc_db_set_taxonomy(db, _np_ptr(p), p.size))


def mc_classify(db: int, reads, offsets, n_reads: int, out_labels, stream=None) -> None:
    _check(lib().mc_classify(db, _dev_ptr(reads), _dev_ptr(offsets), n_reads,
                             _dev_ptr(out_labels), _stream(stream)))


def mc_classify_ex(db: int, reads, offsets, n_records: int, opts: QueryOpts, out_labels,
                   out_top=None, stream=None) -> None:
    top = _dev_ptr(out_top) if out_top is not None else None
    _check(lib().mc_classify_ex(db, _dev_ptr(reads), _dev_ptr(offsets), n_records,
                                C.byref(opts), _dev_ptr(out_labels), top, _stream(stream)))


def mc_classify_noalloc(db: int, reads, offsets, n_records: int, opts: QueryOpts, out_labels,
                        out_top=None, stream=None) -> None:
    """As mc_classify_ex, with the library's fixed per-device scratch (no
    device allocation; at most NOALLOC_MAX_RECORDS records a call)."""
    top = _dev_ptr(out_top) if out_top is not None else None
    _check(lib().mc_classify_noalloc(db, _dev_ptr(reads), _dev_ptr(offsets), n_records,
                                     C.byref(opts), _dev_ptr(out_labels), top, _stream(stream)))


def mc_db_query_status(db: int, stream=None) -> int:
    n = C.c_uint64(0)
    rc = lib().mc_db_query_status(db, _stream(stream), C.byref(n))
    if rc not in (MC_OK, MC_ERR_LIST):
        _check(rc)
    return int(n.value)


def mc_db_get_stats(db: int) -> dict:
    s = DbStats()
    _check(lib().mc_db_get_stats(db, C.byref(s)))
    return s.as_dict()


def mc_db_dump(db: int, lo: int = 0, hi: int = 0xFFFFFFFF) -> tuple[np.ndarray, np.ndarray]:
    n = C.c_uint64(0)
    _check(lib().mc_db_dump(db, lo, hi, None, None, 0, C.byref(n)))
    cap = int(n.value)
    f = np.zeros(max(cap, 1), np.uint32)
    l = np.zeros(max(cap, 1), np.uint32)
    _check(lib().mc_db_dump(db, lo, hi, _np_ptr(f), _np_ptr(l), cap, C.byref(n)))
    return f[:int(n.value)], l[:int(n.value)]


def mc_db_sketch(db: int, seqs_dev, lengths, out_counts, out_features, stream=None) -> None:
    L = np.ascontiguousarray(lengths, dtype=np.uint64)
    _check(lib().mc_db_sketch(db, _dev_ptr(seqs_dev), _np_ptr(L), L.size, _dev_ptr(out_counts),
                              _dev_ptr(out_features), _stream(stream)))


def mc_db_set_profiling(db: int, enable: bool) -> None:
    _check(lib().mc_db_set_profiling(db, int(enable)))


KERNEL_KINDS = ("sketch", "scatter", "insert", "classify")


def mc_db_kernel_times(db: int) -> dict:
    """Summed ms and launch counts per profiled kernel kind since the last call."""
    ms = np.zeros(len(KERNEL_KINDS), np.float64)
    n = np.zeros(len(KERNEL_KINDS), np.uint64)
    _check(lib().mc_db_kernel_times(db, _np_ptr(ms), _np_ptr(n)))
    return {k: {"ms": float(ms[i]), "launches": int(n[i])} for i, k in enumerate(KERNEL_KINDS)}


def mc_db_set_launch_config(db: int, list_capacity: int, waves_per_block: int,
                            max_blocks: int) -> None:
    c = LaunchConfig(list_capacity, waves_per_block, max_blocks)
    _check(lib().mc_db_set_launch_config(db, C.byref(c)))


def mc_db_get_launch_config(db: int) -> tuple:
    c = LaunchConfig()
    _check(lib().mc_db_get_launch_config(db, C.byref(c)))
    return c.as_tuple()


def mc_db_set_routing(db: int, max_windows, shapes) -> None:
    """Size classes: max_windows of every class but the last (ascending) and one
    (list capacity, waves per workgroup, largest grid) shape per class."""
    shapes = list(shapes)
    r = RouteConfig()
    r.n_classes = len(shapes)
    for i, m in enumerate(max_windows):
        r.max_windows[i] = m
    for i, sh in enumerate(shapes):
        r.shape[i] = LaunchConfig(*sh)
    _check(lib().mc_db_set_routing(db, C.byref(r)))


def mc_db_get_routing(db: int) -> tuple:
    r = RouteConfig()
    _check(lib().mc_db_get_routing(db, C.byref(r)))
    n = r.n_classes
    return ([r.max_windows[i] for i in range(n - 1)], [r.shape[i].as_tuple() for i in range(n)])


def mc_db_autotune(db: int, reads, offsets, n_records: int, opts: QueryOpts, out_labels,
                   stream=None) -> tuple:
    c, ms = LaunchConfig(), C.c_double(0)
    _check(lib().mc_db_autotune(db, _dev_ptr(reads), _dev_ptr(offsets), n_records,
                                C.byref(opts), _dev_ptr(out_labels), _stream(stream),
                                C.byref(c), C.byref(ms)))
    return c.as_tuple(), ms.value


class ClassifyGraph:
    """One classification call captured into a HIP graph (fixed device buffers)."""

    def __init__(self, db: int, reads, offsets, n_records: int, opts: QueryOpts, out_labels,
                 out_top=None, stream=None):
        self._keep = (reads, offsets, out_labels, out_top)
        top = _dev_ptr(out_top) if out_top is not None else None
        self.h = lib().mc_classify_graph_create(db, _dev_ptr(reads), _dev_ptr(offsets),
                                                n_records, C.byref(opts), _dev_ptr(out_labels),
                                                top, _stream(stream))
        if not self.h:
            raise MCError(MC_ERR_HIP, lib().mc_last_error().decode(errors="replace"))

    def launch(self, stream=None):
        _check(lib().mc_classify_graph_launch(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().mc_classify_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mc_server_create(db: int, slots: int = 4, memory_budget: int = 0,
                     staging_bytes: int = 0) -> int:
    o = ServerOpts(slots, memory_budget, staging_bytes)
    h = lib().mc_server_create(db, C.byref(o))
    if not h:
        raise MCError(MC_ERR_INVALID_ARG, lib().mc_last_error().decode(errors="replace"))
    return h


def mc_server_destroy(srv: int) -> None:
    _check(lib().mc_server_destroy(srv))


def mc_server_get_stats(srv: int) -> dict:
    s = ServerStats()
    _check(lib().mc_server_get_stats(srv, C.byref(s)))
    return s.as_dict()


# ------------------------------------------------------------ wrapper ----
class Database:
    """Owning wrapper of an ``mc_db`` handle with torch-friendly helpers."""

    def __init__(self, k: int = 16, window: int = 128, sketch_size: int = 16,
                 max_locations: int = 254):
        self.k, self.window, self.sketch_size, self.max_locations = (
            k, window, sketch_size, max_locations)
        self.h = mc_db_create(k, window, sketch_size, max_locations)

    def close(self):
        if getattr(self, "h", None):
            mc_db_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, n_pairs: int, load_factor: float = 0.0):
        mc_db_reserve(self.h, n_pairs, load_factor)

    def condense(self, release_table: bool = False):
        mc_db_condense(self.h, release_table)

    def add_targets(self, genomes, lengths, taxon_ids):
        """Host arrays (numpy) or a device uint8 tensor for ``genomes``."""
        if hasattr(genomes, "is_cuda") and genomes.is_cuda:
            mc_db_add_targets_device(self.h, genomes, lengths, taxon_ids)
        else:
            mc_db_add_targets(self.h, genomes, lengths, taxon_ids)

    def set_taxonomy(self, parents):
        mc_db_set_taxonomy(self.h, parents)

    def stats(self) -> dict:
        return mc_db_get_stats(self.h)

    def dump(self, lo: int = 0, hi: int = 0xFFFFFFFF):
        return mc_db_dump(self.h, lo, hi)

    def classify(self, reads, offsets, n_records: int | None = None, top_m: int = 4,
                 min_hits: int = 4, hit_diff: int = 0, insert_size: int = 0,
                 paired: bool = False, with_top: bool = False, stream=None):
        """Device tensors in, device tensors out (labels int32 viewed as u32)."""
        import torch
        if n_records is None:
            n_records = (offsets.numel() - 1) // (2 if paired else 1)
        dev = reads.device
        labels = torch.empty(max(n_records, 1), dtype=torch.int32, device=dev)
        top = (torch.empty((max(n_records, 1), top_m, 3), dtype=torch.int32, device=dev)
               if with_top else None)
        opts = QueryOpts(top_m, min_hits, hit_diff, insert_size, int(paired))
        mc_classify_ex(self.h, reads, offsets, n_records, opts, labels, top, stream)
        return (labels[:n_records], top[:n_records] if top is not None else None)


class Server:
    """Persistent request loop over a Database (host buffers in and out).

    ``submit`` queues a batch and returns a ticket at once; ``wait`` returns the
    batch's labels (and top hits) with its latency. ``add_targets`` queues an
    on-demand genome addition, ordered with the batches.
    """

    def __init__(self, db: Database, slots: int = 4, memory_budget: int = 0,
                 staging_bytes: int = 0):
        self.db = db
        self.h = mc_server_create(db.h, slots, memory_budget, staging_bytes)
        self._jobs = {}

    def submit(self, reads_text, offsets, paired: bool = False, top_m: int = 4,
               min_hits: int = 4, hit_diff: int = 0, insert_size: int = 0,
               with_top: bool = False) -> int:
        """reads_text: numpy uint8 array, or a pinned CPU torch uint8 tensor (copied to
        the device directly)."""
        pinned = hasattr(reads_text, "is_pinned") and reads_text.is_pinned()
        if pinned:
            text, text_ptr = reads_text, C.c_void_p(reads_text.data_ptr())
        else:
            text = np.ascontiguousarray(reads_text, dtype=np.uint8)
            text_ptr = _np_ptr(text)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = (off.size - 1) // (2 if paired else 1)
        labels = np.empty(max(n, 1), np.uint32)
        top = np.empty((max(n, 1), top_m, 3), np.uint32) if with_top else None
        opts = QueryOpts(top_m, min_hits, hit_diff, insert_size, int(paired))
        t = C.c_uint64(0)
        _check(lib().mc_server_submit(self.h, text_ptr, _np_ptr(off), n, C.byref(opts),
                                      _np_ptr(labels), _np_ptr(top) if top is not None else None,
                                      MC_SUBMIT_PINNED if pinned else 0, C.byref(t)))
        self._jobs[t.value] = (text, off, labels, top, n)   # keep buffers alive
        return t.value

    def add_targets(self, genomes, lengths, taxon_ids, parents=None) -> int:
        g = np.ascontiguousarray(genomes, dtype=np.uint8)
        L = np.ascontiguousarray(lengths, dtype=np.uint64)
        x = np.ascontiguousarray(taxon_ids, dtype=np.uint32)
        p = np.ascontiguousarray(parents, dtype=np.uint32) if parents is not None else None
        t = C.c_uint64(0)
        _check(lib().mc_server_add_targets(self.h, _np_ptr(g), _np_ptr(L), _np_ptr(x), L.size,
                                           _np_ptr(p) if p is not None else None,
                                           0 if p is None else p.size, C.byref(t)))
        self._jobs[t.value] = ("add", g, L, x, p)   # the server reads them in place
        return t.value

    def wait(self, ticket: int):
        """(labels, top hits, latency ms) of a batch; (None, None, ms) for an addition."""
        labels, top, times = self.wait_times(ticket)
        return labels, top, times["total_ms"]

    def wait_times(self, ticket: int):
        """As wait, with the latency split by stage (mc_batch_times) as a dict."""
        t = BatchTimes()
        rc = lib().mc_server_wait_times(self.h, ticket, C.byref(t))
        job = self._jobs.pop(ticket, None)
        _check(rc)
        if job is None or isinstance(job[0], str):   # an addition
            return None, None, t.as_dict()
        _, _, labels, top, n = job
        return labels[:n], (top[:n] if top is not None else None), t.as_dict()

    def stats(self) -> dict:
        return mc_server_get_stats(self.h)

    def close(self):
        if getattr(self, "h", None):
            mc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
