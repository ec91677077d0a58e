"""CPU oracle of the minhash classifier (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``libmc_oracle.so`` (plain C++,
built from ``mc_oracle.cpp``) with numpy-friendly helpers and shares no code
with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mc_oracle.cpp")
LIB = os.path.join(HERE, "libmc_oracle.so")

UNCLASSIFIED = 0xFFFFFFFF

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        u32, u64, vp = C.c_uint32, C.c_uint64, C.c_void_p
        L.orc_h1.argtypes, L.orc_h1.restype = [u32], u32
        L.orc_num_windows.argtypes, L.orc_num_windows.restype = [u64, u32, u32], u64
        L.orc_sws.argtypes, L.orc_sws.restype = [u64, u32, u32], u32
        L.orc_kmers.argtypes, L.orc_kmers.restype = [vp, u64, u32, vp, vp], None
        L.orc_bottom_s.argtypes, L.orc_bottom_s.restype = [vp, u32, u32, vp], u32
        L.orc_sketch_windows.argtypes = [vp, u64, u32, u32, u32, vp, vp]
        L.orc_sketch_windows.restype = u64
        L.orc_db_create.argtypes, L.orc_db_create.restype = [u32, u32, u32, u32], vp
        L.orc_db_destroy.argtypes, L.orc_db_destroy.restype = [vp], None
        L.orc_db_set_filter.argtypes, L.orc_db_set_filter.restype = [vp, vp, u64], None
        L.orc_db_set_filter_range.argtypes = [vp, u32, u32]
        L.orc_db_set_filter_range.restype = None
        L.orc_db_add_targets.argtypes = [vp, vp, vp, vp, u32, C.c_int]
        L.orc_db_add_targets.restype = C.c_int
        L.orc_db_add_targets_stop_at_cap.argtypes = [vp, vp, vp, vp, u32]
        L.orc_db_add_targets_stop_at_cap.restype = C.c_int
        L.orc_db_set_taxonomy.argtypes, L.orc_db_set_taxonomy.restype = [vp, vp, u32], None
        L.orc_db_num_pairs.argtypes, L.orc_db_num_pairs.restype = [vp], u64
        L.orc_db_num_features.argtypes, L.orc_db_num_features.restype = [vp], u64
        L.orc_db_dump.argtypes, L.orc_db_dump.restype = [vp, vp, vp], None
        L.orc_lca.argtypes, L.orc_lca.restype = [vp, u32, u32], u32
        L.orc_decide.argtypes = [vp, vp, vp, u32, u32, u32]
        L.orc_decide.restype = u32
        L.orc_classify.argtypes = [vp, vp, vp, u64, u64, u32, u32, u32, u32, u32, vp, vp,
                                   C.c_int]
        L.orc_classify.restype = C.c_int
        L.orc_query_features.argtypes = [u32, u32, u32, vp, vp, u64, u64, u32, vp, u64]
        L.orc_query_features.restype = u64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _bytes(seq) -> np.ndarray:
    if isinstance(seq, (bytes, bytearray)):
        return np.frombuffer(bytes(seq), dtype=np.uint8)
    if isinstance(seq, str):
        return np.frombuffer(seq.encode(), dtype=np.uint8)
    return np.ascontiguousarray(seq, dtype=np.uint8)


def h1(x: int) -> int:
    return int(lib().orc_h1(x))


def num_windows(length: int, k: int, w: int) -> int:
    return int(lib().orc_num_windows(length, k, w))


def sws(F: int, k: int, w: int) -> int:
    return int(lib().orc_sws(F, k, w))


def kmers(seq, k: int) -> tuple[np.ndarray, np.ndarray]:
    s = _bytes(seq)
    n = max(0, s.size - k + 1)
    canon = np.zeros(n, np.uint32)
    valid = np.zeros(n, np.uint8)
    lib().orc_kmers(_p(s), s.size, k, _p(canon), _p(valid))
    return canon, valid.astype(bool)


def bottom_s(values, s: int) -> list[int]:
    v = np.ascontiguousarray(values, dtype=np.uint32)
    out = np.zeros(max(1, s), np.uint32)
    n = lib().orc_bottom_s(_p(v), v.size, s, _p(out))
    return [int(x) for x in out[:n]]


def sketch_windows(seq, k: int, w: int, s: int) -> list[list[int]]:
    t = _bytes(seq)
    nw = num_windows(t.size, k, w)
    counts = np.zeros(max(1, nw), np.uint32)
    feats = np.zeros(max(1, nw * s), np.uint32)
    lib().orc_sketch_windows(_p(t), t.size, k, w, s, _p(counts), _p(feats))
    return [[int(x) for x in feats[j * s:j * s + counts[j]]] for j in range(nw)]


def query_features(reads_text, offsets, k: int, w: int, s: int, first: int, count: int,
                   paired: bool) -> np.ndarray:
    t = _bytes(reads_text)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = lib().orc_query_features(k, w, s, _p(t), _p(off), first, count, int(paired), None, 0)
    out = np.zeros(max(1, n), np.uint32)
    lib().orc_query_features(k, w, s, _p(t), _p(off), first, count, int(paired), _p(out), n)
    return out[:n]


class OracleDB:
    """std::multimap index with the paper's cap rule; per-read brute-force scoring."""

    def __init__(self, k: int = 16, window: int = 128, sketch_size: int = 16,
                 max_locations: int = 254):
        self.k, self.w, self.s, self.cap = k, window, sketch_size, max_locations
        self.h = lib().orc_db_create(k, window, sketch_size, max_locations)
        if not self.h:
            raise ValueError("invalid oracle parameters")

    def close(self):
        if self.h:
            lib().orc_db_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_filter(self, feats):
        f = np.ascontiguousarray(feats, dtype=np.uint32)
        lib().orc_db_set_filter(self.h, _p(f), f.size)

    def set_filter_range(self, lo: int, hi: int):
        lib().orc_db_set_filter_range(self.h, lo, hi)

    def add_targets(self, text, lengths, taxa, threads: int = 1, stop_at_cap: bool = False):
        t = _bytes(text)
        L = np.ascontiguousarray(lengths, dtype=np.uint64)
        X = np.ascontiguousarray(taxa, dtype=np.uint32)
        if stop_at_cap:
            rc = lib().orc_db_add_targets_stop_at_cap(self.h, _p(t), _p(L), _p(X), L.size)
        else:
            rc = lib().orc_db_add_targets(self.h, _p(t), _p(L), _p(X), L.size, threads)
        if rc:
            raise ValueError(f"oracle add_targets failed ({rc})")

    def set_taxonomy(self, parents):
        p = np.ascontiguousarray(parents, dtype=np.uint32)
        lib().orc_db_set_taxonomy(self.h, _p(p), p.size)

    @property
    def num_pairs(self) -> int:
        return int(lib().orc_db_num_pairs(self.h))

    @property
    def num_features(self) -> int:
        return int(lib().orc_db_num_features(self.h))

    def dump(self) -> tuple[np.ndarray, np.ndarray]:
        n = self.num_pairs
        f = np.zeros(max(1, n), np.uint32)
        l = np.zeros(max(1, n), np.uint32)
        lib().orc_db_dump(self.h, _p(f), _p(l))
        return f[:n], l[:n]

    def lca(self, a: int, b: int) -> int:
        return int(lib().orc_lca(self.h, a, b))

    def decide(self, targets, scores, min_hits: int = 4, hit_diff: int = 0) -> int:
        t = np.ascontiguousarray(targets, dtype=np.uint32)
        s = np.ascontiguousarray(scores, dtype=np.uint32)
        return int(lib().orc_decide(self.h, _p(t), _p(s), t.size, min_hits, hit_diff))

    def classify(self, reads_text, offsets, paired: bool = False, top_m: int = 4,
                 min_hits: int = 4, hit_diff: int = 0, insert_size: int = 0,
                 first: int = 0, count: int | None = None, threads: int = 1):
        t = _bytes(reads_text)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        n_rec = (off.size - 1) // (2 if paired else 1)
        if count is None:
            count = n_rec - first
        labels = np.zeros(max(1, count), np.uint32)
        top = np.zeros((max(1, count), top_m, 3), np.uint32)
        rc = lib().orc_classify(self.h, _p(t), _p(off), first, count, top_m, min_hits,
                                hit_diff, insert_size, int(paired), _p(labels), _p(top),
                                threads)
        if rc:
            raise ValueError(f"oracle classify failed ({rc})")
        return labels[:count], top[:count]
