"""Measured memory-system ceilings of the current GPU (roofline denominators).

Runs the probes of ``libmc_peaks.so``: streaming copy, random 64-bit CAS,
random 128-byte and 64-byte line reads, and the read-line-then-CAS pattern of
a table insert, each on a working set of a given size.

    python -m paper_2106_08150_amd.peaks [--table-gb 16] [--json]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmc_peaks.so")

KINDS = {"copy_gbs": 0, "cas_gops": 1, "line128_glines": 2, "line64_glines": 3,
         "read_cas_ginserts": 4}


def lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP libraries first")
    L = C.CDLL(LIB_PATH)
    L.mcp_measure.restype = C.c_int
    L.mcp_measure.argtypes = [C.c_int, C.c_uint64, C.c_uint64, C.c_int,
                              C.POINTER(C.c_double), C.POINTER(C.c_double)]
    return L


def measure(kind: str, table_bytes: int, n_ops: int = 1 << 28, reps: int = 3) -> dict:
    rate, ms = C.c_double(0), C.c_double(0)
    rc = lib().mcp_measure(KINDS[kind], int(table_bytes), int(n_ops), reps, C.byref(rate),
                           C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"mcp_measure({kind}) failed with {rc}")
    return {"rate": rate.value, "ms": ms.value, "table_bytes": int(table_bytes),
            "n_ops": int(n_ops)}


def all_peaks(table_gb: float = 16.0, small_mb: float = 64.0) -> dict:
    big = int(table_gb * (1 << 30))
    small = int(small_mb * (1 << 20))
    out = {"copy_gbs": measure("copy_gbs", big // 4, reps=5)}
    for name in ("cas_gops", "line128_glines", "line64_glines", "read_cas_ginserts"):
        out[name] = measure(name, big)
        out[name + "_small"] = measure(name, small)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--table-gb", type=float, default=16.0)
    ap.add_argument("--small-mb", type=float, default=64.0)
    ap.add_argument("--copy-only", type=float, default=0.0,
                    help="run only a copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_only:
        r = measure("copy_gbs", int(args.copy_only * (1 << 30)), reps=1)
        print(json.dumps(r))
        return
    r = all_peaks(args.table_gb, args.small_mb)
    for k, v in r.items():
        print(f"{k:28s} {v['rate']:10.2f}  ({v['ms']:.3f} ms, {v['table_bytes'] / 2**20:.0f} MiB)",
              file=sys.stderr)
    print(json.dumps(r))


if __name__ == "__main__":
    main()
