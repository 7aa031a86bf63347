"""Measurement helpers for the roofline figures.

    python -m paper_2204_04321_amd.measure copy --mib 1024
        a plain device-to-device copy of known size (torch's copy kernel), run under
        `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` to calibrate what those
        counters report for a kernel that reads and writes exactly N bytes;
    python -m paper_2204_04321_amd.measure counters <results.db> <kernel-substring>
        prints, per counter, the average per dispatch of the matching kernels from a
        rocprofv3 database;
    python -m paper_2204_04321_amd.measure peaks
        the FP64 vector FMA rate and the streaming copy bandwidth this device reaches
        (libfo_probe.so), next to the published MI355X figures.
"""
from __future__ import annotations

import argparse
import json
import sqlite3
import sys


def copy_probe(mib: int, reps: int = 5) -> None:
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 8, "reps": reps}))


SPEC_FP64_TFLOPS = 78.6
SPEC_HBM_GBS = 8000.0


def peaks(fma_iters: int = 4096, copy_mib: int = 4096, reps: int = 10) -> dict:
    """Measured FP64 FMA rate (TFLOP/s) and copy bandwidth (GB/s, bytes read + written)."""
    import ctypes
    import os

    import torch
    lib = ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfo_probe.so"))
    lib.fo_probe_fma64.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.fo_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    lib.fo_probe_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.fo_probe_write.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    blocks = n_cu * 32
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    t = timed(lambda: lib.fo_probe_fma64(blocks, fma_iters, ctypes.c_void_p(out.data_ptr()), s))
    fma_tflops = 2.0 * 16 * fma_iters * blocks * 256 / t / 1e12
    n = copy_mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    by_grid, rd, wr = {}, {}, {}
    part = torch.empty(n_cu * 256 * 256, dtype=torch.float64, device="cuda")
    for per_cu in (8, 16, 32, 64, 128, 256):
        g = n_cu * per_cu
        t = timed(lambda: lib.fo_probe_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, g, s))
        by_grid[per_cu] = 2.0 * n * 8 / t / 1e9
        t = timed(lambda: lib.fo_probe_read(ctypes.c_void_p(a.data_ptr()), n, g, ctypes.c_void_p(part.data_ptr()), s))
        rd[per_cu] = n * 8 / t / 1e9
        t = timed(lambda: lib.fo_probe_write(ctypes.c_void_p(b.data_ptr()), n, 1.0, g, s))
        wr[per_cu] = n * 8 / t / 1e9
    copy_gbs = max(by_grid.values())
    return {"fp64_fma_tflops": fma_tflops, "fp64_spec_tflops": SPEC_FP64_TFLOPS,
            "copy_gbs": copy_gbs, "copy_gbs_by_blocks_per_cu": by_grid,
            "read_gbs": max(rd.values()), "read_gbs_by_blocks_per_cu": rd,
            "write_gbs": max(wr.values()), "write_gbs_by_blocks_per_cu": wr, "hbm_spec_gbs": SPEC_HBM_GBS,
            "copy_bytes_each_way": n * 8,
            "compute_units": n_cu}


def counters(db: str, kernel: str) -> dict:
    con = sqlite3.connect(db)
    cols = [d[0] for d in con.execute("select * from counters_collection limit 1").description]
    rows = con.execute("select * from counters_collection").fetchall()
    out: dict = {}
    ci = {c: i for i, c in enumerate(cols)}
    name_col = "kernel_name" if "kernel_name" in ci else "name"
    for r in rows:
        if kernel not in str(r[ci[name_col]]):
            continue
        cname = r[ci["counter_name"]]
        val = float(r[ci["value"]])
        did = r[ci["dispatch_id"]] if "dispatch_id" in ci else None
        d = out.setdefault(cname, {})
        d[did] = d.get(did, 0.0) + val
    return {k: sum(v.values()) / len(v) for k, v in out.items()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    k = sub.add_parser("counters")
    k.add_argument("db")
    k.add_argument("kernel")
    sub.add_parser("peaks")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_probe(a.mib)
    elif a.cmd == "peaks":
        print(json.dumps(peaks(), indent=1))
    else:
        print(json.dumps(counters(a.db, a.kernel), indent=1))


if __name__ == "__main__":
    sys.exit(main())
