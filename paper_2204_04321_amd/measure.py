"""Measurement helpers for the roofline figures.

    python -m paper_2204_04321_amd.measure copy --mib 1024
        a plain device-to-device copy of known size (torch's copy kernel), run under
        `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` to calibrate what those
        counters report for a kernel that reads and writes exactly N bytes;
    python -m paper_2204_04321_amd.measure counters <results.db> <kernel-substring>
        prints, per counter, the average per dispatch of the matching kernels from a
        rocprofv3 database.
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
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_probe(a.mib)
    else:
        print(json.dumps(counters(a.db, a.kernel), indent=1))


if __name__ == "__main__":
    sys.exit(main())
