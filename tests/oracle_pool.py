"""Oracle comparison of a whole assembled mesh, split over host processes (test helper).

The parent writes the GPU residual, Jacobian values and CSR pattern to .npy files; each
worker takes a range of vertex columns, assembles the oracle residual and Jacobian rows of
those columns from the cells around them (with both parity scales), and compares them with
the memory-mapped GPU values.  Imports neither torch nor the HIP library, so workers
started with the "spawn" method never touch the device.
"""
from __future__ import annotations

import os

import numpy as np

_STATE = {}


def init_worker(mesh_factory, files):
    """Pool initializer: build the seeded mesh once per worker and map the GPU outputs.  A
    mesh with ocean fronts has its front-face terms (independent of U) formed once here, and
    the oracle's front_face_terms returns them for this mesh instead of recomputing them for
    every column range."""
    from threadpoolctl import threadpool_limits

    from oracle import fo_oracle as fo
    threadpool_limits(limits=1)
    m, U = mesh_factory()
    if fo._has_front(m):
        terms = fo.front_face_terms(m)
        original = fo.front_face_terms
        fo.front_face_terms = lambda mesh: terms if mesh is m else original(mesh)
    _STATE.update(m=m, U=U, **{k: np.load(v, mmap_mode="r") for k, v in files.items()})


def compare_columns(bounds):
    """Errors of the GPU rows of vertex columns [v0, v1) on the three parity scales.

    Returns a dict with, for R, J (FP64) and J32 (FP32 values), the maxima of the per-term
    row-scaled error, the element-level row-scaled error and the absolute difference, the
    rows where they peak, the row maxima of |R| and |J| (for norm-wise errors), and whether
    the CSR columns of every row equal the oracle's."""
    from oracle import fo_oracle as fo
    v0, v1 = bounds
    m, U = _STATE["m"], _STATE["U"]
    L1 = m.n_layers + 1
    r0, r1 = 2 * v0 * L1, 2 * v1 * L1
    nodes = np.arange(v0 * L1, v1 * L1)
    cells = fo.cells_touching_nodes(m, nodes)
    R_o, J_o = fo.assemble(m, U, cells=cells)
    SR, SJ = fo.abs_terms(m, U, cells=cells)
    ER, EJ = fo.element_scales(m, U, cells=cells)
    R_o, SR, ER = R_o[r0:r1], SR[r0:r1], ER[r0:r1]
    J_o, SJ = J_o[r0:r1], SJ[r0:r1]
    EJ = EJ[r0:r1]
    sj_row = np.asarray(SJ.max(axis=1).todense()).ravel()
    rowptr = _STATE["rowptr"]
    lo, hi = int(rowptr[r0]), int(rowptr[r1])
    cols = np.asarray(_STATE["colidx"][lo:hi], dtype=np.int64)
    rp = np.asarray(rowptr[r0:r1 + 1], dtype=np.int64) - lo
    pattern_ok = bool(np.array_equal(rp, J_o.indptr) and np.array_equal(cols, J_o.indices))
    rows = np.repeat(np.arange(r1 - r0), np.diff(J_o.indptr))
    out = {"pattern_ok": pattern_ok, "rows": r1 - r0, "cells": int(cells.shape[0]),
           "R_ref_max": float(np.abs(R_o).max()), "J_ref_max": float(np.abs(J_o.data).max())}
    dR = np.abs(np.asarray(_STATE["R"][r0:r1]) - R_o)
    _put(out, "R", dR / SR, dR / ER, dR, r0)
    for key in ("J", "J32"):
        vals = np.asarray(_STATE[key][lo:hi], dtype=np.float64)
        d = np.abs(vals - J_o.data) if pattern_ok else np.full(J_o.data.shape, np.inf)
        dmax = np.zeros(r1 - r0)
        np.maximum.at(dmax, rows, d)
        _put(out, key, dmax / sj_row, dmax / EJ, dmax, r0)
    return out


def _put(out, key, term, elem, absd, r0):
    out[key] = {"term": float(term.max()), "term_row": int(r0 + term.argmax()),
                "elem": float(elem.max()), "elem_row": int(r0 + elem.argmax()),
                "abs": float(absd.max())}


def merge(results):
    """Whole-mesh maxima from the per-range results of compare_columns."""
    tot = {"pattern_ok": all(r["pattern_ok"] for r in results),
           "rows": sum(r["rows"] for r in results),
           "R_ref_max": max(r["R_ref_max"] for r in results),
           "J_ref_max": max(r["J_ref_max"] for r in results)}
    for key in ("R", "J", "J32"):
        t = {}
        for f in ("term", "elem"):
            best = max(results, key=lambda r: r[key][f])
            t[f] = best[key][f]
            t[f + "_row"] = best[key][f + "_row"]
        t["plain"] = max(r[key]["abs"] for r in results) / tot["R_ref_max" if key == "R" else "J_ref_max"]
        tot[key] = t
    return tot


def icesheet_tetrahedra():
    """The ice-sheet configuration extruded to tetrahedra (3 per prism)."""
    from fo_inputs import config1_icesheet
    m, U = config1_icesheet()
    return m.with_fields(elem="tet"), U


def marine_bench_sheet():
    """The marine ice sheet the benchmark assembles (125k base points, 10 layers)."""
    from fo_inputs import marine_sheet
    return marine_sheet(seed=7, n_points=125_000, n_layers=10, a=600e3, b=350e3)


def column_ranges(n_verts, n_chunks):
    step = (n_verts + n_chunks - 1) // n_chunks
    return [(v, min(v + step, n_verts)) for v in range(0, n_verts, step)]


def scratch_dir():
    """A private directory for the exchanged arrays (in memory where /dev/shm exists)."""
    import tempfile
    base = "/dev/shm" if os.path.isdir("/dev/shm") and os.access("/dev/shm", os.W_OK) else None
    return tempfile.mkdtemp(prefix="fo_parity_", dir=base)
