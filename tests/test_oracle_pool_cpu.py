"""The whole-mesh comparison harness (tests/oracle_pool.py) on the CPU: fed the oracle's own
assembly it reports rounding-level errors and an exact pattern; a value planted in the
"GPU" arrays is found on its row; the spawn pool runs it in separate processes."""
import multiprocessing as mp
import os
import shutil

import numpy as np
import pytest
import scipy.sparse as sp

import oracle_pool
from oracle import fo_oracle as fo


def small_cap():
    from fo_inputs.meshgen import ExtrudedMesh, _dome_fields, dome_velocity, ellipse_mesh
    rng = np.random.default_rng(31)
    a, b = 50e3, 30e3
    xy, tri = ellipse_mesh(160, a, b, rng)
    s, H, beta = _dome_fields(xy, a, b, rng, 2000.0, 300.0, 500.0, 1.0, 15e3, 60e3)
    m = ExtrudedMesh("wedge", xy, tri, s, H, beta, np.linspace(0, 1, 5), A=1e-16)
    return m, dome_velocity(m, a, b, rng, 150.0)


def _write(m, U, plant=None):
    R, J = fo.assemble(m, U)
    vals = J.data.copy()
    if plant is not None:
        vals[plant] *= 1.0 + 1e-9
    d = oracle_pool.scratch_dir()
    files = {}
    for k, a in (("R", R), ("J", vals), ("J32", vals.astype(np.float32)),
                 ("rowptr", J.indptr.astype(np.int64)), ("colidx", J.indices.astype(np.int32))):
        files[k] = os.path.join(d, k + ".npy")
        np.save(files[k], a)
    return d, files, J


def test_harness_reports_oracle_against_itself():
    m, U = small_cap()
    d, files, J = _write(m, U)
    try:
        oracle_pool.init_worker(small_cap, files)
        res = [oracle_pool.compare_columns(b) for b in oracle_pool.column_ranges(m.n_verts, 5)]
        tot = oracle_pool.merge(res)
    finally:
        shutil.rmtree(d)
    assert tot["pattern_ok"] and tot["rows"] == m.n_dofs
    # the oracle against itself over cell subsets: only summation order differs
    for key in ("R", "J"):
        assert tot[key]["term"] <= 1e-14 and tot[key]["plain"] <= 1e-14, (key, tot[key])
    assert 1e-9 < tot["J32"]["plain"] < 1e-6        # the FP32 rounding of the values


def test_harness_finds_a_planted_value():
    m, U = small_cap()
    J = fo.assemble(m, U)[1]
    k = int(np.argmax(np.abs(J.data)) // 2 + 7)
    row = int(np.searchsorted(J.indptr, k, side="right") - 1)
    d, files, _ = _write(m, U, plant=k)
    try:
        oracle_pool.init_worker(small_cap, files)
        res = [oracle_pool.compare_columns(b) for b in oracle_pool.column_ranges(m.n_verts, 3)]
        tot = oracle_pool.merge(res)
    finally:
        shutil.rmtree(d)
    assert tot["J"]["term_row"] == row
    assert tot["J"]["term"] > 1e-11


def test_harness_in_spawned_processes():
    m, U = small_cap()
    d, files, _ = _write(m, U)
    try:
        with mp.get_context("spawn").Pool(2, initializer=oracle_pool.init_worker,
                                          initargs=(small_cap, files)) as pool:
            res = pool.map(oracle_pool.compare_columns, oracle_pool.column_ranges(m.n_verts, 4))
    finally:
        shutil.rmtree(d)
    tot = oracle_pool.merge(res)
    assert tot["pattern_ok"] and tot["J"]["term"] <= 1e-14
