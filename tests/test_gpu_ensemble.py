"""Batched ensemble (uneven meshes, per-member beta and A) in one persistent launch:
every member equals its own single-mesh assembly bit for bit, and the oracle to 1e-12."""
import numpy as np
import pytest
import torch

from fo_inputs import ensemble_member
from oracle import fo_oracle as fo

from gpu_util import gpu_jacobian, gpu_mesh, parity_errors, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def members():
    out = []
    for i in range(7):
        m, U = ensemble_member(i, n_layers=10 - (i % 3), tri_range=(300, 5000))
        out.append((m, U, gpu_mesh(m)))
    print("\n[ensemble] cells per member:", [M.n_cells for _, _, M in out], flush=True)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ensemble_equals_single_mesh(members, dtype):
    from paper_2204_04321_amd.api import Ensemble
    E = Ensemble([M for _, _, M in members])
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Us = [to_dev(U) for _, U, _ in members]
    Rs = [torch.full((M.n_dofs,), float("nan"), dtype=torch.float64, device="cuda") for _, _, M in members]
    Js = [torch.full((M.nnz,), float("nan"), dtype=tdt, device="cuda") for _, _, M in members]
    E.assemble(Us, Rs, Js, dtype=dtype)
    E.assemble(Us, Rs, Js, dtype=dtype)          # second call reuses the member table
    torch.cuda.synchronize()
    for (m, U, M), Ud, R, J in zip(members, Us, Rs, Js):
        R1, J1 = M.jacobian(Ud, dtype=dtype)
        torch.cuda.synchronize()
        assert torch.equal(R, R1) and torch.equal(J, J1)


def test_ensemble_residual_only(members):
    from paper_2204_04321_amd.api import Ensemble
    E = Ensemble([M for _, _, M in members])
    Us = [to_dev(U) for _, U, _ in members]
    Rs = [torch.empty(M.n_dofs, dtype=torch.float64, device="cuda") for _, _, M in members]
    E.assemble(Us, Rs, None)
    torch.cuda.synchronize()
    for (m, U, M), Ud, R in zip(members, Us, Rs):
        assert torch.equal(R, M.residual(Ud))


@pytest.mark.parametrize("k", [0, 4])
def test_ensemble_member_vs_oracle(members, k):
    from paper_2204_04321_amd.api import Ensemble
    E = Ensemble([M for _, _, M in members])
    Us = [to_dev(U) for _, U, _ in members]
    Rs = [torch.empty(M.n_dofs, dtype=torch.float64, device="cuda") for _, _, M in members]
    Js = [torch.empty(M.nnz, dtype=torch.float64, device="cuda") for _, _, M in members]
    E.assemble(Us, Rs, Js)
    m, U, M = members[k]
    rowptr, colidx = M.pattern()
    torch.cuda.synchronize()
    import scipy.sparse as sp
    Jg = sp.csr_matrix((Js[k].cpu().numpy(), colidx.cpu().numpy().astype(np.int64), rowptr.cpu().numpy()),
                       shape=(M.n_dofs, M.n_dofs))
    Ro, Jo = fo.assemble(m, U)
    e = parity_errors(Rs[k].cpu().numpy(), Jg, Ro, Jo, fo.abs_scales(m, U), fo.element_scales(m, U))
    print(f"[ensemble member {k}] {e}")
    assert max(e["term"]) <= 1e-12 and max(e["elem"]) <= 1e-12 and max(e["plain"]) <= 1e-12
    assert m.A != members[0][0].A or k == 0     # members carry their own rate factor


def test_hexahedral_ensemble_equals_single_mesh():
    """Hexahedral members (uneven sizes and layer counts) through the same persistent launch."""
    from test_gpu_assembly import _box
    from paper_2204_04321_amd.api import Ensemble
    hex_members = [_box(nx, ny, L, "hex", 40 + i) for i, (nx, ny, L) in enumerate([(3, 2, 1), (9, 7, 4), (20, 13, 6)])]
    Ms = [gpu_mesh(m) for m, _ in hex_members]
    E = Ensemble(Ms)
    Us = [to_dev(U) for _, U in hex_members]
    for dtype, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        Rs = [torch.full((M.n_dofs,), float("nan"), dtype=torch.float64, device="cuda") for M in Ms]
        Js = [torch.full((M.nnz,), float("nan"), dtype=tdt, device="cuda") for M in Ms]
        E.assemble(Us, Rs, Js, dtype=dtype)
        torch.cuda.synchronize()
        for M, Ud, R, J in zip(Ms, Us, Rs, Js):
            R1, J1 = M.jacobian(Ud, dtype=dtype)
            torch.cuda.synchronize()
            assert torch.equal(R, R1) and torch.equal(J, J1)
    # and the largest member against the oracle
    (m, U), M = hex_members[-1], Ms[-1]
    R1, J1 = gpu_jacobian(M, U)
    Ro, Jo = fo.assemble(m, U)
    e = parity_errors(R1, J1, Ro, Jo, fo.abs_scales(m, U), fo.element_scales(m, U))
    print(f"[hex ensemble, largest member] {e}")
    assert max(e["term"]) <= 1e-12 and max(e["elem"]) <= 1e-12 and max(e["plain"]) <= 1e-12


def test_wedge_ensemble_with_general_exponent():
    """A wedge member with n != 3 beside an n = 3 one: residual and both Jacobian types agree
    with the oracle for every member (a mixed ensemble takes the general power law for all)."""
    from test_gpu_assembly import _box
    from paper_2204_04321_amd.api import Ensemble
    mus = [_box(4, 3, 2, "wedge", 50), _box(5, 4, 3, "wedge", 51)]
    mus[1] = (mus[1][0].with_fields(n=1.0, A=2e-13), mus[1][1])
    Ms = [gpu_mesh(m) for m, _ in mus]
    E = Ensemble(Ms)
    Us = [to_dev(U) for _, U in mus]
    Rs = [torch.full((M.n_dofs,), float("nan"), dtype=torch.float64, device="cuda") for M in Ms]
    E.assemble(Us, Rs)
    torch.cuda.synchronize()
    # the n != 3 member equals its own residual bit for bit, the n = 3 one agrees with the
    # oracle to 1e-12 (general power law instead of the n = 3 evaluation)
    assert torch.equal(Rs[1], Ms[1].residual(Us[1]))
    for (m, U), R in zip(mus, Rs):
        Ro = fo.residual(m, U)
        rs, _ = fo.abs_scales(m, U)
        er_, _ = fo.element_scales(m, U)
        d = np.abs(R.cpu().numpy() - Ro)
        assert np.max(d / rs) <= 1e-12 and np.max(d / er_) <= 1e-12 and d.max() <= 1e-12 * np.abs(Ro).max()
    import scipy.sparse as sp
    for dtype, tdt, tol, tol_plain in (("f64", torch.float64, 1e-12, 1e-12), ("f32", torch.float32, 1e-5, 1e-6)):
        Js = [torch.full((M.nnz,), float("nan"), dtype=tdt, device="cuda") for M in Ms]
        E.assemble(Us, Rs, Js, dtype=dtype)
        torch.cuda.synchronize()
        R1, J1 = Ms[1].jacobian(Us[1], dtype=dtype)
        torch.cuda.synchronize()
        assert torch.equal(Rs[1], R1) and torch.equal(Js[1], J1)
        for (m, U), R, J, M in zip(mus, Rs, Js, Ms):
            rowptr, colidx = M.pattern()
            Jg = sp.csr_matrix((J.double().cpu().numpy(), colidx.cpu().numpy().astype(np.int64),
                                rowptr.cpu().numpy()), shape=(M.n_dofs, M.n_dofs))
            Ro, Jo = fo.assemble(m, U)
            e = parity_errors(R.cpu().numpy(), Jg, Ro, Jo, fo.abs_scales(m, U), fo.element_scales(m, U))
            assert e["term"][0] <= 1e-12 and e["elem"][0] <= 1e-12 and e["plain"][0] <= 1e-12, (dtype, e)
            assert e["term"][1] <= tol and e["elem"][1] <= tol and e["plain"][1] <= tol_plain, (dtype, e)


def test_tetrahedral_ensemble_with_fronts_equals_single_mesh():
    """Tetrahedral members, one of them with ocean fronts: the persistent launch and the
    front loads added after it give each member's single-mesh result bit for bit; a wedge
    member in the same ensemble is refused (one element type per launch)."""
    from fo_inputs import marine_sheet
    from test_gpu_assembly import _box
    from paper_2204_04321_amd import _lib
    from paper_2204_04321_amd.api import Ensemble
    mar, Umar = marine_sheet(seed=8, n_points=300, n_layers=4)
    tets = [_box(nx, ny, L, "tet", 60 + i) for i, (nx, ny, L) in enumerate([(3, 2, 2), (8, 6, 5)])]
    tets.append((mar.with_fields(elem="tet"), Umar))
    Ms = [gpu_mesh(m) for m, _ in tets]
    E = Ensemble(Ms)
    Us = [to_dev(U) for _, U in tets]
    for dtype, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        Rs = [torch.full((M.n_dofs,), float("nan"), dtype=torch.float64, device="cuda") for M in Ms]
        Js = [torch.full((M.nnz,), float("nan"), dtype=tdt, device="cuda") for M in Ms]
        E.assemble(Us, Rs, Js, dtype=dtype)
        torch.cuda.synchronize()
        for M, Ud, R, J in zip(Ms, Us, Rs, Js):
            R1, J1 = M.jacobian(Ud, dtype=dtype)
            torch.cuda.synchronize()
            assert torch.equal(R, R1) and torch.equal(J, J1)
    (m, U), M = tets[-1], Ms[-1]
    R1, J1 = gpu_jacobian(M, U)
    Ro, Jo = fo.assemble(m, U)
    e = parity_errors(R1, J1, Ro, Jo, fo.abs_scales(m, U), fo.element_scales(m, U))
    print(f"\n[tet ensemble, marine member] {e}")
    assert max(e["term"]) <= 1e-12 and max(e["elem"]) <= 1e-12 and max(e["plain"]) <= 1e-12
    w, _ = _box(3, 2, 2, "wedge", 70)
    with pytest.raises(_lib.FoError):
        Ensemble([Ms[0], gpu_mesh(w)])


def test_full_size_64_member_ensemble():
    """The benchmark's ensemble (64 seeded members of 10k-200k base triangles, 10 layers) in
    one persistent launch: every member's residual and FP64 Jacobian bit for bit equal to its
    own single-mesh assembly, and the smallest and the largest member, whole mesh, against the
    oracle (every row, in host processes)."""
    import functools
    import multiprocessing as mp
    import os

    from paper_2204_04321_amd.api import Ensemble
    from test_gpu_assembly import _full_mesh_parity
    with mp.get_context("spawn").Pool(min(16, len(os.sched_getaffinity(0)))) as pool:
        pairs = pool.map(ensemble_member, range(64))
    meshes = [gpu_mesh(m) for m, _ in pairs]
    cells = [M.n_cells for M in meshes]
    print(f"\n[ensemble64] {sum(cells)} wedges, members {min(cells)}..{max(cells)}", flush=True)
    E = Ensemble(meshes)
    Us = [to_dev(U) for _, U in pairs]
    Rs = [torch.full((M.n_dofs,), float("nan"), dtype=torch.float64, device="cuda") for M in meshes]
    Js = [torch.full((M.nnz,), float("nan"), dtype=torch.float64, device="cuda") for M in meshes]
    E.assemble(Us, Rs, Js)
    torch.cuda.synchronize()
    for i, (M, Ud) in enumerate(zip(meshes, Us)):
        R1, J1 = M.jacobian(Ud)
        torch.cuda.synchronize()
        assert torch.equal(Rs[i], R1) and torch.equal(Js[i], J1), i
        del R1, J1
    print("[ensemble64] every member equals its single-mesh assembly bit for bit", flush=True)
    small, large = int(np.argmin(cells)), int(np.argmax(cells))
    del Rs, Js, E, meshes, Us
    torch.cuda.empty_cache()
    for i in (small, large):
        _full_mesh_parity(functools.partial(ensemble_member, i), f"member{i}")
