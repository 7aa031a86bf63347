"""Helpers for GPU tests: run the HIP library through its C ABI and bring results back."""
import numpy as np
import scipy.sparse as sp
import torch


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def gpu_mesh(desc):
    from paper_2204_04321_amd.api import Mesh
    return Mesh(desc)


def gpu_jacobian(M, U, dtype="f64", kind="newton"):
    Ud = to_dev(U)
    R, J = M.jacobian(Ud, dtype=dtype, kind=kind)
    rowptr, colidx = M.pattern()
    torch.cuda.synchronize()
    Jc = sp.csr_matrix((J.double().cpu().numpy(), colidx.cpu().numpy().astype(np.int64),
                        rowptr.cpu().numpy()), shape=(M.n_dofs, M.n_dofs))
    return R.cpu().numpy(), Jc


def gpu_residual(M, U):
    R = M.residual(to_dev(U))
    torch.cuda.synchronize()
    return R.cpu().numpy()


def row_scaled_errors(R_gpu, J_gpu, R_ref, J_ref, rscale, jscale):
    """max_i |dR_i| / sum_e |R_e,i| and max_ij |dJ_ij| / max_j sum_e |J_e,ij|."""
    er = np.max(np.abs(R_gpu - R_ref) / np.maximum(rscale, 1e-300))
    D = (J_gpu - J_ref).tocsr()
    D.sum_duplicates()
    if D.nnz == 0:
        return er, 0.0
    rows = np.repeat(np.arange(D.shape[0]), np.diff(D.indptr))
    ej = np.max(np.abs(D.data) / np.maximum(jscale[rows], 1e-300))
    return er, ej
