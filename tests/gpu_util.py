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


def _row_max_abs(D):
    """max_j |D_ij| per row of a CSR matrix (0 for empty rows)."""
    out = np.zeros(D.shape[0])
    if D.nnz:
        rows = np.repeat(np.arange(D.shape[0]), np.diff(D.indptr))
        np.maximum.at(out, rows, np.abs(D.data))
    return out


def parity_errors(R_gpu, J_gpu, R_ref, J_ref, term_scales, elem_scales):
    """Errors of a GPU residual / Jacobian against the oracle on three scales:
    'term'  - row-scaled by the per-term scale (|dR_i| / S^R_i, max_j |dJ_ij| / max_j S^J_ij),
    'elem'  - row-scaled by the element-level scale (sum_e |R_e,i|, max_j sum_e |J_e,ij|),
    'plain' - norm-wise, ||dR||_inf / ||R||_inf and max |dJ| / max |J|.
    Returns {scale: (err_R, err_J)} and, under 'worst_elem', the rows where the element-level
    errors peak."""
    dR = np.abs(R_gpu - R_ref)
    D = (J_gpu - J_ref).tocsr()
    D.sum_duplicates()
    dJ = _row_max_abs(D)
    out = {}
    for name, (rs, js) in (("term", term_scales), ("elem", elem_scales)):
        er = dR / np.maximum(rs, 1e-300)
        ej = dJ / np.maximum(js, 1e-300)
        out[name] = (float(er.max()), float(ej.max()))
        if name == "elem":
            out["worst_elem"] = (int(er.argmax()), int(ej.argmax()))
    out["plain"] = (float(dR.max() / np.abs(R_ref).max()),
                    float(dJ.max() / np.abs(J_ref.data).max()) if J_ref is not None else 0.0)
    return out
