"""Python binding over the C ABI: marshals arrays and PyTorch device tensors into
library calls.  Every step of the computation runs in the HIP library; PyTorch
only supplies device memory and the current stream."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import FO_F32, FO_F64, FO_HEX8, FO_JAC_NEWTON, FO_JAC_PICARD, FO_TET4, FO_WEDGE6, check


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return int(t.data_ptr())


def mesh_desc(desc, keep: list) -> "_lib.MeshDesc":
    """fo_mesh_desc for `desc` (fields elem 'wedge', 'tet' or 'hex', xy [V,2], cells [T,3|4],
    surface, thickness, beta [V], sigma [L+1], constants A, n, rho, g, eps0, and optionally
    front_edges [n,2] with rho_w).  The host arrays it points to are appended to `keep`,
    which must outlive fo_mesh_create."""
    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    d = _lib.MeshDesc()
    d.elem = {"wedge": FO_WEDGE6, "tet": FO_TET4, "hex": FO_HEX8}[desc.elem]
    d.n_base_verts = int(desc.xy.shape[0])
    d.n_base_cells = int(desc.cells.shape[0])
    d.n_layers = int(len(desc.sigma) - 1)
    d.base_xy = arr(desc.xy, np.float64)
    d.base_cells = arr(desc.cells, np.int32)
    d.surface = arr(desc.surface, np.float64)
    d.thickness = arr(desc.thickness, np.float64)
    d.beta = arr(desc.beta, np.float64)
    d.sigma = arr(desc.sigma, np.float64)
    d.A, d.n, d.rho, d.g, d.eps0 = (float(desc.A), float(desc.n), float(desc.rho),
                                     float(desc.g), float(desc.eps0))
    fe = getattr(desc, "front_edges", None)
    if fe is not None and len(fe) > 0:
        d.front_edges = arr(np.asarray(fe).reshape(-1, 2), np.int32)
        d.n_front_edges = int(np.asarray(fe).reshape(-1, 2).shape[0])
        d.rho_w = float(desc.rho_w)
    return d


class Mesh:
    """An uploaded extruded mesh.  `desc` is any object with the fields elem ('wedge' or
    'hex'), xy [V,2], cells [T,3|4], surface, thickness, beta [V], sigma [L+1], and the
    constants A, n, rho, g, eps0."""

    def __init__(self, desc, stream=None):
        L = _lib.lib()
        self._keep = []
        d = mesh_desc(desc, self._keep)
        h = C.c_void_p()
        check(L.fo_mesh_create(C.byref(d), _stream(stream), C.byref(h)))
        self._keep = []
        self.handle = h
        nn, nd, nc, nz = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        check(L.fo_mesh_info(h, C.byref(nn), C.byref(nd), C.byref(nc), C.byref(nz)))
        self.n_nodes, self.n_dofs, self.n_cells, self.nnz = nn.value, nd.value, nc.value, nz.value
        self.elem = desc.elem
        self.n_layers = int(len(desc.sigma) - 1)
        self.n_verts = int(desc.xy.shape[0])
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().fo_mesh_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- pattern ---------------------------------------------------------------------------
    def pattern(self, stream=None):
        rowptr = torch.empty(self.n_dofs + 1, dtype=torch.int64, device=self.device)
        colidx = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        check(_lib.lib().fo_jacobian_pattern(self.handle, _ptr(rowptr), _ptr(colidx), _stream(stream)))
        return rowptr, colidx

    # ---- assembly --------------------------------------------------------------------------
    def residual(self, U: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        self._check_vec(U)
        R = out if out is not None else torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        check(_lib.lib().fo_assemble_residual(self.handle, _ptr(U), _ptr(R), _stream(stream)))
        return R

    def jacobian(self, U: torch.Tensor, dtype: str = "f64", kind: str = "newton",
                 with_residual: bool = True, Jvals: torch.Tensor | None = None,
                 R: torch.Tensor | None = None, stream=None):
        self._check_vec(U)
        tdt = torch.float64 if dtype == "f64" else torch.float32
        if Jvals is None:
            Jvals = torch.empty(self.nnz, dtype=tdt, device=self.device)
        if with_residual and R is None:
            R = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        check(_lib.lib().fo_assemble_jacobian(
            self.handle, _ptr(U), _ptr(R) if with_residual else None, _ptr(Jvals),
            FO_F64 if dtype == "f64" else FO_F32,
            FO_JAC_NEWTON if kind == "newton" else FO_JAC_PICARD, _stream(stream)))
        return (R, Jvals) if with_residual else Jvals

    def sia(self, out: torch.Tensor | None = None, stream=None):
        U = out if out is not None else torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        check(_lib.lib().fo_initial_guess_sia(self.handle, _ptr(U), _stream(stream)))
        return U

    # ---- Newton solve ---------------------------------------------------------------------
    def newton_opts(self, **kw) -> "_lib.NewtonOpts":
        o = _lib.NewtonOpts()
        _lib.lib().fo_newton_default_opts(C.byref(o))
        for k, v in kw.items():
            if k == "jac_dtype":
                v = FO_F64 if v in ("f64", FO_F64) else FO_F32
            elif k == "init":
                v = {"user": _lib.FO_INIT_USER, "sia": _lib.FO_INIT_SIA, "learned": _lib.FO_INIT_LEARNED}.get(v, v)
            elif k in ("mlp_params", "mlp_norm"):
                v = _ptr(v) if isinstance(v, torch.Tensor) else v
            elif k == "linear_solver":
                v = {"gmres": _lib.FO_LIN_GMRES, "pcg": _lib.FO_LIN_PCG}.get(v, v)
            elif k == "preconditioner":
                v = {"column": _lib.FO_PREC_COLUMN, "mdsc": _lib.FO_PREC_MDSC}.get(v, v)
            elif k == "mdsc":
                v = v.handle.value if isinstance(v, Mdsc) else v
            setattr(o, k, v)
        return o

    def workspace_bytes(self, opts) -> int:
        n = _lib.lib().fo_newton_workspace_bytes(self.handle, C.byref(opts))
        if n == 0:
            raise ValueError("bad Newton options")
        return int(n)

    def newton_solve(self, U: torch.Tensor, workspace: torch.Tensor | None = None,
                     check_status: bool = False, stream=None, **kw) -> dict:
        """Damped Newton in place on U (device float64 [n_dofs]).  Returns the report as a
        dict; status != 0 (not converged, non-finite) is reported, raised only if
        check_status."""
        self._check_vec(U)
        opts = self.newton_opts(**kw)
        need = self.workspace_bytes(opts)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        rep = _lib.NewtonReport()
        st = _lib.lib().fo_newton_solve(self.handle, _ptr(U), C.byref(opts), C.byref(rep),
                                        _ptr(workspace), workspace.numel(), _stream(stream))
        d = rep.as_dict()
        d["status"] = st
        d["message"] = _lib.lib().fo_last_error().decode() if st != 0 else ""
        if check_status:
            check(st)
        return d

    # ---- learned initial guess --------------------------------------------------------------
    def features(self, norm: torch.Tensor | None = None, out: torch.Tensor | None = None, stream=None):
        F = out if out is not None else torch.empty(self.n_verts, 10, dtype=torch.float32, device=self.device)
        check(_lib.lib().fo_column_features(self.handle, _ptr(norm), _ptr(F), _stream(stream)))
        return F

    def learned_guess(self, params: torch.Tensor, norm: torch.Tensor, out: torch.Tensor | None = None,
                      workspace: torch.Tensor | None = None, fallback: int = 1, smooth: int = 0, stream=None):
        """(U, used_network): network guess, its correction smoothed by `smooth` sweeps over the
        base mesh, with the shallow-ice fallback (1: non-finite or larger residual norm; 0:
        non-finite only)."""
        U = out if out is not None else torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        need = int(_lib.lib().fo_learned_workspace_bytes(self.handle))
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        used = C.c_int32()
        check(_lib.lib().fo_initial_guess_learned(self.handle, _ptr(params), _ptr(norm), _ptr(U), int(fallback),
                                                  int(smooth), _ptr(workspace), workspace.numel(), C.byref(used),
                                                  _stream(stream)))
        return U, bool(used.value)

    def learned_guess_noalloc(self, params: torch.Tensor, norm: torch.Tensor, out: torch.Tensor | None = None,
                              fallback: int = 1, smooth: int = 0, stream=None):
        """learned_guess with the library's own device array as workspace (no allocation in
        the call; meshes up to the array's size)."""
        U = out if out is not None else torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        used = C.c_int32()
        check(_lib.lib().fo_initial_guess_learned_noalloc(self.handle, _ptr(params), _ptr(norm), _ptr(U),
                                                          int(fallback), int(smooth), C.byref(used),
                                                          _stream(stream)))
        return U, bool(used.value)

    def learned_targets(self, U: torch.Tensor, U_sia: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        """Training targets [V, 22] (FP32) of a converged solution U against the shallow-ice guess."""
        self._check_vec(U)
        self._check_vec(U_sia)
        T = out if out is not None else torch.empty(self.n_verts, 22, dtype=torch.float32, device=self.device)
        check(_lib.lib().fo_learned_targets(self.handle, _ptr(U), _ptr(U_sia), _ptr(T), _stream(stream)))
        return T

    # ---- measurement ----------------------------------------------------------------------
    def profile(self, on: bool = True):
        check(_lib.lib().fo_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        """(summed assembly-kernel milliseconds, launches) since the last read."""
        ms, n = C.c_double(), C.c_int64()
        check(_lib.lib().fo_profile_read(self.handle, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def _check_vec(self, U):
        if U.dtype != torch.float64 or U.numel() != self.n_dofs:
            raise ValueError(f"expected float64 vector of {self.n_dofs} dofs")


def aggregate_graph(ptr: np.ndarray, idx: np.ndarray):
    """Host aggregation of a graph given as sorted neighbour lists (with the vertex itself):
    returns (agg [n] int32, n_agg).  No device needed."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n = len(ptr) - 1
    agg = np.empty(max(n, 0), dtype=np.int32)
    n_agg = C.c_int32()
    check(_lib.lib().fo_mdsc_aggregate_graph(n, ptr.ctypes.data, idx.ctypes.data, agg.ctypes.data, C.byref(n_agg)))
    return agg, n_agg.value


class Mdsc:
    """Two-level column semicoarsening preconditioner of one mesh (the library object)."""

    def __init__(self, mesh: Mesh, stream=None):
        self.mesh = mesh
        h = C.c_void_p()
        check(_lib.lib().fo_mdsc_create(mesh.handle, _stream(stream), C.byref(h)))
        self.handle = h
        nl = C.c_int32()
        check(_lib.lib().fo_mdsc_levels(h, C.byref(nl), None))
        nv = np.empty(nl.value + 1, dtype=np.int32)
        check(_lib.lib().fo_mdsc_levels(h, C.byref(nl), nv.ctypes.data))
        self.n_levels = nl.value
        self.level_verts = [int(x) for x in nv]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().fo_mdsc_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def graph(self, level: int):
        """(ptr, idx, agg) of a plane level (agg None on the coarsest)."""
        n = self.level_verts[level]
        ptr = np.empty(n + 1, dtype=np.int32)
        check(_lib.lib().fo_mdsc_graph(self.handle, level, ptr.ctypes.data, None, None))
        idx = np.empty(int(ptr[-1]), dtype=np.int32)
        agg = np.empty(n, dtype=np.int32) if level < self.n_levels else None
        check(_lib.lib().fo_mdsc_graph(self.handle, level, None, idx.ctypes.data,
                                       agg.ctypes.data if agg is not None else None))
        return ptr, idx, agg

    def setup(self, Jvals: torch.Tensor, stream=None):
        dt = FO_F64 if Jvals.dtype == torch.float64 else FO_F32
        check(_lib.lib().fo_mdsc_setup(self.handle, _ptr(Jvals), dt, _stream(stream)))

    def apply(self, r: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        self.mesh._check_vec(r)
        z = out if out is not None else torch.empty_like(r)
        check(_lib.lib().fo_mdsc_apply(self.handle, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def export(self, what: str, level: int = 0, stream=None) -> np.ndarray:
        field = {"weights": _lib.FO_MDSC_WEIGHTS, "plane": _lib.FO_MDSC_PLANE, "bound": _lib.FO_MDSC_BOUND}[what]
        if field == _lib.FO_MDSC_WEIGHTS:
            n = 4 * self.mesh.n_nodes
        elif field == _lib.FO_MDSC_PLANE:
            n = 4 * int(self.graph(level)[0][-1])
        else:
            n = 1
        out = np.empty(n, dtype=np.float64)
        check(_lib.lib().fo_mdsc_export(self.handle, field, level, out.ctypes.data, n, _stream(stream)))
        return out


class Ensemble:
    """Several uploaded meshes (same element type) assembled by one persistent launch."""

    def __init__(self, meshes, stream=None):
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = C.c_void_p()
        check(_lib.lib().fo_ensemble_create(arr, len(self.meshes), _stream(stream), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().fo_ensemble_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self, Us, Rs=None, Js=None, dtype: str = "f64", kind: str = "newton", stream=None):
        """Us: list of device float64 vectors; Rs: list (or None); Js: list of value
        buffers (or None for residuals only).  Buffers are written in place."""
        n = len(self.meshes)
        for M, U in zip(self.meshes, Us):
            M._check_vec(U)
        P = C.c_void_p * n
        u = P(*[_ptr(U) for U in Us])
        r = P(*[(_ptr(R) if R is not None else None) for R in Rs]) if Rs is not None else None
        j = P(*[_ptr(J) for J in Js]) if Js is not None else None
        check(_lib.lib().fo_ensemble_assemble(
            self.handle, u, r, j, FO_F64 if dtype == "f64" else FO_F32,
            FO_JAC_NEWTON if kind == "newton" else FO_JAC_PICARD, _stream(stream)))


class MLP:
    """Thin wrapper over the network kernels (parameters and Adam moments as FP32 tensors)."""
    LAYERS = (10, 128, 128, 128, 22)

    def __init__(self, params: torch.Tensor):
        n = int(_lib.lib().fo_mlp_param_count())
        if params.numel() != n or params.dtype != torch.float32 or not params.is_cuda:
            raise ValueError(f"expected {n} FP32 device parameters")
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grads = torch.zeros_like(params)
        self.step_count = 0

    def forward(self, X: torch.Tensor, acts: torch.Tensor | None = None, stream=None):
        B = X.shape[0]
        acts = acts if acts is not None else torch.empty(3, B, 128, dtype=torch.float32, device=X.device)
        Y = torch.empty(B, 22, dtype=torch.float32, device=X.device)
        check(_lib.lib().fo_mlp_forward(_ptr(self.params), _ptr(X), B, _ptr(acts), _ptr(Y), _stream(stream)))
        return Y, acts

    def backward(self, X, acts, dY, stream=None):
        B = X.shape[0]
        dacts = torch.empty(2, B, 128, dtype=torch.float32, device=X.device)
        check(_lib.lib().fo_mlp_backward(_ptr(self.params), _ptr(X), B, _ptr(acts), _ptr(dY), _ptr(dacts),
                                         _ptr(self.grads), _stream(stream)))
        return self.grads

    @staticmethod
    def feature_stats(X: torch.Tensor, normalised: bool = False, stream=None):
        """Normalisation [20] (10 means, 10 standard deviations + 1e-6) of raw features X [n, 10];
        with normalised=True also the normalised features: (norm, Xn)."""
        if X.dtype != torch.float32 or X.dim() != 2 or X.shape[1] != 10:
            raise ValueError("expected FP32 features [n, 10]")
        norm = torch.empty(20, dtype=torch.float32, device=X.device)
        Xn = torch.empty_like(X) if normalised else None
        check(_lib.lib().fo_feature_stats(_ptr(X), X.shape[0], _ptr(norm), _ptr(Xn), _stream(stream)))
        return (norm, Xn) if normalised else norm

    @staticmethod
    def mse_grad(Y, T, loss: torch.Tensor | None = None, stream=None):
        dY = torch.empty_like(Y)
        check(_lib.lib().fo_mse_grad(_ptr(Y), _ptr(T), Y.numel(), _ptr(dY), _ptr(loss), _stream(stream)))
        return dY

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        check(_lib.lib().fo_adam_step(_ptr(self.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v),
                                      self.params.numel(), lr, b1, b2, eps, self.step_count, _stream(stream)))
