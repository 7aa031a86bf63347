// Damped Newton solve of F(U) = 0 (arXiv:2204.04321 Sec. 3.1, eq. linearsystem):
// J(U_k) delta = -F(U_k), U_{k+1} = U_k + alpha_k delta.  Each linear system is solved
// by restarted GMRES (Sec. 3.1) with right preconditioning by the vertical-column
// block factorisation, or by the two-level column semicoarsening preconditioner built on
// it (Sec. 3.3, fo_mdsc).  Readings where the paper is silent: alpha from backtracking
// 1, 1/2, 1/4, ... accepting ||F(U + alpha delta)|| <= (1 - 1e-4 alpha) ||F(U)||;
// convergence when ||F(U)||_2 <= tol ||F(0)||_2 (F(0) is the gravity load and does
// not depend on the initial guess).  The timers carry the paper's names (Sec. 5):
// Total Fill (all assembly calls), Preconditioner Construction, Linear Solve, Total Solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "fo_internal.h"
#include "fo_mdsc.h"
#include "fo_solver.h"

namespace fo {
namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t J, R, Rt, Ut, dU, W, Z, T, fac, V, V_bytes, partial, dots, total;
};

Layout layout(const fo_mesh *m, const fo_newton_opts *o) {
  const size_t n = size_t(m->view.n_dofs);
  const size_t esz = o->jac_dtype == FO_F32 ? 4 : 8;
  const int mres = o->gmres_restart;
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off += up(bytes); return at; };
  L.J = take(esz * size_t(m->nnz));
  L.R = take(8 * n);
  L.Rt = take(8 * n);
  L.Ut = take(8 * n);
  L.dU = take(8 * n);
  L.W = take(8 * n);
  L.Z = take(8 * n);
  L.T = take(8 * n);
  L.fac = take(4 * size_t(m->view.V) * size_t(m->view.L + 1) * 12);
  // the Krylov basis region also holds the learned guess's workspace before the first step
  L.V_bytes = std::max(8 * n * size_t(mres + 1), o->init == FO_INIT_LEARNED ? learned_workspace_bytes(m) : 0);
  L.V = take(L.V_bytes);
  L.partial = take(8 * std::max(size_t(multidot_blocks(int64_t(n))) * size_t(mres + 2),
                                 2 * size_t(dot2_blocks(int64_t(n)))));
  L.dots = take(8 * std::max(size_t(mres + 2), size_t(8)));   // GMRES: h and norms; CG: 6 scalars
  L.total = off;
  return L;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct Ctx {
  const fo_mesh *m;
  hipStream_t s;
  char *ws;
  Layout L;
  double *host;   // pinned scratch for reductions
  int64_t n;
  double *dptr(size_t off) { return reinterpret_cast<double *>(ws + off); }
};

// ||x||_2 with a deterministic device reduction
fo_status norm2(Ctx &c, const double *x, double &out) {
  fo_status st = multidot(c.n, nullptr, 0, 0, x, c.dptr(c.L.partial), c.dptr(c.L.dots), c.s);
  if (st != FO_OK) return st;
  FO_HIP_TRY(hipMemcpyAsync(c.host, c.dptr(c.L.dots), sizeof(double), hipMemcpyDeviceToHost, c.s));
  FO_HIP_TRY(hipStreamSynchronize(c.s));
  out = std::sqrt(c.host[0]);
  return FO_OK;
}

// z = M^{-1} r with the preconditioner the options name
fo_status precondition(Ctx &c, const fo_newton_opts *o, const double *r, double *z) {
  if (o->preconditioner == FO_PREC_MDSC) return fo_mdsc_apply(o->mdsc, r, z, c.s);
  return colblock_apply(c.m, reinterpret_cast<const float *>(c.ws + c.L.fac), r, z, c.s);
}

// GMRES(m), right preconditioned: solve J x = b, x0 = 0.  Returns iterations in `its`.
fo_status gmres(Ctx &c, const fo_newton_opts *o, const void *Jv, const double *b, double *x, int64_t &its,
                double &rel_out) {
  const int64_t n = c.n;
  const int mres = o->gmres_restart;
  double *V = c.dptr(c.L.V);
  double *w = c.dptr(c.L.W);
  double *z = c.dptr(c.L.Z);
  double *t = c.dptr(c.L.T);
  fo_status st;
  its = 0;
  double bnorm;
  if ((st = norm2(c, b, bnorm)) != FO_OK) return st;
  if ((st = launch_fill_zero(x, sizeof(double) * n, c.s)) != FO_OK) return st;   // x = 0
  rel_out = 0.0;
  if (bnorm == 0.0) return FO_OK;
  if (!std::isfinite(bnorm)) return fail(FO_ENONFINITE, "gmres: non-finite right-hand side");
  std::vector<double> H(size_t(mres + 1) * mres), cs(mres), sn(mres), g(mres + 1), y(mres);
  // r = b (x = 0)
  if ((st = axpby(n, 1.0, b, 0.0, w, c.s)) != FO_OK) return st;
  double beta = bnorm;
  bool done = false;
  while (!done) {
    if ((st = axpby(n, 1.0 / beta, w, 0.0, V, c.s)) != FO_OK) return st;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = -1;
    for (int j = 0; j < mres; ++j) {
      double *vj = V + int64_t(j) * n;
      if ((st = precondition(c, o, vj, z)) != FO_OK) return st;
      if ((st = spmv(c.m, Jv, o->jac_dtype, z, w, c.s)) != FO_OK) return st;
      // classical Gram-Schmidt with one selective reorthogonalisation.  A pass that
      // shrinks w by kappa = ||w|| / ||w - V h|| leaves it orthogonal to V only to about
      // eps kappa, and the norm from ||w - V h||^2 = ||w||^2 - ||h||^2 is then good to
      // about eps kappa^2; the second pass runs when kappa > 1e3 (both bounds near 1e-10)
      double hsum[512];
      for (int pass = 0; pass < 2; ++pass) {
        if ((st = multidot(n, V, n, j + 1, w, c.dptr(c.L.partial), c.dptr(c.L.dots), c.s)) != FO_OK) return st;
        if ((st = multiaxpy(n, V, n, j + 1, c.dptr(c.L.dots), w, -1.0, c.s)) != FO_OK) return st;
        FO_HIP_TRY(hipMemcpyAsync(c.host, c.dptr(c.L.dots), sizeof(double) * (j + 2), hipMemcpyDeviceToHost, c.s));
        FO_HIP_TRY(hipStreamSynchronize(c.s));
        for (int i = 0; i <= j; ++i) hsum[i] = (pass == 0 ? 0.0 : hsum[i]) + c.host[i];
        double h2 = 0.0;
        for (int i = 0; i <= j; ++i) h2 += c.host[i] * c.host[i];
        const double wn2 = c.host[j + 1] - h2;   // ||w||^2 after this projection
        H[size_t(j + 1) * mres + j] = std::sqrt(wn2 > 0 ? wn2 : 0.0);
        if (pass == 0 && wn2 > 1e-6 * c.host[j + 1]) break;
      }
      for (int i = 0; i <= j; ++i) H[size_t(i) * mres + j] = hsum[i];
      const double hn = H[size_t(j + 1) * mres + j];
      if (!std::isfinite(hn)) return fail(FO_ENONFINITE, "gmres: non-finite Krylov vector");
      if (hn > 0 && j + 1 <= mres)
        if ((st = axpby(n, 1.0 / hn, w, 0.0, V + int64_t(j + 1) * n, c.s)) != FO_OK) return st;
      // Givens rotations
      for (int i = 0; i < j; ++i) {
        const double a = H[size_t(i) * mres + j], bb = H[size_t(i + 1) * mres + j];
        H[size_t(i) * mres + j] = cs[i] * a + sn[i] * bb;
        H[size_t(i + 1) * mres + j] = -sn[i] * a + cs[i] * bb;
      }
      const double a = H[size_t(j) * mres + j], bb = H[size_t(j + 1) * mres + j];
      const double r = std::hypot(a, bb);
      cs[j] = r > 0 ? a / r : 1.0;
      sn[j] = r > 0 ? bb / r : 0.0;
      H[size_t(j) * mres + j] = r;
      H[size_t(j + 1) * mres + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      jend = j;
      const double rel = std::fabs(g[j + 1]) / bnorm;
      rel_out = rel;
      if (rel <= o->lin_rtol || its >= o->max_lin || hn == 0.0) {
        done = true;
        break;
      }
    }
    // y = H^{-1} g; x += M^{-1} V y
    const int k = jend + 1;
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int q = i + 1; q < k; ++q) acc -= H[size_t(i) * mres + q] * y[q];
      y[i] = acc / H[size_t(i) * mres + i];
    }
    std::memcpy(c.host, y.data(), sizeof(double) * k);
    FO_HIP_TRY(hipMemcpyAsync(c.dptr(c.L.dots), c.host, sizeof(double) * k, hipMemcpyHostToDevice, c.s));
    if ((st = launch_fill_zero(t, sizeof(double) * n, c.s)) != FO_OK) return st;
    if ((st = multiaxpy(n, V, n, k, c.dptr(c.L.dots), t, 1.0, c.s)) != FO_OK) return st;
    if ((st = precondition(c, o, t, z)) != FO_OK) return st;
    if ((st = axpby(n, 1.0, z, 1.0, x, c.s)) != FO_OK) return st;
    if (!done) {
      // restart: r = b - J x
      if ((st = spmv(c.m, Jv, o->jac_dtype, x, w, c.s)) != FO_OK) return st;
      if ((st = axpby(n, 1.0, b, -1.0, w, c.s)) != FO_OK) return st;
      if ((st = norm2(c, w, beta)) != FO_OK) return st;
      rel_out = beta / bnorm;
      if (beta <= o->lin_rtol * bnorm || beta == 0.0) done = true;
    }
    FO_HIP_TRY(hipStreamSynchronize(c.s));   // y staging buffer is reused
  }
  return FO_OK;
}

// Preconditioned conjugate gradients, x0 = 0, for the symmetric positive definite Newton
// system (J is the Hessian of a convex energy; M, the column block preconditioner, is SPD in
// exact arithmetic).  Stops when ||b - J x|| <= lin_rtol ||b|| (the recursively updated
// residual) or after max_lin iterations.  A direction with non-positive curvature (possible
// only through rounding: FP32 Jacobian values and the FP32 column factors make J and M^-1
// symmetric to about 1e-7 relative) ends the solve with FO_ENOTCONV.
fo_status pcg(Ctx &c, const fo_newton_opts *o, const void *Jv, const double *b, double *x, int64_t &its,
              double &rel_out) {
  const int64_t n = c.n;
  double *r = c.dptr(c.L.W), *z = c.dptr(c.L.Z), *p = c.dptr(c.L.T), *q = c.dptr(c.L.V);
  const float *fac = reinterpret_cast<const float *>(c.ws + c.L.fac);
  fo_status st;
  its = 0;
  rel_out = 0.0;
  double bnorm;
  if ((st = norm2(c, b, bnorm)) != FO_OK) return st;
  if ((st = launch_fill_zero(x, sizeof(double) * n, c.s)) != FO_OK) return st;   // x = 0
  if (bnorm == 0.0) return FO_OK;
  if (!std::isfinite(bnorm)) return fail(FO_ENONFINITE, "pcg: non-finite right-hand side");
  // device scalars: d[0] = p . q (d[1] = q . q, unused), d[2 + 2 s] = r . z and
  // d[3 + 2 s] = r . r of the two alternating slots s; one host synchronisation per iteration
  double *d = c.dptr(c.L.dots);
  double *part = c.dptr(c.L.partial);
  if ((st = axpby(n, 1.0, b, 0.0, r, c.s)) != FO_OK) return st;        // r = b
  if ((st = colblock_apply(c.m, fac, r, z, c.s)) != FO_OK) return st;  // z = M^-1 r
  if ((st = axpby(n, 1.0, z, 0.0, p, c.s)) != FO_OK) return st;        // p = z
  if ((st = dot2(n, z, r, part, d + 2, c.s)) != FO_OK) return st;
  FO_HIP_TRY(hipMemcpyAsync(c.host, d + 2, sizeof(double), hipMemcpyDeviceToHost, c.s));
  FO_HIP_TRY(hipStreamSynchronize(c.s));
  double rz = c.host[0];
  int slot = 0;
  while (its < o->max_lin) {
    if (!std::isfinite(rz)) return fail(FO_ENONFINITE, "pcg: non-finite Krylov vector");
    if (!(rz > 0.0))
      return fail(FO_ENOTCONV, "pcg: the preconditioned residual has non-positive norm (M^-1 is not positive "
                               "definite in this precision); use FO_LIN_GMRES");
    if ((st = spmv(c.m, Jv, o->jac_dtype, p, q, c.s)) != FO_OK) return st;              // q = J p
    if ((st = dot2(n, p, q, part, d, c.s)) != FO_OK) return st;                         // p . q
    if ((st = cg_step(n, d + 2 + 2 * slot, d, p, q, x, r, c.s)) != FO_OK) return st;    // x, r
    if ((st = colblock_apply(c.m, fac, r, z, c.s)) != FO_OK) return st;                 // z = M^-1 r
    const int nxt = slot ^ 1;
    if ((st = dot2(n, z, r, part, d + 2 + 2 * nxt, c.s)) != FO_OK) return st;            // r . z, r . r
    FO_HIP_TRY(hipMemcpyAsync(c.host, d, 6 * sizeof(double), hipMemcpyDeviceToHost, c.s));
    FO_HIP_TRY(hipStreamSynchronize(c.s));
    const double pq = c.host[0], rz1 = c.host[2 + 2 * nxt], rr = c.host[3 + 2 * nxt];
    if (!std::isfinite(pq)) return fail(FO_ENONFINITE, "pcg: non-finite curvature");
    if (!(pq > 0.0))
      return fail(FO_ENOTCONV, "pcg: a search direction has non-positive curvature (the Jacobian is not "
                               "positive definite in this precision); use FO_LIN_GMRES");
    ++its;
    rel_out = std::sqrt(rr) / bnorm;
    if (rel_out <= o->lin_rtol) break;
    if ((st = xpay(n, z, rz1 / rz, p, p, c.s)) != FO_OK) return st;   // p = z + beta p
    rz = rz1;
    slot = nxt;
  }
  return FO_OK;
}

}  // namespace
}  // namespace fo

using namespace fo;

extern "C" void fo_newton_default_opts(fo_newton_opts *o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_newton = 50;
  o->lin_rtol = 1e-6;
  o->gmres_restart = 100;
  o->max_lin = 500;
  o->jac_dtype = FO_F64;
  o->max_backtracks = 10;
  o->init = FO_INIT_USER;
  o->linear_solver = FO_LIN_GMRES;
  o->mlp_params = nullptr;
  o->mlp_norm = nullptr;
  o->learned_fallback = 1;
  o->learned_smooth = 0;
  o->preconditioner = FO_PREC_COLUMN;
  o->mdsc = nullptr;
}

extern "C" size_t fo_newton_workspace_bytes(const fo_mesh *m, const fo_newton_opts *o) {
  if (!m || !o || o->gmres_restart < 1 || o->gmres_restart > 500) return 0;
  return layout(m, o).total;
}

extern "C" fo_status fo_newton_solve(const fo_mesh *m, double *U, const fo_newton_opts *o,
                                     fo_newton_report *rep, void *ws, size_t ws_bytes, void *stream) {
  if (!m || !U || !o || !rep || !ws) return fail(FO_EINVAL, "fo_newton_solve: NULL argument");
  if (o->gmres_restart < 1 || o->gmres_restart > 500 || o->max_lin < 1 || o->max_newton < 0 ||
      !(o->tol > 0) || !(o->lin_rtol > 0) || o->max_backtracks < 0 ||
      (o->jac_dtype != FO_F64 && o->jac_dtype != FO_F32) ||
      (o->init != FO_INIT_USER && o->init != FO_INIT_SIA && o->init != FO_INIT_LEARNED) ||
      (o->init == FO_INIT_LEARNED && (!o->mlp_params || !o->mlp_norm)) ||
      (o->linear_solver != FO_LIN_GMRES && o->linear_solver != FO_LIN_PCG) ||
      (o->preconditioner != FO_PREC_COLUMN && o->preconditioner != FO_PREC_MDSC))
    return fail(FO_EINVAL, "fo_newton_solve: bad options");
  if (o->preconditioner == FO_PREC_MDSC) {
    if (!o->mdsc || o->mdsc->mesh != m)
      return fail(FO_EINVAL, "fo_newton_solve: FO_PREC_MDSC needs a fo_mdsc created on this mesh");
    if (o->linear_solver != FO_LIN_GMRES)
      return fail(FO_EINVAL, "fo_newton_solve: FO_PREC_MDSC is not symmetric; use FO_LIN_GMRES");
  }
  if ((reinterpret_cast<uintptr_t>(U) & 15) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(FO_EINVAL, "fo_newton_solve: U must be 16-byte and workspace 256-byte aligned");
  Ctx c;
  c.m = m;
  c.s = static_cast<hipStream_t>(stream);
  c.ws = static_cast<char *>(ws);
  c.L = layout(m, o);
  c.n = m->view.n_dofs;
  if (ws_bytes < c.L.total) return fail(FO_EINVAL, "fo_newton_solve: workspace too small");
  std::memset(rep, 0, sizeof(*rep));
  if (hipHostMalloc(reinterpret_cast<void **>(&c.host), sizeof(double) * 1024) != hipSuccess)
    return fail(FO_ENOMEM, "fo_newton_solve: pinned host buffer");
  struct HostFree { double *p; ~HostFree() { if (p) (void)hipHostFree(p); } } hf{c.host};

  const auto t_start = std::chrono::steady_clock::now();
  double *R = c.dptr(c.L.R), *Rt = c.dptr(c.L.Rt), *Ut = c.dptr(c.L.Ut), *dU = c.dptr(c.L.dU);
  void *Jv = c.ws + c.L.J;
  fo_status st;
  auto fill = [&](const double *Uin, double *Rout) -> fo_status {
    const auto t0 = std::chrono::steady_clock::now();
    fo_status s2 = launch_assemble(m, Uin, Rout, nullptr, FO_F64, FO_JAC_NEWTON, false, c.s);
    if (s2 == FO_OK && hipStreamSynchronize(c.s) != hipSuccess) s2 = fail(FO_EDEVICE, "assembly failed");
    rep->ms_total_fill += ms_since(t0);
    rep->residual_calls++;
    return s2;
  };
  rep->init_used = o->init;
  if (o->init == FO_INIT_SIA && (st = launch_sia(m, U, c.s)) != FO_OK) return st;
  if (o->init == FO_INIT_LEARNED) {
    int32_t used = 0, n_res = 0;
    if ((st = learned_guess(m, o->mlp_params, o->mlp_norm, U, o->learned_fallback, o->learned_smooth,
                            c.ws + c.L.V, c.L.V_bytes, &used, &n_res, c.s)) != FO_OK)
      return st;
    rep->residual_calls += n_res;   // the residual-norm check of the fallback rule
    if (!used) {
      rep->init_used = FO_INIT_SIA;
      rep->learned_fallbacks = 1;
    }
  }
  // ||F(0)||: the gravity load
  if ((st = launch_fill_zero(Ut, sizeof(double) * c.n, c.s)) != FO_OK) return st;
  if ((st = fill(Ut, Rt)) != FO_OK) return st;
  double f0;
  if ((st = norm2(c, Rt, f0)) != FO_OK) return st;
  rep->f0_norm = f0;
  if ((st = fill(U, R)) != FO_OK) return st;
  double nr;
  if ((st = norm2(c, R, nr)) != FO_OK) return st;
  fo_status result = FO_ENOTCONV;
  int it = 0;
  for (;;) {
    if (!std::isfinite(nr)) { result = fail(FO_ENONFINITE, "fo_newton_solve: non-finite residual norm"); break; }
    if (it < 64) rep->res_hist[it] = nr / f0;
    if (nr <= o->tol * f0) { result = FO_OK; break; }
    if (it >= o->max_newton) { result = fail(FO_ENOTCONV, "fo_newton_solve: Newton iteration cap reached"); break; }
    // Total Fill: Jacobian (and residual) at U
    auto t0 = std::chrono::steady_clock::now();
    if ((st = launch_assemble(m, U, R, Jv, o->jac_dtype, FO_JAC_NEWTON, true, c.s)) != FO_OK) return st;
    FO_HIP_TRY(hipStreamSynchronize(c.s));
    rep->ms_total_fill += ms_since(t0);
    rep->jacobian_calls++;
    // Preconditioner Construction
    t0 = std::chrono::steady_clock::now();
    if (o->preconditioner == FO_PREC_MDSC) {
      if ((st = fo_mdsc_setup(o->mdsc, Jv, o->jac_dtype, c.s)) != FO_OK) return st;
    } else if ((st = colblock_factor(m, Jv, o->jac_dtype, reinterpret_cast<float *>(c.ws + c.L.fac), c.s)) != FO_OK) {
      return st;
    }
    FO_HIP_TRY(hipStreamSynchronize(c.s));
    rep->ms_prec_construction += ms_since(t0);
    // Linear Solve: J dU = -R
    t0 = std::chrono::steady_clock::now();
    if ((st = axpby(c.n, -1.0, R, 0.0, Rt, c.s)) != FO_OK) return st;
    int64_t lits = 0;
    double lrel = 0.0;
    if (o->linear_solver == FO_LIN_PCG) {
      if ((st = pcg(c, o, Jv, Rt, dU, lits, lrel)) != FO_OK) return st;
    } else if ((st = gmres(c, o, Jv, Rt, dU, lits, lrel)) != FO_OK) {
      return st;
    }
    rep->ms_linear_solve += ms_since(t0);
    rep->lin_its += lits;
    // backtracking line search
    double alpha = 1.0, nt = 0.0;
    bool accepted = false;
    for (int bt = 0; bt <= o->max_backtracks; ++bt) {
      if ((st = xpay(c.n, U, alpha, dU, Ut, c.s)) != FO_OK) return st;
      if ((st = fill(Ut, Rt)) != FO_OK) return st;
      if ((st = norm2(c, Rt, nt)) != FO_OK) return st;
      if (std::isfinite(nt) && nt <= (1.0 - 1e-4 * alpha) * nr) { accepted = true; break; }
      alpha *= 0.5;
      rep->backtracks++;
    }
    if (!accepted) { result = fail(FO_ENOTCONV, "fo_newton_solve: line search failed"); break; }
    FO_HIP_TRY(hipMemcpyAsync(U, Ut, sizeof(double) * c.n, hipMemcpyDeviceToDevice, c.s));
    FO_HIP_TRY(hipMemcpyAsync(R, Rt, sizeof(double) * c.n, hipMemcpyDeviceToDevice, c.s));
    nr = nt;
    ++it;
  }
  FO_HIP_TRY(hipStreamSynchronize(c.s));
  rep->newton_its = it;
  rep->final_norm = nr;
  rep->final_rel = nr / f0;
  rep->status = result;
  rep->ms_total_solve = ms_since(t_start);
  return result;
}
