// Mesh-derived device work: the Jacobian's CSR pattern (built once at upload) and
// the shallow-ice velocity profile used as the plain Newton initial guess.
#include <hip/hip_runtime.h>

#include "fo_device.h"
#include "fo_internal.h"

namespace fo {
namespace {

__device__ __forceinline__ int nlev(int k, int L) { return (k == 0 || k == L) ? 2 : 3; }
__device__ __forceinline__ int cumlev(int k) { return k == 0 ? 0 : 3 * k - 1; }

// One thread per row (dof).  Row (v, k, c) couples every neighbouring column w of v
// (sorted, v included) on levels max(k-1,0)..min(k+1,L), both components.
__global__ void pattern_kernel(MeshView m, const int32_t *__restrict__ nbr_ptr,
                               const int32_t *__restrict__ nbr_idx, int64_t *__restrict__ rowptr,
                               int32_t *__restrict__ colidx) {
  const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= m.n_dofs) return;
  const int L = m.L;
  const int64_t node = row >> 1;
  const int c = int(row & 1);
  const int v = int(node / (L + 1));
  const int k = int(node - int64_t(v) * (L + 1));
  const int D = m.deg[v];
  const int nl = nlev(k, L);
  const int kmin = k > 0 ? k - 1 : 0;
  const int64_t start = m.colptr[v] + int64_t(4) * D * cumlev(k) + int64_t(c) * 2 * nl * D;
  rowptr[row] = start;
  if (row == m.n_dofs - 1) rowptr[m.n_dofs] = m.colptr[m.V];
  int64_t pos = start;
  const int p0 = nbr_ptr[v];
  for (int r = 0; r < D; ++r) {
    const int64_t w = nbr_idx[p0 + r];
    for (int kk = kmin; kk < kmin + nl; ++kk) {
      colidx[pos++] = int32_t(2 * (w * (L + 1) + kk));
      colidx[pos++] = int32_t(2 * (w * (L + 1) + kk) + 1);
    }
  }
}

// One thread per base vertex: area-weighted mean of the adjacent cells' surface
// gradients, then the shallow-ice profile on every level of the column.
__global__ void sia_kernel(MeshView m, const int32_t *__restrict__ vc_ptr,
                           const int32_t *__restrict__ vc_idx, double *__restrict__ U) {
  const int v = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= m.V) return;
  double gx, gy;
  vertex_surface_gradient(m, vc_ptr, vc_idx, v, gx, gy);
  const double4 gv = m.geo[v];
  const double H = gv.w, beta = m.sb[v].y;
  const double n = m.n_glen;
  const double gm = hypot(gx, gy);
  const double drive = m.rho_g * H * gm;
  const double cap = 1e4;
  const bool capped = beta * cap <= drive;
  const double ub = capped ? cap : drive / beta;
  const double dx = gm > 0 ? -gx / gm : 0.0, dy = gm > 0 ? -gy / gm : 0.0;
  const double ubx = ub * dx, uby = ub * dy;
  const double coef = 2.0 * m.A / (n + 1.0) * pow(m.rho_g, n) * pow(gm, n - 1.0);
  const double Hn1 = pow(H, n + 1.0);
  const int L = m.L;
  for (int k = 0; k <= L; ++k) {
    const double depth = H * (1.0 - m.sigma[k]);
    const double shape = Hn1 - pow(depth, n + 1.0);
    const int64_t node = int64_t(v) * (L + 1) + k;
    U[2 * node] = ubx - coef * gx * shape;
    U[2 * node + 1] = uby - coef * gy * shape;
  }
}

}  // namespace

fo_status launch_pattern(const fo_mesh *mesh, hipStream_t s) {
  const MeshView &m = mesh->view;
  const int64_t blocks = (m.n_dofs + 255) / 256;
  hipLaunchKernelGGL(pattern_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, m, mesh->nbr_ptr,
                     mesh->nbr_idx, mesh->rowptr, mesh->colidx);
  FO_LAUNCH_CHECK("pattern_kernel");
  return FO_OK;
}

fo_status launch_sia(const fo_mesh *mesh, double *U, hipStream_t s) {
  const MeshView &m = mesh->view;
  const int blocks = (m.V + 255) / 256;
  hipLaunchKernelGGL(sia_kernel, dim3(blocks), dim3(256), 0, s, m, mesh->vc_ptr, mesh->vc_idx, U);
  FO_LAUNCH_CHECK("sia_kernel");
  return FO_OK;
}

}  // namespace fo
