// Mesh-derived device work: the Jacobian's CSR pattern (built once at upload) and
// the shallow-ice velocity profile used as the plain Newton initial guess.
#include <hip/hip_runtime.h>

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
  const int nv = m.nv;
  double wsum = 0.0, gxs = 0.0, gys = 0.0;
  for (int p = vc_ptr[v]; p < vc_ptr[v + 1]; ++p) {
    const int t = vc_idx[p];
    double px[4], py[4], ps[4];
    for (int a = 0; a < nv; ++a) {
      const int w = m.cells[int64_t(t) * nv + a];
      const double4 g = m.geo[w];
      px[a] = g.x; py[a] = g.y; ps[a] = m.sb[w].x;
    }
    double gx, gy, area;
    if (nv == 3) {
      const double area2 = (px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]);
      gx = ((ps[1] - ps[0]) * (py[2] - py[0]) - (ps[2] - ps[0]) * (py[1] - py[0])) / area2;
      gy = ((ps[2] - ps[0]) * (px[1] - px[0]) - (ps[1] - ps[0]) * (px[2] - px[0])) / area2;
      area = 0.5 * area2;
    } else {
      // bilinear map at the cell centre: d phi / d(xi, eta)
      const double dxi[4] = {-0.5, 0.5, 0.5, -0.5}, deta[4] = {-0.5, -0.5, 0.5, 0.5};
      double j00 = 0, j01 = 0, j10 = 0, j11 = 0, d0 = 0, d1 = 0;
      for (int a = 0; a < 4; ++a) {
        j00 += px[a] * dxi[a]; j01 += px[a] * deta[a];
        j10 += py[a] * dxi[a]; j11 += py[a] * deta[a];
        d0 += ps[a] * dxi[a];  d1 += ps[a] * deta[a];
      }
      const double det = j00 * j11 - j01 * j10;
      gx = (j11 * d0 - j10 * d1) / det;
      gy = (-j01 * d0 + j00 * d1) / det;
      double sh = 0.0;
      for (int a = 0; a < 4; ++a) sh += px[a] * py[(a + 1) & 3] - px[(a + 1) & 3] * py[a];
      area = 0.5 * fabs(sh);
    }
    wsum += area;
    gxs += area * gx;
    gys += area * gy;
  }
  const double gx = gxs / wsum, gy = gys / wsum;
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
