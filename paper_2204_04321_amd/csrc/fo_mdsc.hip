// Two-level column semicoarsening preconditioner on the device (arXiv:2204.04321 Sec. 3.3:
// vertical coarsening to a single layer with a matrix-dependent prolongator, then aggregation
// AMG on the plane; Sec. 4.4: the prolongator built line by line by LU without pivoting of each
// vertical line's block-tridiagonal system, Chebyshev smoothing on GPUs).
//
// Setup (per Jacobian): column factors (the column preconditioner's own kernel), the collapse
// weights W of every column by an FP64 block-tridiagonal solve with two right-hand sides, then
// one pass over J that forms J P0 and the plane operator P0^T J P0 block by block, the plane
// levels' diagonal inverses and Gershgorin bounds, Galerkin sums through precomputed gather
// lists (fixed order, no atomics) and the coarsest inverse in one workgroup's LDS.
// Application: restrict with W, a V-cycle over the plane levels (Chebyshev before and after
// each coarse correction, degree 2 on the first plane level and 1 below it, each step one
// kernel that forms the residual it needs), then the column smoother on r - J P0 y fused with
// the prolongation P0 y.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fo_mdsc.h"
#include "fo_solver.h"

namespace fo {
namespace {

constexpr int NC_MAX = 2 * kMdscCoarsestMax;   // coarsest dofs held in LDS
constexpr double CHEB_RATIO = 30.0;
enum { FLAG_DIAG = 0, FLAG_COARSE = 1, N_FLAGS = 4 };

__device__ __forceinline__ int nlev(int k, int L) { return (k == 0 || k == L) ? 2 : 3; }
__device__ __forceinline__ int cumlev(int k) { return k == 0 ? 0 : 3 * k - 1; }

// 2x2 helpers, [2 r + c]
__device__ __forceinline__ void mul22(const double *a, const double *b, double *o) {
  o[0] = a[0] * b[0] + a[1] * b[2];
  o[1] = a[0] * b[1] + a[1] * b[3];
  o[2] = a[2] * b[0] + a[3] * b[2];
  o[3] = a[2] * b[1] + a[3] * b[3];
}

// Collapse weights of one vertex column per thread.  Forward: S_k = D_k - Lo_k G_{k-1},
// G_k = S_k^-1 Up_k, Y_k = S_k^-1 (I - Lo_k Y_{k-1}) for the two right-hand sides e_u, e_v at
// once (Y_k is 2x2: rows the level's components, columns the right-hand sides); backward
// Z_k = Y_k - G_k Z_{k+1}; then each right-hand side's solution is divided by the mean of its
// own component over the levels (e_c itself where that is not usable).  The block's columns
// (4 (L+1) values each, G and Y/Z) live in LDS and leave with coalesced stores, in FP64 and
// rounded to FP32.
template <class JT>
__global__ __launch_bounds__(64) void weights_kernel(MeshView m, const int32_t *__restrict__ self_rank,
                                                     const JT *__restrict__ J, double *__restrict__ W,
                                                     float *__restrict__ W32) {
  extern __shared__ double wsh[];   // [2][blockDim.x][4 (L + 1)]: Z then G
  const int L = m.L, nw = 4 * (L + 1);
  const int64_t v0 = int64_t(blockIdx.x) * blockDim.x;
  const int nv = int(m.V - v0 < int64_t(blockDim.x) ? m.V - v0 : int64_t(blockDim.x));
  if (int(threadIdx.x) < nv) {
    const int64_t v = v0 + threadIdx.x;
    const int D = m.deg[v], sr = self_rank[v];
    const int64_t base = m.colptr[v];
    double *Wv = wsh + threadIdx.x * nw;
    double *Gv = wsh + (blockDim.x + threadIdx.x) * nw;
    double Gp[4] = {0, 0, 0, 0}, Yp[4] = {0, 0, 0, 0};
    for (int k = 0; k <= L; ++k) {
      const int nl = nlev(k, L), kmin = k > 0 ? k - 1 : 0;
      double Dk[4], Lo[4] = {0, 0, 0, 0}, Up[4] = {0, 0, 0, 0};
      for (int c = 0; c < 2; ++c) {
        const int64_t row = base + int64_t(4) * D * cumlev(k) + int64_t(c) * 2 * nl * D + int64_t(sr) * 2 * nl;
        for (int d = 0; d < 2; ++d) {
          Dk[2 * c + d] = double(J[row + 2 * (k - kmin) + d]);
          if (k > 0) Lo[2 * c + d] = double(J[row + 2 * (k - 1 - kmin) + d]);
          if (k < L) Up[2 * c + d] = double(J[row + 2 * (k + 1 - kmin) + d]);
        }
      }
      double T[4] = {1, 0, 0, 1};
      if (k > 0) {
        double t[4];
        mul22(Lo, Gp, t);
        for (int i = 0; i < 4; ++i) Dk[i] -= t[i];
        mul22(Lo, Yp, t);
        for (int i = 0; i < 4; ++i) T[i] -= t[i];
      }
      const double det = Dk[0] * Dk[3] - Dk[1] * Dk[2];
      const double Si[4] = {Dk[3] / det, -Dk[1] / det, -Dk[2] / det, Dk[0] / det};
      mul22(Si, Up, Gp);
      mul22(Si, T, Yp);
      for (int i = 0; i < 4; ++i) {
        Gv[4 * k + i] = Gp[i];
        Wv[4 * k + i] = Yp[i];
      }
    }
    double Z[4] = {Wv[4 * L], Wv[4 * L + 1], Wv[4 * L + 2], Wv[4 * L + 3]};
    for (int k = L - 1; k >= 0; --k) {
      const double G[4] = {Gv[4 * k], Gv[4 * k + 1], Gv[4 * k + 2], Gv[4 * k + 3]};
      double t[4];
      mul22(G, Z, t);
      for (int i = 0; i < 4; ++i) {
        Z[i] = Wv[4 * k + i] - t[i];
        Wv[4 * k + i] = Z[i];
      }
    }
    for (int c = 0; c < 2; ++c) {
      double sum = 0.0;
      bool finite = true;
      for (int k = 0; k <= L; ++k) {
        sum += Wv[4 * k + 2 * c + c];
        finite = finite && isfinite(Wv[4 * k + c]) && isfinite(Wv[4 * k + 2 + c]);
      }
      const double mean = sum / double(L + 1);
      const bool ok = finite && isfinite(mean) && mean > 0.0;
      for (int k = 0; k <= L; ++k)
        for (int cp = 0; cp < 2; ++cp)
          Wv[4 * k + 2 * cp + c] = ok ? Wv[4 * k + 2 * cp + c] / mean : (cp == c ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nv * nw; e += blockDim.x) {
    const double w = wsh[e];
    W[v0 * nw + e] = w;
    W32[v0 * nw + e] = float(w);
  }
}

// One thread per plane block e = (v, neighbour r = w): the rows of J P0 of column v against
// column w, T[(k, c')][d] = sum over the levels l of J_{(v,k,c'),(w,l,d')} W_w[l][d'][d], and
// the block A_0[v][w][c][d] = sum_k sum_c' W_v[k][c'][c] T[(k, c')][d] from the FP64 values.
// J P0 is stored in FP32 by block: entry d of row q of block e at (2 e + d) 2 (L+1) + q (for a
// column, entry (r, d) of row q at (2 (nbr_ptr[v] + r) + d) 2 (L+1) + q), so a workgroup's
// blocks own one contiguous range, staged in LDS and written with coalesced stores.
template <class JT>
__global__ __launch_bounds__(256) void plane_kernel(MeshView m, const int32_t *__restrict__ nbr_ptr,
                                                    const int32_t *__restrict__ nbr_idx,
                                                    const int32_t *__restrict__ blk_row, int32_t nnzb,
                                                    const JT *__restrict__ J, const double *__restrict__ W,
                                                    float *__restrict__ JP, double *__restrict__ A0) {
  extern __shared__ float jsh[];   // [blockDim.x][2][2 (L + 1)]
  const int L = m.L, nb = 2 * (L + 1);
  const int e0 = int(blockIdx.x) * blockDim.x, e = e0 + threadIdx.x;
  const int ne = nnzb - e0 < int(blockDim.x) ? nnzb - e0 : int(blockDim.x);
  if (e < nnzb) {
    const int v = blk_row[e], nb0 = nbr_ptr[v], r = e - nb0, D = nbr_ptr[v + 1] - nb0, w = nbr_idx[e];
    const int64_t base = m.colptr[v];
    const double *Wv = W + int64_t(v) * (L + 1) * 4, *Ww = W + int64_t(w) * (L + 1) * 4;
    float *J0 = jsh + threadIdx.x * 2 * nb, *J1 = J0 + nb;
    double a[4] = {0, 0, 0, 0};
    for (int k = 0; k <= L; ++k) {
      const int nl = nlev(k, L), klo = k > 0 ? k - 1 : 0;
      double T[4] = {0, 0, 0, 0};
      for (int cp = 0; cp < 2; ++cp) {
        const int64_t row = base + int64_t(4) * D * cumlev(k) + int64_t(cp) * 2 * nl * D + int64_t(r) * 2 * nl;
        for (int lev = 0; lev < nl; ++lev) {
          const double j0 = double(J[row + 2 * lev]), j1 = double(J[row + 2 * lev + 1]);
          const double *wl = Ww + 4 * (klo + lev);
          T[2 * cp] += j0 * wl[0] + j1 * wl[2];
          T[2 * cp + 1] += j0 * wl[1] + j1 * wl[3];
        }
        J0[2 * k + cp] = float(T[2 * cp]);
        J1[2 * k + cp] = float(T[2 * cp + 1]);
      }
      const double *wv = Wv + 4 * k;
      for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) a[2 * c + d] += wv[c] * T[d] + wv[2 + c] * T[2 + d];
    }
    for (int i = 0; i < 4; ++i) A0[4 * int64_t(e) + i] = a[i];
  }
  __syncthreads();
  float *out = JP + int64_t(2) * nb * e0;
  for (int t = threadIdx.x; t < ne * 2 * nb; t += blockDim.x) out[t] = jsh[t];
}

// Diagonal-block inverse of every plane vertex and its Gershgorin row bound
// max over its two rows of sum_w |(D_v^-1 A_vw)| (entries of both columns).
__global__ __launch_bounds__(256) void diag_kernel(int n, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ diag, const double *__restrict__ A,
                                                   double *__restrict__ Dinv, double *__restrict__ bound,
                                                   int32_t *__restrict__ flag) {
  const int v = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double *a = A + 4 * int64_t(diag[v]);
  const double det = a[0] * a[3] - a[1] * a[2];
  double di[4] = {a[3] / det, -a[1] / det, -a[2] / det, a[0] / det};
  double s0 = 0.0, s1 = 0.0;
  for (int e = ptr[v]; e < ptr[v + 1]; ++e) {
    const double *b = A + 4 * int64_t(e);
    double t[4];
    mul22(di, b, t);
    s0 += fabs(t[0]) + fabs(t[1]);
    s1 += fabs(t[2]) + fabs(t[3]);
  }
  bool ok = det != 0.0 && isfinite(det);
  for (int i = 0; i < 4; ++i) ok = ok && isfinite(di[i]);
  if (!ok) {
    flag[FLAG_DIAG] = 1;
    for (int i = 0; i < 4; ++i) di[i] = 0.0;
  }
  for (int i = 0; i < 4; ++i) Dinv[4 * int64_t(v) + i] = di[i];
  bound[v] = ok ? fmax(s0, s1) : 0.0;
}

// g = max of the row bounds (one workgroup); a bound that is not a positive finite number
// marks the setup as failed.
__global__ __launch_bounds__(1024) void max_kernel(int n, const double *__restrict__ x, double *__restrict__ out,
                                                   int32_t *__restrict__ flag) {
  __shared__ double sh[1024];
  double mx = 0.0;
  bool bad = false;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double t = x[i];
    bad = bad || !isfinite(t);
    mx = t > mx ? t : mx;
  }
  sh[threadIdx.x] = bad ? -1.0 : mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      const double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
      sh[threadIdx.x] = (a < 0.0 || b < 0.0) ? -1.0 : (a > b ? a : b);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sh[0];
    if (!(sh[0] > 0.0)) flag[FLAG_DIAG] = 1;
  }
}

// Galerkin operator of unsmoothed aggregation: every coarse block is the sum of the fine
// blocks listed for it (ascending fine index).
__global__ __launch_bounds__(256) void galerkin_kernel(int nnz_c, const int32_t *__restrict__ gptr,
                                                       const int32_t *__restrict__ gidx, const double *__restrict__ Af,
                                                       double *__restrict__ Ac) {
  const int c = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nnz_c) return;
  double s[4] = {0, 0, 0, 0};
  for (int i = gptr[c]; i < gptr[c + 1]; ++i) {
    const double4 b = reinterpret_cast<const double4 *>(Af)[gidx[i]];
    s[0] += b.x;
    s[1] += b.y;
    s[2] += b.z;
    s[3] += b.w;
  }
  reinterpret_cast<double4 *>(Ac)[c] = make_double4(s[0], s[1], s[2], s[3]);
}

// Inverse of the coarsest operator (nc = 2 n <= NC_MAX dofs) by Gauss-Jordan elimination with
// partial (row) pivoting in LDS, one workgroup: for each column k the pivot row is swapped
// in, scaled, and eliminated from every other row; the column swaps that undo the row
// pivoting are applied in reverse order at the end.  Written column-major.
__global__ __launch_bounds__(1024) void coarse_inverse_kernel(int n, const int32_t *__restrict__ ptr,
                                                             const int32_t *__restrict__ idx,
                                                             const double *__restrict__ A, double *__restrict__ Ainv,
                                                             int32_t *__restrict__ flag) {
  __shared__ double a[NC_MAX * NC_MAX];
  __shared__ double fcol[NC_MAX];
  __shared__ int perm[NC_MAX];
  __shared__ int piv_row;
  const int nc = 2 * n, tid = threadIdx.x, bd = blockDim.x;
  for (int t = tid; t < nc * nc; t += bd) a[t] = 0.0;
  __syncthreads();
  for (int v = tid; v < n; v += bd)
    for (int e = ptr[v]; e < ptr[v + 1]; ++e) {
      const int w = idx[e];
      for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) a[(2 * v + c) * nc + 2 * w + d] = A[4 * int64_t(e) + 2 * c + d];
    }
  __syncthreads();
  bool singular = false;
  for (int k = 0; k < nc; ++k) {
    if (tid < 64) {   // pivot search: largest |a[i][k]|, i >= k, lowest row on ties
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < nc; i += 64) {
        const double t = fabs(a[i * nc + k]);
        if (t > best) { best = t; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) { piv_row = bi; perm[k] = bi; }
    }
    __syncthreads();
    const int p = piv_row;
    if (p != k)
      for (int j = tid; j < nc; j += bd) {
        const double t = a[k * nc + j];
        a[k * nc + j] = a[p * nc + j];
        a[p * nc + j] = t;
      }
    __syncthreads();
    const double piv = a[k * nc + k];
    if (!(piv != 0.0) || !isfinite(piv)) { singular = true; break; }   // the same for every thread
    __syncthreads();
    for (int j = tid; j < nc; j += bd) a[k * nc + j] = (j == k ? 1.0 : a[k * nc + j]) / piv;
    for (int i = tid; i < nc; i += bd) fcol[i] = i == k ? 0.0 : a[i * nc + k];
    __syncthreads();
    for (int i = tid >> 4; i < nc; i += bd >> 4) {   // 16 threads per row group, no divisions
      if (i == k) continue;
      const double f = fcol[i];
      for (int j = tid & 15; j < nc; j += 16) a[i * nc + j] = (j == k ? 0.0 : a[i * nc + j]) - f * a[k * nc + j];
    }
    __syncthreads();
  }
  if (singular) {
    if (tid == 0) flag[FLAG_COARSE] = 1;
    return;
  }
  for (int k = nc - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < nc; i += bd) {
        const double t = a[i * nc + k];
        a[i * nc + k] = a[i * nc + p];
        a[i * nc + p] = t;
      }
    __syncthreads();
  }
  for (int t = tid; t < nc * nc; t += bd) Ainv[t] = a[t];
}

// ---- application ------------------------------------------------------------------------

struct Cheb {
  double inv_theta, c1, c2;
};

// Degree-2 Chebyshev coefficients over [g / ratio, g]: d_0 = D^-1 r_0 / theta and
// d_1 = rho_1 rho_0 d_0 + 2 rho_1 / delta D^-1 r_1.
__device__ __forceinline__ Cheb cheb_coeffs(double g) {
  const double lo = g / CHEB_RATIO;
  const double theta = 0.5 * (g + lo), delta = 0.5 * (g - lo);
  const double sigma = theta / delta, rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
  return {1.0 / theta, rho1 * rho0, 2.0 * rho1 / delta};
}

__device__ __forceinline__ double2 apply22(const double *Dv, double2 x) {
  return make_double2(Dv[0] * x.x + Dv[1] * x.y, Dv[2] * x.x + Dv[3] * x.y);
}

// b_0[(v, c)] = sum over the column's levels and components of W[v][k][c'][c] r[(v, k, c')].
// The products of a block of columns are staged in LDS (coalesced loads of r and of the FP32
// weights, whose two columns c sit next to each other for every row), then one thread per
// (column, c) sums its column's rows in level order.
__global__ __launch_bounds__(128) void restrict_fine_kernel(int V, int L, int cols, const float *__restrict__ W32,
                                                            const double *__restrict__ r, double *__restrict__ b0) {
  extern __shared__ double rsh[];   // [2][cols][2 (L + 1)]
  const int nb = 2 * (L + 1);
  const int64_t v0 = int64_t(blockIdx.x) * cols;
  const int nv = int(V - v0 < int64_t(cols) ? V - v0 : int64_t(cols));
  const float2 *W2 = reinterpret_cast<const float2 *>(W32);
  for (int e = threadIdx.x; e < nv * nb; e += blockDim.x) {
    const float2 w = W2[v0 * nb + e];
    const double rv = r[v0 * nb + e];
    rsh[e] = double(w.x) * rv;
    rsh[cols * nb + e] = double(w.y) * rv;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 2 * nv; t += blockDim.x) {
    const int v = t >> 1, c = t & 1;
    const double *p = rsh + c * cols * nb + v * nb;
    double sum = 0.0;
    for (int q = 0; q < nb; ++q) sum += p[q];
    b0[2 * (v0 + v) + c] = sum;
  }
}

// The V-cycle's kernels.  The first plane level smooths with Chebyshev of degree 2 (x kept
// between the steps), the coarser ones with degree 1, whose pre-smoothed value from zero,
// x1 = D^-1 b / theta, is formed wherever it is needed instead of stored.  A vertex's row
// blocks are taken by G = 8 lanes (consecutive blocks, coalesced 32-byte loads) and summed
// with shuffles; the restriction takes one wave per aggregate.
constexpr int G = 8;

// x1 of vertex w: D_w^-1 b_w / theta
__device__ __forceinline__ double2 x1_of(const LevelDev &P, int w, double inv_theta) {
  const double2 t = apply22(P.Dinv + 4 * int64_t(w), reinterpret_cast<const double2 *>(P.b)[w]);
  return make_double2(t.x * inv_theta, t.y * inv_theta);
}

// partial sums of A_vw u_w over this lane's blocks of row v
template <class U>
__device__ __forceinline__ double2 row_partial(const LevelDev &P, int v, int sub, U u) {
  double2 s = make_double2(0.0, 0.0);
  for (int e = P.ptr[v] + sub; e < P.ptr[v + 1]; e += G) {
    const double2 xw = u(P.idx[e]);
    const double4 a = reinterpret_cast<const double4 *>(P.A)[e];
    s.x += a.x * xw.x + a.y * xw.y;
    s.y += a.z * xw.x + a.w * xw.y;
  }
  return s;
}

__device__ __forceinline__ double2 group_sum(double2 s) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    s.x += __shfl_xor(s.x, off, G);
    s.y += __shfl_xor(s.y, off, G);
  }
  return s;
}

// Degree-2 pre-smoothing from x = 0 on the first level: x1 = D^-1 b / theta,
// x = x1 + c1 x1 + c2 D^-1 (b - A x1).
__global__ __launch_bounds__(256) void pre2_kernel(const LevelDev *__restrict__ lv, int l) {
  const LevelDev P = lv[l];
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int v = int(gid / G), sub = int(gid % G);
  const Cheb ch = cheb_coeffs(P.g[0]);
  double2 s = make_double2(0.0, 0.0);
  if (v < P.n) s = row_partial(P, v, sub, [&](int w) { return x1_of(P, w, ch.inv_theta); });
  s = group_sum(s);
  if (v < P.n && sub == 0) {
    const double2 b = reinterpret_cast<const double2 *>(P.b)[v];
    const double2 ds = apply22(P.Dinv + 4 * int64_t(v), make_double2(b.x - s.x, b.y - s.y));
    const double2 x1 = x1_of(P, v, ch.inv_theta);
    reinterpret_cast<double2 *>(P.x)[v] =
        make_double2(x1.x + (ch.c1 * x1.x + ch.c2 * ds.x), x1.y + (ch.c1 * x1.y + ch.c2 * ds.y));
  }
}

// Residual and restriction in one pass, one wave per aggregate a of the next level:
// b_C[a] = sum over the members v of (b_v - A_v x), x the pre-smoothed vector (stored for
// degree 2, x1 formed on the fly for degree 1).  Lanes take (member, block) pairs, 8 members
// and 8 blocks per pass.
template <int DEG>
__global__ __launch_bounds__(256) void resid_restrict_kernel(const LevelDev *__restrict__ lv, int l) {
  const LevelDev P = lv[l], C = lv[l + 1];
  const int a = int((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63, mi = lane / G, sub = lane % G;
  double2 s = make_double2(0.0, 0.0);
  if (a < C.n) {
    const double inv_theta = DEG == 2 ? 0.0 : cheb_coeffs(P.g[0]).inv_theta;
    const double2 *x2 = reinterpret_cast<const double2 *>(P.x);
    for (int i = P.mptr[a] + mi; i < P.mptr[a + 1]; i += 64 / G) {
      const int v = P.midx[i];
      double2 t;
      if constexpr (DEG == 2) t = row_partial(P, v, sub, [&](int w) { return x2[w]; });
      else t = row_partial(P, v, sub, [&](int w) { return x1_of(P, w, inv_theta); });
      if (sub == 0) {
        const double2 b = reinterpret_cast<const double2 *>(P.b)[v];
        t.x -= b.x;
        t.y -= b.y;
      }
      s.x -= t.x;
      s.y -= t.y;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s.x += __shfl_xor(s.x, off, 64);
    s.y += __shfl_xor(s.y, off, 64);
  }
  if (a < C.n && lane == 0) reinterpret_cast<double2 *>(C.b)[a] = s;
}

// Prolongation and the first post-smoothing step: x' = x + x_C[agg], d = D^-1 (b - A x') / theta,
// x_out = x' + d (x' of the neighbours formed on the fly; x is x1 for degree 1).  Degree 2
// writes x2 and d for the second step; degree 1 writes the level's final x.
template <int DEG>
__global__ __launch_bounds__(256) void post0_kernel(const LevelDev *__restrict__ lv, int l) {
  const LevelDev P = lv[l], C = lv[l + 1];
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int v = int(gid / G), sub = int(gid % G);
  const Cheb ch = cheb_coeffs(P.g[0]);
  const double2 *xv2 = reinterpret_cast<const double2 *>(P.x);
  const double2 *xc2 = reinterpret_cast<const double2 *>(C.x);
  auto xp = [&](int w) {
    const double2 xw = DEG == 2 ? xv2[w] : x1_of(P, w, ch.inv_theta);
    const double2 cw = xc2[P.agg[w]];
    return make_double2(xw.x + cw.x, xw.y + cw.y);
  };
  double2 s = make_double2(0.0, 0.0);
  if (v < P.n) s = row_partial(P, v, sub, xp);
  s = group_sum(s);
  if (v < P.n && sub == 0) {
    const double2 b = reinterpret_cast<const double2 *>(P.b)[v];
    const double2 dv = apply22(P.Dinv + 4 * int64_t(v), make_double2(b.x - s.x, b.y - s.y));
    const double dx = dv.x * ch.inv_theta, dy = dv.y * ch.inv_theta;
    const double2 xo = xp(v);
    const double2 out = make_double2(xo.x + dx, xo.y + dy);
    if constexpr (DEG == 2) {
      reinterpret_cast<double2 *>(P.x2)[v] = out;
      reinterpret_cast<double2 *>(P.d)[v] = make_double2(dx, dy);
    } else {
      reinterpret_cast<double2 *>(P.x)[v] = out;
    }
  }
}

// Second degree-2 post-smoothing step: x = x2 + c1 d + c2 D^-1 (b - A x2).
__global__ __launch_bounds__(256) void post1_kernel(const LevelDev *__restrict__ lv, int l) {
  const LevelDev P = lv[l];
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int v = int(gid / G), sub = int(gid % G);
  const Cheb ch = cheb_coeffs(P.g[0]);
  const double2 *xv2 = reinterpret_cast<const double2 *>(P.x2);
  double2 s = make_double2(0.0, 0.0);
  if (v < P.n) s = row_partial(P, v, sub, [&](int w) { return xv2[w]; });
  s = group_sum(s);
  if (v < P.n && sub == 0) {
    const double2 b = reinterpret_cast<const double2 *>(P.b)[v];
    const double2 ds = apply22(P.Dinv + 4 * int64_t(v), make_double2(b.x - s.x, b.y - s.y));
    const double2 dv = reinterpret_cast<const double2 *>(P.d)[v];
    const double2 xo = xv2[v];
    reinterpret_cast<double2 *>(P.x)[v] =
        make_double2(xo.x + (ch.c1 * dv.x + ch.c2 * ds.x), xo.y + (ch.c1 * dv.y + ch.c2 * ds.y));
  }
}

// x = Ainv b on the coarsest level: one wave per row of the row-major inverse, lanes over its
// columns, a shuffle sum per row.
__global__ __launch_bounds__(1024) void coarse_solve_kernel(const LevelDev *__restrict__ lv, int last,
                                                            const double *__restrict__ Ainv) {
  const LevelDev C = lv[last];
  const int nc = 2 * C.n, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int i = wave; i < nc; i += nwave) {
    double sum = 0.0;
    for (int j = lane; j < nc; j += 64) sum += Ainv[int64_t(i) * nc + j] * C.b[j];
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (lane == 0) C.x[i] = sum;
  }
}

unsigned blocks_for(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace
}  // namespace fo

using namespace fo;

static void free_mdsc(fo_mdsc *p) {
  if (!p) return;
  auto F = [](void *q) { if (q) (void)hipFree(q); };
  for (PlaneLevel &l : p->lv) {
    F(l.own_ptr); F(l.own_idx); F(l.diag); F(l.A); F(l.Dinv); F(l.bound); F(l.g); F(l.agg);
    F(l.mptr); F(l.midx); F(l.gptr); F(l.gidx); F(l.b); F(l.x); F(l.x2); F(l.d);
  }
  F(p->blk_row); F(p->lv_dev); F(p->fac); F(p->W); F(p->W32); F(p->JP); F(p->Ainv); F(p->flag);
  if (p->flag_host) (void)hipHostFree(p->flag_host);
  delete p;
}

namespace {
template <class T>
bool dev_alloc(T *&p, size_t count) {
  return hipMalloc(reinterpret_cast<void **>(&p), sizeof(T) * std::max<size_t>(count, 1)) == hipSuccess;
}
template <class T>
bool upload(T *&p, const std::vector<T> &h, hipStream_t s) {
  if (!dev_alloc(p, h.size())) return false;
  return h.empty() || hipMemcpyAsync(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s) == hipSuccess;
}
}  // namespace

extern "C" fo_status fo_mdsc_create(const fo_mesh *m, void *stream, fo_mdsc **out) {
  if (!out) return fail(FO_EINVAL, "fo_mdsc_create: out is NULL");
  *out = nullptr;
  if (!m) return fail(FO_EINVAL, "fo_mdsc_create: mesh is NULL");
  int dev = -1;
  FO_HIP_TRY(hipGetDevice(&dev));
  if (dev != m->device) return fail(FO_EINVAL, "fo_mdsc_create: the mesh's device must be current");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int V = m->view.V, L = m->view.L;
  std::vector<int32_t> ptr(static_cast<size_t>(V) + 1), self(static_cast<size_t>(V));
  FO_HIP_TRY(hipStreamSynchronize(s));
  FO_HIP_TRY(hipMemcpy(ptr.data(), m->nbr_ptr, sizeof(int32_t) * (V + 1), hipMemcpyDeviceToHost));
  std::vector<int32_t> idx(static_cast<size_t>(ptr[V]));
  FO_HIP_TRY(hipMemcpy(idx.data(), m->nbr_idx, sizeof(int32_t) * ptr[V], hipMemcpyDeviceToHost));
  FO_HIP_TRY(hipMemcpy(self.data(), m->self_rank, sizeof(int32_t) * V, hipMemcpyDeviceToHost));

  fo_mdsc *p = new fo_mdsc();
  p->mesh = m;
  p->device = dev;
  auto bail = [&](fo_status st, const std::string &msg) { free_mdsc(p); return fail(st, msg); };
  // symbolic hierarchy on the host
  std::vector<PlaneTables> tabs;
  p->lv.emplace_back();
  p->lv[0].ptr_h = ptr;
  p->lv[0].idx_h = idx;
  while (p->lv.back().ptr_h.size() - 1 > size_t(kMdscCoarsestMax)) {
    if (int(p->lv.size()) >= kMdscMaxLevels) return bail(FO_EINVAL, "fo_mdsc_create: aggregation did not coarsen");
    PlaneLevel &f = p->lv.back();
    const int32_t n_agg = aggregate_graph(f.ptr_h, f.idx_h, f.agg_h);
    tabs.emplace_back();
    coarse_tables(f.ptr_h, f.idx_h, f.agg_h, n_agg, tabs.back());
    PlaneLevel c;
    c.ptr_h = tabs.back().cptr;
    c.idx_h = tabs.back().cidx;
    p->lv.push_back(std::move(c));
  }
  const size_t last = p->lv.size() - 1;
  // device arrays
  for (size_t l = 0; l <= last; ++l) {
    PlaneLevel &q = p->lv[l];
    q.n = int32_t(q.ptr_h.size()) - 1;
    q.nnzb = q.ptr_h[q.n];
    std::vector<int32_t> diag(static_cast<size_t>(q.n));
    for (int32_t v = 0; v < q.n; ++v)
      diag[v] = l == 0 ? ptr[v] + self[v]
                       : int32_t(std::lower_bound(q.idx_h.begin() + q.ptr_h[v], q.idx_h.begin() + q.ptr_h[v + 1], v) -
                                 q.idx_h.begin());
    bool ok = true;
    if (l == 0) {
      q.ptr = m->nbr_ptr;
      q.idx = m->nbr_idx;
    } else {
      ok = ok && upload(q.own_ptr, q.ptr_h, s) && upload(q.own_idx, q.idx_h, s);
      q.ptr = q.own_ptr;
      q.idx = q.own_idx;
    }
    ok = ok && upload(q.diag, diag, s) && dev_alloc(q.A, 4 * size_t(q.nnzb)) && dev_alloc(q.b, 2 * size_t(q.n)) &&
         dev_alloc(q.x, 2 * size_t(q.n));
    if (l < last) {
      const PlaneTables &t = tabs[l];
      ok = ok && dev_alloc(q.Dinv, 4 * size_t(q.n)) && dev_alloc(q.bound, size_t(q.n)) && dev_alloc(q.g, 1) &&
           (l > 0 || (dev_alloc(q.x2, 2 * size_t(q.n)) && dev_alloc(q.d, 2 * size_t(q.n)))) &&
           upload(q.agg, q.agg_h, s) && upload(q.mptr, t.mptr, s) && upload(q.midx, t.midx, s) &&
           upload(q.gptr, t.gptr, s) && upload(q.gidx, t.gidx, s);
    }
    if (!ok) return bail(FO_ENOMEM, "fo_mdsc_create: device allocation failed");
  }
  std::vector<int32_t> blk_row(static_cast<size_t>(ptr[V]));
  for (int32_t v = 0; v < V; ++v)
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e) blk_row[e] = v;
  const size_t nodes = size_t(V) * size_t(L + 1);
  const int nc = 2 * p->lv[last].n;
  p->jp_count = size_t(2 * (L + 1)) * 2 * size_t(ptr[V]);
  // device views of the levels
  std::vector<LevelDev> views(p->lv.size());
  for (size_t l = 0; l <= last; ++l) {
    const PlaneLevel &q = p->lv[l];
    views[l] = LevelDev{q.n, q.ptr, q.idx, q.agg, q.mptr, q.midx, q.A, q.Dinv, q.g, q.b, q.x, q.x2, q.d};
  }
  if (!upload(p->blk_row, blk_row, s) || !upload(p->lv_dev, views, s) || !dev_alloc(p->fac, 12 * nodes) ||
      !dev_alloc(p->W, 4 * nodes) || !dev_alloc(p->W32, 4 * nodes) || !dev_alloc(p->JP, p->jp_count) ||
      !dev_alloc(p->Ainv, size_t(nc) * nc) || !dev_alloc(p->flag, N_FLAGS))
    return bail(FO_ENOMEM, "fo_mdsc_create: device allocation failed");
  if (hipHostMalloc(reinterpret_cast<void **>(&p->flag_host), sizeof(int32_t) * N_FLAGS) != hipSuccess)
    return bail(FO_ENOMEM, "fo_mdsc_create: pinned allocation failed");
  if (hipStreamSynchronize(s) != hipSuccess) return bail(FO_EDEVICE, "fo_mdsc_create: upload failed");
  *out = p;
  return FO_OK;
}

extern "C" void fo_mdsc_destroy(fo_mdsc *p) { free_mdsc(p); }

extern "C" fo_status fo_mdsc_levels(const fo_mdsc *p, int32_t *n_levels, int32_t *n_verts) {
  if (!p) return fail(FO_EINVAL, "fo_mdsc_levels: NULL object");
  if (n_levels) *n_levels = int32_t(p->lv.size()) - 1;
  if (n_verts)
    for (size_t l = 0; l < p->lv.size(); ++l) n_verts[l] = p->lv[l].n;
  return FO_OK;
}

extern "C" fo_status fo_mdsc_graph(const fo_mdsc *p, int32_t level, int32_t *ptr, int32_t *idx, int32_t *agg) {
  if (!p || level < 0 || level >= int32_t(p->lv.size())) return fail(FO_EINVAL, "fo_mdsc_graph: bad object or level");
  const PlaneLevel &q = p->lv[level];
  if (agg && level == int32_t(p->lv.size()) - 1) return fail(FO_EINVAL, "fo_mdsc_graph: the coarsest level has no aggregates");
  if (ptr) std::copy(q.ptr_h.begin(), q.ptr_h.end(), ptr);
  if (idx) std::copy(q.idx_h.begin(), q.idx_h.end(), idx);
  if (agg) std::copy(q.agg_h.begin(), q.agg_h.end(), agg);
  return FO_OK;
}

namespace {
template <class JT>
fo_status setup_t(fo_mdsc *p, const JT *J, hipStream_t s) {
  const fo_mesh *m = p->mesh;
  const MeshView &mv = m->view;
  const PlaneLevel &l0 = p->lv[0];
  // columns per block: the block's weights and factors (8 (L+1) doubles per column) within 64 KB of LDS
  const size_t col_bytes = size_t(8) * (mv.L + 1) * sizeof(double);
  int cols = 64;
  while (cols > 1 && cols * col_bytes > 65536) cols /= 2;
  hipLaunchKernelGGL(weights_kernel<JT>, dim3(blocks_for(mv.V, cols)), dim3(cols), cols * col_bytes, s, mv,
                     m->self_rank, J, p->W, p->W32);
  FO_LAUNCH_CHECK("mdsc weights");
  // blocks per workgroup: their J P0 rows (4 (L+1) floats each) within 64 KB of LDS
  const size_t blk_bytes = size_t(4) * (mv.L + 1) * sizeof(float);
  int tpb = 256;
  while (tpb > 1 && tpb * blk_bytes > 65536) tpb /= 2;
  hipLaunchKernelGGL(plane_kernel<JT>, dim3(blocks_for(l0.nnzb, tpb)), dim3(tpb), tpb * blk_bytes, s, mv, m->nbr_ptr,
                     m->nbr_idx, p->blk_row, l0.nnzb, J, p->W, p->JP, l0.A);
  FO_LAUNCH_CHECK("mdsc plane");
  return FO_OK;
}
}  // namespace

extern "C" fo_status fo_mdsc_setup(fo_mdsc *p, const void *J, int32_t dtype, void *stream) {
  if (!p || !J) return fail(FO_EINVAL, "fo_mdsc_setup: NULL argument");
  if (dtype != FO_F64 && dtype != FO_F32) return fail(FO_EINVAL, "fo_mdsc_setup: bad dtype");
  hipStream_t s = static_cast<hipStream_t>(stream);
  p->ready = false;
  fo_status st;
  if ((st = launch_fill_zero(p->flag, sizeof(int32_t) * N_FLAGS, s)) != FO_OK) return st;
  if ((st = colblock_factor(p->mesh, J, dtype, p->fac, s)) != FO_OK) return st;
  st = dtype == FO_F64 ? setup_t(p, static_cast<const double *>(J), s) : setup_t(p, static_cast<const float *>(J), s);
  if (st != FO_OK) return st;
  const size_t last = p->lv.size() - 1;
  for (size_t l = 0; l < last; ++l) {
    PlaneLevel &q = p->lv[l];
    hipLaunchKernelGGL(diag_kernel, dim3(blocks_for(q.n, 256)), dim3(256), 0, s, q.n, q.ptr, q.diag, q.A, q.Dinv,
                       q.bound, p->flag);
    FO_LAUNCH_CHECK("mdsc diag");
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, q.n, q.bound, q.g, p->flag);
    FO_LAUNCH_CHECK("mdsc bound");
    const PlaneLevel &c = p->lv[l + 1];
    hipLaunchKernelGGL(galerkin_kernel, dim3(blocks_for(c.nnzb, 256)), dim3(256), 0, s, c.nnzb, q.gptr, q.gidx, q.A,
                       c.A);
    FO_LAUNCH_CHECK("mdsc galerkin");
  }
  const PlaneLevel &c = p->lv[last];
  // 1024 threads: the elimination's LDS loads depend on the stores before them, so each
  // thread's short chain of entries is latency-bound (64 threads: 350 us, 256: 149 us, 1024: 101 us)
  hipLaunchKernelGGL(coarse_inverse_kernel, dim3(1), dim3(1024), 0, s, c.n, c.ptr, c.idx, c.A, p->Ainv, p->flag);
  FO_LAUNCH_CHECK("mdsc coarse inverse");
  FO_HIP_TRY(hipMemcpyAsync(p->flag_host, p->flag, sizeof(int32_t) * N_FLAGS, hipMemcpyDeviceToHost, s));
  FO_HIP_TRY(hipStreamSynchronize(s));
  if (p->flag_host[FLAG_DIAG])
    return fail(FO_ENONFINITE, "fo_mdsc_setup: a plane diagonal block is singular or not finite");
  if (p->flag_host[FLAG_COARSE])
    return fail(FO_ENONFINITE, "fo_mdsc_setup: the coarsest plane operator is singular or not finite");
  p->ready = true;
  return FO_OK;
}

extern "C" fo_status fo_mdsc_apply(const fo_mdsc *p, const double *r, double *z, void *stream) {
  if (!p || !r || !z || r == z) return fail(FO_EINVAL, "fo_mdsc_apply: NULL or aliased vectors");
  if ((reinterpret_cast<uintptr_t>(r) & 15) || (reinterpret_cast<uintptr_t>(z) & 15))
    return fail(FO_EINVAL, "fo_mdsc_apply: vectors must be 16-byte aligned");
  if (!p->ready) return fail(FO_EINVAL, "fo_mdsc_apply: no successful fo_mdsc_setup");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const MeshView &mv = p->mesh->view;
  const size_t last = p->lv.size() - 1;
  const PlaneLevel &l0 = p->lv[0];
  {
    const size_t col_bytes = size_t(4) * (mv.L + 1) * sizeof(double);
    int cols = 64;
    while (cols > 1 && cols * col_bytes > 65536) cols /= 2;
    hipLaunchKernelGGL(restrict_fine_kernel, dim3(blocks_for(mv.V, cols)), dim3(128), cols * col_bytes, s, mv.V,
                       mv.L, cols, p->W32, r, l0.b);
    FO_LAUNCH_CHECK("mdsc restrict");
  }
  // level 0 smooths with degree 2, the coarser levels with degree 1
  const int nl = int(last);
  for (int l = 0; l < nl; ++l) {
    const unsigned gv = blocks_for(int64_t(p->lv[l].n) * G, 256), ga = blocks_for(int64_t(p->lv[l + 1].n) * 64, 256);
    if (l == 0) {
      hipLaunchKernelGGL(pre2_kernel, dim3(gv), dim3(256), 0, s, p->lv_dev, l);
      hipLaunchKernelGGL(resid_restrict_kernel<2>, dim3(ga), dim3(256), 0, s, p->lv_dev, l);
    } else {
      hipLaunchKernelGGL(resid_restrict_kernel<1>, dim3(ga), dim3(256), 0, s, p->lv_dev, l);
    }
    FO_LAUNCH_CHECK("mdsc pre-smoothing");
  }
  hipLaunchKernelGGL(coarse_solve_kernel, dim3(1), dim3(1024), 0, s, p->lv_dev, nl, p->Ainv);
  FO_LAUNCH_CHECK("mdsc coarse solve");
  for (int l = nl - 1; l >= 0; --l) {
    const unsigned gv = blocks_for(int64_t(p->lv[l].n) * G, 256);
    if (l == 0) {
      hipLaunchKernelGGL(post0_kernel<2>, dim3(gv), dim3(256), 0, s, p->lv_dev, l);
      hipLaunchKernelGGL(post1_kernel, dim3(gv), dim3(256), 0, s, p->lv_dev, l);
    } else {
      hipLaunchKernelGGL(post0_kernel<1>, dim3(gv), dim3(256), 0, s, p->lv_dev, l);
    }
    FO_LAUNCH_CHECK("mdsc post-smoothing");
  }
  return colblock_apply_correction(p->mesh, p->fac, p->W32, p->JP, l0.x, r, z, s);
}

extern "C" fo_status fo_mdsc_export(const fo_mdsc *p, int32_t what, int32_t level, double *host, size_t count,
                                    void *stream) {
  if (!p || !host) return fail(FO_EINVAL, "fo_mdsc_export: NULL argument");
  if (!p->ready) return fail(FO_EINVAL, "fo_mdsc_export: no successful fo_mdsc_setup");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double *src = nullptr;
  size_t n = 0;
  const int32_t nl = int32_t(p->lv.size());
  if (what == FO_MDSC_WEIGHTS) {
    src = p->W;
    n = 4 * size_t(p->mesh->view.V) * size_t(p->mesh->view.L + 1);
  } else if (what == FO_MDSC_PLANE && level >= 0 && level < nl) {
    src = p->lv[level].A;
    n = 4 * size_t(p->lv[level].nnzb);
  } else if (what == FO_MDSC_BOUND && level >= 0 && level < nl - 1) {
    src = p->lv[level].g;
    n = 1;
  } else {
    return fail(FO_EINVAL, "fo_mdsc_export: bad field or level");
  }
  if (count != n) return fail(FO_EINVAL, "fo_mdsc_export: count must be " + std::to_string(n));
  FO_HIP_TRY(hipMemcpyAsync(host, src, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  FO_HIP_TRY(hipStreamSynchronize(s));
  return FO_OK;
}
