// Linear-algebra kernels behind fo_newton_solve: SpMV over the Jacobian layout with FP64 or FP32 values,
// the vertical-column block preconditioner, and the fused Krylov vector kernels.
//
// Preconditioner.  Each vertex column of the extruded mesh couples its own 2(L+1)
// dofs through a block-tridiagonal matrix (2x2 blocks, one per level).  Extracting
// that block from J and factoring it by block LU without pivoting, one vertical line
// per thread, follows the batched per-line solve the paper uses inside its
// semicoarsening multigrid (arXiv:2204.04321 Sec. 4.4); here it is used directly as
// a block-Jacobi preconditioner for GMRES (Sec. 3.1 names GMRES as the Krylov method).
#include <hip/hip_runtime.h>

#include "fo_internal.h"
#include "fo_solver.h"

namespace fo {
namespace {

__device__ __forceinline__ int nlev(int k, int L) { return (k == 0 || k == L) ? 2 : 3; }
__device__ __forceinline__ int cumlev(int k) { return k == 0 ? 0 : 3 * k - 1; }

constexpr int SPMV_LANES = 8;   // lanes per node (pair of rows)
constexpr int APPLY_MAX_COLS = 64;      // columns per preconditioner-apply block
constexpr int APPLY_THREADS = 256;      // its threads: all stage and copy, one per column sweeps

template <class JT> struct Pair2;
template <> struct Pair2<double> { using T = double2; };
template <> struct Pair2<float> { using T = float2; };

// y = J x over the Jacobian's own layout, without the CSR column indices.  The two rows of
// node (v, k) (components u and v) share one column list and follow each other: the row
// block starts at colptr[v] + 4 D cumlev(k), row c at + c 2 nl D, and entry (r, lev, d)
// at + r 2 nl + 2 lev + d couples neighbour r of v (sorted list), level klo + lev,
// component d.  Each lane takes whole (u, v) column pairs: one 16-byte x load and one
// two-value load per row.
template <class JT>
__global__ __launch_bounds__(256) void spmv_kernel(int V, int L, const int64_t *__restrict__ colptr,
                                                   const int32_t *__restrict__ nbr_ptr,
                                                   const int32_t *__restrict__ nbr_idx,
                                                   const JT *__restrict__ vals, const double *__restrict__ x,
                                                   double *__restrict__ y) {
  using T2 = typename Pair2<JT>::T;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t node = gid / SPMV_LANES;
  const int sub = int(gid % SPMV_LANES);
  const int64_t n_nodes = int64_t(V) * (L + 1);
  double a0 = 0.0, a1 = 0.0;
  if (node < n_nodes) {
    const int v = int(node / (L + 1)), k = int(node - int64_t(v) * (L + 1));
    const int nb = nbr_ptr[v], D = nbr_ptr[v + 1] - nb;
    const int nl = nlev(k, L);
    const int klo = k > 0 ? k - 1 : 0;
    const JT *row = vals + colptr[v] + int64_t(4) * D * cumlev(k);
    const int len = 2 * nl * D;
    if constexpr (sizeof(JT) == 4) {
      // FP32 values: two column pairs per lane, one 16-byte load per row (the second row
      // starts 2 nl D entries later, so its loads are only 8-byte aligned)
      for (int q = 2 * sub; q + 1 < nl * D; q += 2 * SPMV_LANES) {
        const int r0 = nl == 3 ? (q * 43691) >> 17 : q >> 1, r1 = nl == 3 ? ((q + 1) * 43691) >> 17 : (q + 1) >> 1;
        const int64_t c0 = 2 * (int64_t(nbr_idx[nb + r0]) * (L + 1) + klo + (q - r0 * nl));
        const int64_t c1 = 2 * (int64_t(nbr_idx[nb + r1]) * (L + 1) + klo + (q + 1 - r1 * nl));
        const double2 x0 = *reinterpret_cast<const double2 *>(x + c0);
        const double2 x1 = *reinterpret_cast<const double2 *>(x + c1);
        float4 v0, v1;
        __builtin_memcpy(&v0, row + 2 * q, sizeof v0);
        __builtin_memcpy(&v1, row + len + 2 * q, sizeof v1);
        a0 = fma(double(v0.x), x0.x, fma(double(v0.y), x0.y, a0));
        a0 = fma(double(v0.z), x1.x, fma(double(v0.w), x1.y, a0));
        a1 = fma(double(v1.x), x0.x, fma(double(v1.y), x0.y, a1));
        a1 = fma(double(v1.z), x1.x, fma(double(v1.w), x1.y, a1));
      }
      if ((nl * D) & 1) {   // the last column pair of an odd count
        const int q = nl * D - 1;
        if (sub == (q >> 1) % SPMV_LANES) {
          const int r = nl == 3 ? (q * 43691) >> 17 : q >> 1;
          const int64_t col = 2 * (int64_t(nbr_idx[nb + r]) * (L + 1) + klo + (q - r * nl));
          const double2 xv = *reinterpret_cast<const double2 *>(x + col);
          const T2 v0 = *reinterpret_cast<const T2 *>(row + 2 * q), v1 = *reinterpret_cast<const T2 *>(row + len + 2 * q);
          a0 = fma(double(v0.x), xv.x, fma(double(v0.y), xv.y, a0));
          a1 = fma(double(v1.x), xv.x, fma(double(v1.y), xv.y, a1));
        }
      }
    } else
    for (int q = sub; q < nl * D; q += SPMV_LANES) {
      const int r = nl == 3 ? (q * 43691) >> 17 : q >> 1;   // q / nl, exact for q < 65536
      const int lev = q - r * nl;
      const int64_t col = 2 * (int64_t(nbr_idx[nb + r]) * (L + 1) + klo + lev);
      const double2 xv = *reinterpret_cast<const double2 *>(x + col);
      const T2 v0 = *reinterpret_cast<const T2 *>(row + 2 * q), v1 = *reinterpret_cast<const T2 *>(row + len + 2 * q);
      a0 = fma(double(v0.x), xv.x, fma(double(v0.y), xv.y, a0));
      a1 = fma(double(v1.x), xv.x, fma(double(v1.y), xv.y, a1));
    }
  }
#pragma unroll
  for (int off = SPMV_LANES / 2; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, SPMV_LANES);
    a1 += __shfl_xor(a1, off, SPMV_LANES);
  }
  if (node < n_nodes && sub == 0) {
    y[2 * node] = a0;
    y[2 * node + 1] = a1;
  }
}

// Block-tridiagonal factor of one vertical line (column v): per level k the inverse
// of the Schur complement S_k (2x2), the coupling to level k-1 (Lo_k) and G_k =
// S_k^{-1} Up_k (Up_k: the coupling to level k+1), which is all the backward sweep needs.
// The recursion runs in FP64; the stored factors are FP32 (half the bytes for every
// preconditioner apply), which defines a fixed linear M^{-1} as right preconditioning needs.
template <class JT>
__global__ __launch_bounds__(128) void colblock_factor_kernel(MeshView m, const int32_t *__restrict__ self_rank,
                                                              const JT *__restrict__ vals,
                                                              float *__restrict__ fac) {
  const int v = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= m.V) return;
  const int L = m.L;
  const int D = m.deg[v];
  const int sr = self_rank[v];
  const int64_t base = m.colptr[v];
  const int64_t V = m.V;
  double Gp[4] = {0, 0, 0, 0};      // G_{k-1} = S_{k-1}^{-1} Up_{k-1}
  for (int k = 0; k <= L; ++k) {
    const int nl = nlev(k, L), kmin = k > 0 ? k - 1 : 0;
    double Dk[4], Lo[4] = {0, 0, 0, 0}, Up[4] = {0, 0, 0, 0};
    for (int c = 0; c < 2; ++c) {
      const int64_t row = base + int64_t(4) * D * cumlev(k) + int64_t(c) * 2 * nl * D + int64_t(sr) * 2 * nl;
      for (int d = 0; d < 2; ++d) {
        Dk[2 * c + d] = double(vals[row + 2 * (k - kmin) + d]);
        if (k > 0) Lo[2 * c + d] = double(vals[row + 2 * (k - 1 - kmin) + d]);
        if (k < L) Up[2 * c + d] = double(vals[row + 2 * (k + 1 - kmin) + d]);
      }
    }
    if (k > 0) {
      // S_k = D_k - Lo_k S_{k-1}^{-1} Up_{k-1}
      Dk[0] -= Lo[0] * Gp[0] + Lo[1] * Gp[2];
      Dk[1] -= Lo[0] * Gp[1] + Lo[1] * Gp[3];
      Dk[2] -= Lo[2] * Gp[0] + Lo[3] * Gp[2];
      Dk[3] -= Lo[2] * Gp[1] + Lo[3] * Gp[3];
    }
    const double det = Dk[0] * Dk[3] - Dk[1] * Dk[2];
    const double id = 1.0 / det;
    double Si[4] = {Dk[3] * id, -Dk[1] * id, -Dk[2] * id, Dk[0] * id};
    Gp[0] = Si[0] * Up[0] + Si[1] * Up[2];
    Gp[1] = Si[0] * Up[1] + Si[1] * Up[3];
    Gp[2] = Si[2] * Up[0] + Si[3] * Up[2];
    Gp[3] = Si[2] * Up[1] + Si[3] * Up[3];
    float *Fk = fac + int64_t(k) * 12 * V + v;   // field f of level k at Fk[f V]
    for (int i = 0; i < 4; ++i) {
      Fk[i * V] = float(Si[i]);
      Fk[(4 + i) * V] = float(Lo[i]);
      Fk[(8 + i) * V] = float(Gp[i]);
    }
  }
}

// Forward then backward block substitution of one vertical line, in place on its 2 (L+1)
// values zv (r in, z = M^{-1} r out).  The factors are stored level-major with the vertex index
// fastest, so a wave's loads of one factor field are contiguous.
__device__ __forceinline__ void column_sweep(const float *__restrict__ fac, int64_t Vl, int L, int64_t v, double *zv) {
  // forward: y_k = r_k - Lo_k S_{k-1}^{-1} y_{k-1}; keep w_k = S_k^{-1} y_k.  The next
  // level's factors are loaded one level ahead.
  double f[8], fn[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) fn[i] = double(fac[int64_t(i) * Vl + v]);
  double w0 = 0, w1 = 0;
  for (int k = 0; k <= L; ++k) {
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = fn[i];
    double y0 = zv[2 * k], y1 = zv[2 * k + 1];
    if (k < L) {
      const float *Fn = fac + int64_t(k + 1) * 12 * Vl + v;
#pragma unroll
      for (int i = 0; i < 8; ++i) fn[i] = double(Fn[i * Vl]);
    }
    if (k > 0) {
      y0 -= f[4] * w0 + f[5] * w1;
      y1 -= f[6] * w0 + f[7] * w1;
    }
    w0 = f[0] * y0 + f[1] * y1;
    w1 = f[2] * y0 + f[3] * y1;
    zv[2 * k] = w0;
    zv[2 * k + 1] = w1;
  }
  // backward: z_k = w_k - G_k z_{k+1}, G_k = S_k^{-1} Up_k
  double z0 = zv[2 * L], z1 = zv[2 * L + 1];
  double g[4], gn[4];
  {
    const float *Fk = fac + int64_t(L - 1 >= 0 ? L - 1 : 0) * 12 * Vl + v;
#pragma unroll
    for (int i = 0; i < 4; ++i) gn[i] = double(Fk[(8 + i) * Vl]);
  }
  for (int k = L - 1; k >= 0; --k) {
#pragma unroll
    for (int i = 0; i < 4; ++i) g[i] = gn[i];
    if (k > 0) {
      const float *Fn = fac + int64_t(k - 1) * 12 * Vl + v;
#pragma unroll
      for (int i = 0; i < 4; ++i) gn[i] = double(Fn[(8 + i) * Vl]);
    }
    const double n0 = zv[2 * k] - (g[0] * z0 + g[1] * z1);
    const double n1 = zv[2 * k + 1] - (g[2] * z0 + g[3] * z1);
    z0 = n0;
    z1 = n1;
    zv[2 * k] = z0;
    zv[2 * k + 1] = z1;
  }
}

// z = M^{-1} r for every vertical line.  A block's `cols` columns are contiguous in r and z
// (2 (L+1) values each): all its threads copy them through LDS with coalesced loads and
// stores, and one thread per column runs the column's two sweeps in place in LDS.
__global__ __launch_bounds__(APPLY_THREADS) void colblock_apply_kernel(int V, int L, int cols,
                                                                       const float *__restrict__ fac,
                                                                       const double *__restrict__ r,
                                                                       double *__restrict__ z) {
  extern __shared__ double col_sh[];   // [cols][2 (L + 1)]
  const int n = 2 * (L + 1);
  const int64_t v0 = int64_t(blockIdx.x) * cols;
  const int nv = int(V - v0 < int64_t(cols) ? V - v0 : int64_t(cols));
  for (int e = threadIdx.x; e < nv * n; e += blockDim.x) col_sh[e] = r[v0 * n + e];
  __syncthreads();
  if (int(threadIdx.x) < nv) column_sweep(fac, V, L, v0 + threadIdx.x, col_sh + threadIdx.x * n);
  __syncthreads();
  for (int e = threadIdx.x; e < nv * n; e += blockDim.x) z[v0 * n + e] = col_sh[e];
}

// The last step of the two-level preconditioner: z = P0 y + M^{-1} (r - (J P0) y).  While the
// block's columns are staged in LDS each row subtracts its row of J P0 against the plane vector
// y (J P0 in FP32, column v's block starting at 4 (L+1) nbr_ptr[v] and holding entry (r, d) of
// row q at (2 r + d) 2 (L+1) + q, so consecutive rows of a column are consecutive for each
// entry); after the sweeps each row adds its prolongation sum_c W[v][k][c'][c] y[(v, c)] (FP32
// weights, the two c of a row next to each other).
__global__ __launch_bounds__(APPLY_THREADS) void colblock_correction_kernel(
    int V, int L, int cols, const int32_t *__restrict__ nbr_ptr, const int32_t *__restrict__ nbr_idx,
    const float *__restrict__ fac, const float *__restrict__ W32, const float *__restrict__ JP,
    const double *__restrict__ y, const double *__restrict__ r, double *__restrict__ z) {
  extern __shared__ double col_sh[];   // [cols][2 (L + 1)]
  const int n = 2 * (L + 1);
  const int64_t v0 = int64_t(blockIdx.x) * cols;
  const int nv = int(V - v0 < int64_t(cols) ? V - v0 : int64_t(cols));
  const double2 *y2 = reinterpret_cast<const double2 *>(y);
  for (int e = threadIdx.x; e < nv * n; e += blockDim.x) {
    const int64_t v = v0 + e / n;
    const int q = e - (e / n) * n;
    const int p0 = nbr_ptr[v], D = nbr_ptr[v + 1] - p0;
    const float *jp = JP + int64_t(2 * n) * p0 + q;
    double s = r[v0 * n + e];
    for (int i = 0; i < D; ++i) {
      const double2 yw = y2[nbr_idx[p0 + i]];
      s -= double(jp[(2 * i) * n]) * yw.x + double(jp[(2 * i + 1) * n]) * yw.y;
    }
    col_sh[e] = s;
  }
  __syncthreads();
  if (int(threadIdx.x) < nv) column_sweep(fac, V, L, v0 + threadIdx.x, col_sh + threadIdx.x * n);
  __syncthreads();
  const float2 *W2 = reinterpret_cast<const float2 *>(W32);
  for (int e = threadIdx.x; e < nv * n; e += blockDim.x) {
    const int64_t v = v0 + e / n;
    const float2 w = W2[v0 * n + e];
    const double2 yv = y2[v];
    z[v0 * n + e] = col_sh[e] + (double(w.x) * yv.x + double(w.y) * yv.y);
  }
}

constexpr int RED_BLOCK = 256;

constexpr int MD_GROUP = 24;   // dot products per pass over a block's chunk

// partial[b * (nv + 1) + i] = sum over block b's rows of V_i . w (i < nv), and w . w (i = nv).
// Vectors are taken MD_GROUP at a time, so each pass loads w once for all of them and has
// 2 MD_GROUP independent loads in flight per iteration: each lane takes two consecutive
// entries (16-byte loads; n and ld are even) at two places a grid stride apart.  Blocks
// stride through the vectors together
// (grid-stride), so at any time the grid reads one window of each vector (DRAM page
// locality); the summation order is fixed.
__global__ __launch_bounds__(RED_BLOCK) void multidot_kernel(int64_t n2, const double *__restrict__ V, int64_t ld,
                                                             int nv, const double *__restrict__ w,
                                                             double *__restrict__ partial) {
  __shared__ double red[MD_GROUP][RED_BLOCK / 64];
  const int64_t stride = int64_t(gridDim.x) * RED_BLOCK;
  const double2 *w2 = reinterpret_cast<const double2 *>(w);
  for (int i0 = 0; i0 <= nv; i0 += MD_GROUP) {
    const int g = nv + 1 - i0 < MD_GROUP ? nv + 1 - i0 : MD_GROUP;
    double s[MD_GROUP];
#pragma unroll
    for (int q = 0; q < MD_GROUP; ++q) s[q] = 0.0;
    for (int64_t p = int64_t(blockIdx.x) * RED_BLOCK + threadIdx.x; p < n2; p += 2 * stride) {
      const int64_t p1 = p + stride;
      const bool two = p1 < n2;
      const double2 wp = w2[p];
      const double2 wq = two ? w2[p1] : make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < MD_GROUP; ++q) {
        if (q < g) {
          const int i = i0 + q;
          const double2 *Vi = reinterpret_cast<const double2 *>(V + int64_t(i) * ld);
          const double2 a = i < nv ? Vi[p] : wp;
          const double2 b = two ? (i < nv ? Vi[p1] : wq) : make_double2(0.0, 0.0);
          s[q] = fma(a.x, wp.x, fma(a.y, wp.y, fma(b.x, wq.x, fma(b.y, wq.y, s[q]))));
        }
      }
    }
#pragma unroll
    for (int q = 0; q < MD_GROUP; ++q) {
      double t = s[q];
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
      if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < g) {
      double t = 0.0;
      for (int q = 0; q < RED_BLOCK / 64; ++q) t += red[threadIdx.x][q];
      partial[int64_t(blockIdx.x) * (nv + 1) + i0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// partial[2 b] = sum over block b's entries of a . w, partial[2 b + 1] of w . w; two
// consecutive entries per lane, grid-stride
__global__ __launch_bounds__(RED_BLOCK) void dot2_kernel(int64_t n2, const double *__restrict__ a,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ partial) {
  __shared__ double red[2][RED_BLOCK / 64];
  const int64_t stride = int64_t(gridDim.x) * RED_BLOCK;
  const double2 *a2 = reinterpret_cast<const double2 *>(a);
  const double2 *w2 = reinterpret_cast<const double2 *>(w);
  double s0 = 0.0, s1 = 0.0;
  for (int64_t p = int64_t(blockIdx.x) * RED_BLOCK + threadIdx.x; p < n2; p += stride) {
    const double2 x = a2[p], y = w2[p];
    s0 = fma(x.x, y.x, fma(x.y, y.y, s0));
    s1 = fma(y.x, y.x, fma(y.y, y.y, s1));
  }
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s0;
    red[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int q = 0; q < RED_BLOCK / 64; ++q) t += red[threadIdx.x][q];
    partial[2 * int64_t(blockIdx.x) + threadIdx.x] = t;
  }
}

// out[i] = sum_b partial[b * stride + i], fixed order
__global__ void reduce_partials_kernel(int nb, int stride, const double *__restrict__ partial,
                                       double *__restrict__ out) {
  const int i = blockIdx.x;
  __shared__ double red[256 / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[int64_t(b) * stride + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 4; ++q) t += red[q];
    out[i] = t;
  }
}

// w = w + sign sum_i h_i V_i  (h on the device), two consecutive entries per lane
__global__ __launch_bounds__(256) void multiaxpy_kernel(int64_t n2, const double *__restrict__ V, int64_t ld,
                                                        int nv, const double *__restrict__ h,
                                                        double *__restrict__ w, double sign) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  double2 *w2 = reinterpret_cast<double2 *>(w);
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n2; p += stride) {
    double ax = 0.0, ay = 0.0;
    for (int i = 0; i < nv; ++i) {
      const double2 a = reinterpret_cast<const double2 *>(V + int64_t(i) * ld)[p];
      ax += h[i] * a.x;
      ay += h[i] * a.y;
    }
    double2 t = w2[p];
    t.x += sign * ax;
    t.y += sign * ay;
    w2[p] = t;
  }
}

// conjugate-gradient step with the step length formed on the device:
// alpha = num[0] / den[0], x += alpha p, r -= alpha q
__global__ __launch_bounds__(256) void cg_step_kernel(int64_t n, const double *__restrict__ num,
                                                      const double *__restrict__ den,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q, double *__restrict__ x,
                                                      double *__restrict__ r) {
  const double alpha = num[0] / den[0];
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
  }
}

// y = a x + b y
__global__ __launch_bounds__(256) void axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b,
                                                    double *__restrict__ y) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride)
    y[p] = (b == 0.0 ? 0.0 : b * y[p]) + a * x[p];
}

// z = x + a y
__global__ __launch_bounds__(256) void xpay_kernel(int64_t n, const double *__restrict__ x, double a,
                                                   const double *__restrict__ y, double *__restrict__ z) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += stride)
    z[p] = x[p] + a * y[p];
}

// columns per apply block: the block's columns (2 (L+1) doubles each) stay within 64 KB of LDS
size_t col_bytes(int L) { return size_t(2) * (L + 1) * sizeof(double); }
int apply_cols(int L) {
  int cols = APPLY_MAX_COLS;
  while (cols > 1 && cols * col_bytes(L) > 65536) cols /= 2;
  return cols;
}

unsigned grid_for(int64_t n, int block) {
  const int64_t g = (n + block - 1) / block;
  return unsigned(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

fo_status spmv(const fo_mesh *mesh, const void *vals, int dtype, const double *x, double *y, hipStream_t s) {
  const MeshView &m = mesh->view;
  const int64_t threads = (m.n_dofs / 2) * SPMV_LANES;
  const unsigned blocks = unsigned((threads + 255) / 256);
  if (dtype == FO_F32)
    hipLaunchKernelGGL(spmv_kernel<float>, dim3(blocks), dim3(256), 0, s, m.V, m.L, m.colptr, mesh->nbr_ptr,
                       mesh->nbr_idx, static_cast<const float *>(vals), x, y);
  else
    hipLaunchKernelGGL(spmv_kernel<double>, dim3(blocks), dim3(256), 0, s, m.V, m.L, m.colptr, mesh->nbr_ptr,
                       mesh->nbr_idx, static_cast<const double *>(vals), x, y);
  FO_LAUNCH_CHECK("spmv_kernel");
  return FO_OK;
}

fo_status colblock_factor(const fo_mesh *mesh, const void *vals, int dtype, float *fac, hipStream_t s) {
  const MeshView &m = mesh->view;
  const unsigned blocks = unsigned((m.V + 127) / 128);
  if (dtype == FO_F32)
    hipLaunchKernelGGL(colblock_factor_kernel<float>, dim3(blocks), dim3(128), 0, s, m, mesh->self_rank,
                       static_cast<const float *>(vals), fac);
  else
    hipLaunchKernelGGL(colblock_factor_kernel<double>, dim3(blocks), dim3(128), 0, s, m, mesh->self_rank,
                       static_cast<const double *>(vals), fac);
  FO_LAUNCH_CHECK("colblock_factor_kernel");
  return FO_OK;
}

fo_status colblock_apply(const fo_mesh *mesh, const float *fac, const double *r, double *z, hipStream_t s) {
  const MeshView &m = mesh->view;
  const int cols = apply_cols(m.L);
  const unsigned blocks = unsigned((m.V + cols - 1) / cols);
  hipLaunchKernelGGL(colblock_apply_kernel, dim3(blocks), dim3(APPLY_THREADS), cols * col_bytes(m.L), s, m.V, m.L,
                     cols, fac, r, z);
  FO_LAUNCH_CHECK("colblock_apply_kernel");
  return FO_OK;
}

fo_status colblock_apply_correction(const fo_mesh *mesh, const float *fac, const float *W32, const float *JP,
                                    const double *y, const double *r, double *z, hipStream_t s) {
  const MeshView &m = mesh->view;
  const int cols = apply_cols(m.L);
  const unsigned blocks = unsigned((m.V + cols - 1) / cols);
  hipLaunchKernelGGL(colblock_correction_kernel, dim3(blocks), dim3(APPLY_THREADS), cols * col_bytes(m.L), s, m.V,
                     m.L, cols, mesh->nbr_ptr, mesh->nbr_idx, fac, W32, JP, y, r, z);
  FO_LAUNCH_CHECK("colblock_correction_kernel");
  return FO_OK;
}

int multidot_blocks(int64_t n) {
  const int64_t g = (n + 16 * RED_BLOCK - 1) / (16 * RED_BLOCK);
  return int(g < 512 ? (g > 0 ? g : 1) : 512);
}

fo_status multidot(int64_t n, const double *V, int64_t ld, int nv, const double *w, double *partial,
                   double *out, hipStream_t s) {
  if ((n | ld) & 1) return fail(FO_EINVAL, "multidot: vector length and stride must be even");
  const int nb = multidot_blocks(n);
  hipLaunchKernelGGL(multidot_kernel, dim3(nb), dim3(RED_BLOCK), 0, s, n / 2, V, ld, nv, w, partial);
  FO_LAUNCH_CHECK("multidot_kernel");
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(nv + 1), dim3(256), 0, s, nb, nv + 1, partial, out);
  FO_LAUNCH_CHECK("reduce_partials_kernel");
  return FO_OK;
}

int dot2_blocks(int64_t n) {
  const int64_t g = (n / 2 + 4 * RED_BLOCK - 1) / (4 * RED_BLOCK);
  return int(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

fo_status dot2(int64_t n, const double *a, const double *w, double *partial, double *out, hipStream_t s) {
  if (n & 1) return fail(FO_EINVAL, "dot2: vector length must be even");
  const int nb = dot2_blocks(n);
  hipLaunchKernelGGL(dot2_kernel, dim3(nb), dim3(RED_BLOCK), 0, s, n / 2, a, w, partial);
  FO_LAUNCH_CHECK("dot2_kernel");
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(2), dim3(256), 0, s, nb, 2, partial, out);
  FO_LAUNCH_CHECK("reduce_partials_kernel");
  return FO_OK;
}

fo_status multiaxpy(int64_t n, const double *V, int64_t ld, int nv, const double *h, double *w, double sign,
                    hipStream_t s) {
  if ((n | ld) & 1) return fail(FO_EINVAL, "multiaxpy: vector length and stride must be even");
  const int64_t g = (n / 2 + 255) / 256;
  hipLaunchKernelGGL(multiaxpy_kernel, dim3(unsigned(g < 2048 ? (g > 0 ? g : 1) : 2048)), dim3(256), 0, s, n / 2, V,
                     ld, nv, h, w, sign);
  FO_LAUNCH_CHECK("multiaxpy_kernel");
  return FO_OK;
}

fo_status cg_step(int64_t n, const double *num, const double *den, const double *p, const double *q, double *x,
                  double *r, hipStream_t s) {
  hipLaunchKernelGGL(cg_step_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, num, den, p, q, x, r);
  FO_LAUNCH_CHECK("cg_step_kernel");
  return FO_OK;
}

fo_status axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, a, x, b, y);
  FO_LAUNCH_CHECK("axpby_kernel");
  return FO_OK;
}

fo_status xpay(int64_t n, const double *x, double a, const double *y, double *z, hipStream_t s) {
  hipLaunchKernelGGL(xpay_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, x, a, y, z);
  FO_LAUNCH_CHECK("xpay_kernel");
  return FO_OK;
}

}  // namespace fo
