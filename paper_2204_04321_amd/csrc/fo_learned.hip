// Learned Newton initial guess: per-column features, a 10-128-128-128-22 tanh MLP whose
// products run on gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation),
// its backward pass, MSE gradient and Adam, and the guess itself with its shallow-ice
// fallback.  Not part of the paper: the network only supplies the starting point of the
// damped Newton solve of Sec. 3.1 (eq. linearsystem).
//
// Rounding points: products take BF16 (round to nearest even) copies of inputs, weights,
// hidden activations and backpropagated errors; sums are FP32; biases, tanh and its
// derivative use the unrounded FP32 values.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "fo_device.h"
#include "fo_internal.h"
#include "fo_solver.h"

namespace fo {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NIN = 10, NH = 128, NOUT = 22;
constexpr int LAY[5] = {NIN, NH, NH, NH, NOUT};

// offsets of W_l ([out][in]) and b_l ([out]) in the flat FP32 parameter vector
constexpr int woff(int l) { int o = 0; for (int i = 0; i < l; ++i) o += LAY[i] * LAY[i + 1] + LAY[i + 1]; return o; }
constexpr int boff(int l) { return woff(l) + LAY[l] * LAY[l + 1]; }
constexpr int NPARAM = woff(4);

// ---- column features --------------------------------------------------------------------
__global__ void features_kernel(MeshView m, const int32_t *__restrict__ nbr_ptr,
                                const int32_t *__restrict__ nbr_idx, const int32_t *__restrict__ vc_ptr,
                                const int32_t *__restrict__ vc_idx, const float *__restrict__ norm,
                                float *__restrict__ F) {
  const int v = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= m.V) return;
  double gx, gy;
  vertex_surface_gradient(m, vc_ptr, vc_idx, v, gx, gy);
  const double4 gv = m.geo[v];
  const double Hv = gv.w;
  const double beta = m.sb[v].y;
  double f[10];
  f[0] = Hv;
  f[1] = gx;
  f[2] = gy;
  f[3] = log(beta > 1e-3 ? beta : 1e-3);
  // the 6 nearest neighbours (distance, then index), ordered by angle from -grad s
  const int p0 = nbr_ptr[v], p1 = nbr_ptr[v + 1];
  int sel[6];
  int nsel = 0;
  double last_d2 = -1.0;
  int last_w = -1;
  for (int r = 0; r < 6; ++r) {
    double best_d2 = 0.0;
    int best_w = -1;
    for (int p = p0; p < p1; ++p) {
      const int w = nbr_idx[p];
      if (w == v) continue;
      const double4 g = m.geo[w];
      const double dx = g.x - gv.x, dy = g.y - gv.y;
      const double d2 = dx * dx + dy * dy;
      const bool after = d2 > last_d2 || (d2 == last_d2 && w > last_w);
      const bool better = best_w < 0 || d2 < best_d2 || (d2 == best_d2 && w < best_w);
      if (after && better) { best_d2 = d2; best_w = w; }
    }
    if (best_w < 0) break;
    sel[nsel++] = best_w;
    last_d2 = best_d2;
    last_w = best_w;
  }
  const double ref = (gx != 0.0 || gy != 0.0) ? atan2(-gy, -gx) : 0.0;
  const double twopi = 6.283185307179586476925286766559;
  double ang[6];
  for (int i = 0; i < nsel; ++i) {
    const double4 g = m.geo[sel[i]];
    double a = fmod(atan2(g.y - gv.y, g.x - gv.x) - ref, twopi);
    if (a < 0) a += twopi;
    ang[i] = a;
  }
  for (int i = 1; i < nsel; ++i) {   // insertion sort by (angle, index)
    const double a = ang[i];
    const int w = sel[i];
    int j = i - 1;
    while (j >= 0 && (ang[j] > a || (ang[j] == a && sel[j] > w))) { ang[j + 1] = ang[j]; sel[j + 1] = sel[j]; --j; }
    ang[j + 1] = a;
    sel[j + 1] = w;
  }
  for (int i = 0; i < 6; ++i) f[4 + i] = i < nsel ? m.geo[sel[i]].w : Hv;
  for (int i = 0; i < 10; ++i) {
    const double x = norm ? (f[i] - double(norm[i])) / double(norm[10 + i]) : f[i];
    F[int64_t(v) * 10 + i] = float(x);
  }
}

// ---- GEMM on BF16 matrix cores ------------------------------------------------------------
// C(m,n) = epi(sum_k A(m,k) B(k,n)) with A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn].
// One wave per 16 x 16 tile of C; K is consumed 32 at a time.  Lane (r = l % 16, q = l / 16)
// supplies A row r and B column r, k = 8q..8q+7 of each 32-block; it receives C rows
// 4q..4q+3 of column r.  Epilogues: 0 store, 1 + bias, 2 tanh(+ bias), 3 multiply by
// (1 - aux^2) (tanh derivative from the stored activation), 4 accumulate into C.
__global__ __launch_bounds__(64) void gemm_bf16_kernel(int M, int N, int K, const float *__restrict__ A,
                                                       int64_t sam, int64_t sak, const float *__restrict__ B,
                                                       int64_t sbk, int64_t sbn, float *__restrict__ C,
                                                       int64_t scm, int64_t scn, const float *__restrict__ bias,
                                                       const float *__restrict__ aux, int64_t sxm, int mode) {
  const int tm = blockIdx.x, tn = blockIdx.y;
  const int l = threadIdx.x, r = l & 15, q = l >> 4;
  const int ma = tm * 16 + r, nb = tn * 16 + r;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * q + j;
      a[j] = (ma < M && k < K) ? __bf16(A[int64_t(ma) * sam + int64_t(k) * sak]) : __bf16(0.f);
      b[j] = (nb < N && k < K) ? __bf16(B[int64_t(k) * sbk + int64_t(nb) * sbn]) : __bf16(0.f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int mm = tm * 16 + 4 * q + i, nn = tn * 16 + r;
    if (mm >= M || nn >= N) continue;
    float v = acc[i];
    float *dst = C + int64_t(mm) * scm + int64_t(nn) * scn;
    if (mode == 1 || mode == 2) v += bias[nn];
    if (mode == 2) v = tanhf(v);
    if (mode == 3) { const float a = aux[int64_t(mm) * sxm + nn]; v *= 1.0f - a * a; }
    if (mode == 4) v += *dst;
    *dst = v;
  }
}

// db(n) = sum_m dZ(m, n)
__global__ void colsum_kernel(int M, int N, const float *__restrict__ dZ, float *__restrict__ db) {
  const int n = blockIdx.x;
  __shared__ float red[4];
  float s = 0.f;
  for (int m = threadIdx.x; m < M; m += blockDim.x) s += dZ[int64_t(m) * N + n];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) db[n] = red[0] + red[1] + red[2] + red[3];
}

__global__ void mse_grad_kernel(int64_t n, const float *__restrict__ Y, const float *__restrict__ T,
                                float *__restrict__ dY, double *__restrict__ loss) {
  __shared__ double red[4];
  double s = 0.0;
  const float scale = 2.0f / float(n);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = scale * d;
    s += double(d) * double(d);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) / double(n));
}

__global__ void adam_kernel(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// D = 10 sinh(Y): the network's correction of the shallow-ice profile (a column's outputs are
// its dofs in order)
__global__ void correction_kernel(int64_t n, const float *__restrict__ Y, double *__restrict__ D) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  D[i] = 10.0 * sinh(double(Y[i]));
}

// One Jacobi sweep over the base mesh: Dn_v = (D_v + mean of D_w over v's neighbours w != v) / 2,
// for each of the nd dofs of a column.
__global__ void smooth_kernel(int V, int nd, const int32_t *__restrict__ nbr_ptr, const int32_t *__restrict__ nbr_idx,
                              const double *__restrict__ D, double *__restrict__ Dn) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(V) * nd) return;
  const int v = int(i / nd), r = int(i % nd);
  double s = 0.0;
  int cnt = 0;
  for (int p = nbr_ptr[v]; p < nbr_ptr[v + 1]; ++p) {
    const int w = nbr_idx[p];
    if (w == v) continue;
    s += D[int64_t(w) * nd + r];
    ++cnt;
  }
  const double d = D[i];
  Dn[i] = cnt > 0 ? 0.5 * (d + s / double(cnt)) : d;
}

// U = U_sia + D; flag non-finite values
__global__ void compose_kernel(int64_t n, const double *__restrict__ D, const double *__restrict__ Us,
                               double *__restrict__ U, int *__restrict__ bad) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double u = Us[i] + D[i];
  U[i] = u;
  if (!isfinite(u)) atomicOr(bad, 1);
}

// T = asinh((U - U_sia) / 10), rounded to FP32
__global__ void targets_kernel(int64_t n, const double *__restrict__ U, const double *__restrict__ Us,
                               float *__restrict__ T) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T[i] = float(asinh((U[i] - Us[i]) / 10.0));
}

// Xn = (X - mean) / std per feature, in FP64 and rounded once, as features_kernel normalises
__global__ void normalise_kernel(int64_t n, const float *__restrict__ X, const float *__restrict__ norm,
                                 float *__restrict__ Xn) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = int(i % NIN);
  Xn[i] = float((double(X[i]) - double(norm[j])) / double(norm[NIN + j]));
}

// Per feature column j (one block each): mean, then sqrt(sum (x - mean)^2 / (n - 1)) + 1e-6.
__global__ __launch_bounds__(256) void feature_stats_kernel(const float *__restrict__ X, int64_t n,
                                                            float *__restrict__ norm) {
  const int j = blockIdx.x;
  __shared__ double red[4];
  __shared__ double mean_s;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += double(X[r * NIN + j]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) mean_s = (red[0] + red[1] + red[2] + red[3]) / double(n);
  __syncthreads();
  const double mean = mean_s;
  double q = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double d = double(X[r * NIN + j]) - mean;
    q += d * d;
  }
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    norm[j] = float(mean);
    norm[NIN + j] = float(sqrt((red[0] + red[1] + red[2] + red[3]) / double(n - 1)) + 1e-6);
  }
}

fo_status gemm(int M, int N, int K, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
               int64_t sbn, float *C, int64_t scm, int64_t scn, const float *bias, const float *aux, int64_t sxm,
               int mode, hipStream_t s) {
  if (M <= 0 || N <= 0) return FO_OK;
  const dim3 grid(unsigned((M + 15) / 16), unsigned((N + 15) / 16));
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(64), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn,
                     bias, aux, sxm, mode);
  FO_LAUNCH_CHECK("gemm_bf16_kernel");
  return FO_OK;
}

}  // namespace

// forward through all layers: acts [3][B][NH] (FP32 tanh outputs), Y [B][NOUT]
fo_status mlp_forward_impl(const float *P, const float *X, int B, float *acts, float *Y, hipStream_t s) {
  fo_status st;
  const float *in = X;
  int fin = NIN;
  for (int l = 0; l < 4; ++l) {
    const int fout = LAY[l + 1];
    float *out = l < 3 ? acts + int64_t(l) * B * NH : Y;
    // Z = in [B x fin] . W_l^T (W_l is [fout x fin])
    if ((st = gemm(B, fout, fin, in, fin, 1, P + woff(l), 1, fin, out, fout, 1, P + boff(l), nullptr, 0,
                   l < 3 ? 2 : 1, s)) != FO_OK)
      return st;
    in = out;
    fin = fout;
  }
  return FO_OK;
}

}  // namespace fo

using namespace fo;

extern "C" int32_t fo_mlp_param_count(void) { return NPARAM; }

extern "C" fo_status fo_column_features(const fo_mesh *m, const float *norm, float *F, void *stream) {
  if (!m || !F) return fail(FO_EINVAL, "fo_column_features: NULL argument");
  const int blocks = (m->view.V + 127) / 128;
  hipLaunchKernelGGL(features_kernel, dim3(blocks), dim3(128), 0, static_cast<hipStream_t>(stream), m->view,
                     m->nbr_ptr, m->nbr_idx, m->vc_ptr, m->vc_idx, norm, F);
  FO_LAUNCH_CHECK("features_kernel");
  return FO_OK;
}

extern "C" fo_status fo_mlp_forward(const float *P, const float *X, int32_t B, float *acts, float *Y, void *stream) {
  if (!P || !X || !acts || !Y || B < 0) return fail(FO_EINVAL, "fo_mlp_forward: bad argument");
  return mlp_forward_impl(P, X, B, acts, Y, static_cast<hipStream_t>(stream));
}

extern "C" fo_status fo_mlp_backward(const float *P, const float *X, int32_t B, const float *acts, const float *dY,
                                     float *dacts, float *G, void *stream) {
  if (!P || !X || !acts || !dY || !dacts || !G || B < 0) return fail(FO_EINVAL, "fo_mlp_backward: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  fo_status st;
  // dZ of layer l lives in: l = 3 -> dY [B x NOUT]; l < 3 -> dacts slot (l & 1) [B x NH]
  const float *dZ = dY;
  int fout = NOUT;
  for (int l = 3; l >= 0; --l) {
    const int fin = LAY[l];
    const float *Ain = l > 0 ? acts + int64_t(l - 1) * B * NH : X;
    // dW_l [fout x fin] = dZ^T [fout x B] . Ain [B x fin]
    if ((st = gemm(fout, fin, B, dZ, 1, fout, Ain, fin, 1, G + woff(l), fin, 1, nullptr, nullptr, 0, 0, s)) != FO_OK)
      return st;
    hipLaunchKernelGGL(colsum_kernel, dim3(fout), dim3(256), 0, s, B, fout, dZ, G + boff(l));
    FO_LAUNCH_CHECK("colsum_kernel");
    if (l > 0) {
      // dZ_{l-1} = (dZ [B x fout] . W_l [fout x fin]) * (1 - A_{l-1}^2)
      float *dnext = dacts + int64_t(l & 1) * B * NH;
      if ((st = gemm(B, fin, fout, dZ, fout, 1, P + woff(l), fin, 1, dnext, fin, 1, nullptr, Ain, fin, 3, s)) != FO_OK)
        return st;
      dZ = dnext;
      fout = fin;
    }
  }
  return FO_OK;
}

extern "C" fo_status fo_mse_grad(const float *Y, const float *T, int64_t n, float *dY, double *loss, void *stream) {
  if (!Y || !T || !dY || n <= 0) return fail(FO_EINVAL, "fo_mse_grad: bad argument");
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream), n, Y, T,
                     dY, loss);
  FO_LAUNCH_CHECK("mse_grad_kernel");
  return FO_OK;
}

extern "C" fo_status fo_adam_step(float *P, const float *G, float *Mom, float *Var, int32_t n, float lr, float b1,
                                  float b2, float eps, int32_t step, void *stream) {
  if (!P || !G || !Mom || !Var || n <= 0 || step < 1) return fail(FO_EINVAL, "fo_adam_step: bad argument");
  const float c1 = float(1.0 / (1.0 - std::pow(double(b1), step)));
  const float c2 = float(1.0 / (1.0 - std::pow(double(b2), step)));
  hipLaunchKernelGGL(adam_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), n,
                     P, G, Mom, Var, lr, b1, b2, eps, c1, c2);
  FO_LAUNCH_CHECK("adam_kernel");
  return FO_OK;
}

namespace {
constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
struct LLayout { size_t F, acts, Y, Us, R, D, partial, dots, flag, total; };
LLayout llayout(const fo_mesh *m) {
  const size_t V = size_t(m->view.V), n = size_t(m->view.n_dofs);
  LLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t a = off; off += up(b); return a; };
  L.F = take(4 * V * NIN);
  L.acts = take(4 * 3 * V * NH);
  L.Y = take(4 * V * NOUT);
  L.Us = take(8 * n);
  L.R = take(8 * n);
  L.D = take(8 * 2 * n);
  L.partial = take(8 * size_t(multidot_blocks(int64_t(n))));
  L.dots = take(16);
  L.flag = take(16);
  L.total = off;
  return L;
}
}  // namespace

namespace fo {
size_t learned_workspace_bytes(const fo_mesh *m) { return llayout(m).total; }

fo_status learned_guess(const fo_mesh *m, const float *P, const float *norm, double *U, int32_t fallback,
                        int32_t sweeps, void *ws, size_t ws_bytes, int32_t *used_network, int32_t *n_residuals,
                        hipStream_t s) {
  if (n_residuals) *n_residuals = 0;
  if (!m || !P || !norm || !U || !ws) return fail(FO_EINVAL, "fo_initial_guess_learned: NULL argument");
  if (fallback != 0 && fallback != 1) return fail(FO_EINVAL, "fo_initial_guess_learned: fallback must be 0 or 1");
  if (sweeps < 0 || sweeps > 10000) return fail(FO_EINVAL, "fo_initial_guess_learned: smooth_sweeps must be in 0..10000");
  if (m->view.L + 1 != NOUT / 2) return fail(FO_EINVAL, "fo_initial_guess_learned: the network predicts 11 levels (L = 10)");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(FO_EINVAL, "fo_initial_guess_learned: workspace must be 256-byte aligned");
  const LLayout L = llayout(m);
  if (ws_bytes < L.total) return fail(FO_EINVAL, "fo_initial_guess_learned: workspace too small");
  char *w = static_cast<char *>(ws);
  float *F = reinterpret_cast<float *>(w + L.F), *acts = reinterpret_cast<float *>(w + L.acts);
  float *Y = reinterpret_cast<float *>(w + L.Y);
  double *Us = reinterpret_cast<double *>(w + L.Us), *R = reinterpret_cast<double *>(w + L.R);
  double *D0 = reinterpret_cast<double *>(w + L.D);
  double *part = reinterpret_cast<double *>(w + L.partial), *dots = reinterpret_cast<double *>(w + L.dots);
  int *flag = reinterpret_cast<int *>(w + L.flag);
  const int V = m->view.V;
  const int64_t n = m->view.n_dofs;
  double *D1 = D0 + n;
  fo_status st;
  if ((st = launch_sia(m, Us, s)) != FO_OK) return st;
  if ((st = fo_column_features(m, norm, F, s)) != FO_OK) return st;
  if ((st = mlp_forward_impl(P, F, V, acts, Y, s)) != FO_OK) return st;
  if ((st = launch_fill_zero(flag, 16, s)) != FO_OK) return st;
  const unsigned nb = unsigned((n + 255) / 256);
  hipLaunchKernelGGL(correction_kernel, dim3(nb), dim3(256), 0, s, n, Y, D0);
  FO_LAUNCH_CHECK("correction_kernel");
  for (int k = 0; k < sweeps; ++k) {
    hipLaunchKernelGGL(smooth_kernel, dim3(nb), dim3(256), 0, s, V, NOUT, m->nbr_ptr, m->nbr_idx, D0, D1);
    FO_LAUNCH_CHECK("smooth_kernel");
    std::swap(D0, D1);
  }
  hipLaunchKernelGGL(compose_kernel, dim3(nb), dim3(256), 0, s, n, D0, Us, U, flag);
  FO_LAUNCH_CHECK("compose_kernel");
  // fall back to the shallow-ice guess if the network output is non-finite, or (fallback = 1)
  // if its residual norm exceeds the shallow-ice guess's
  double hv[2] = {0.0, 0.0};
  int bad = 0;
  FO_HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  if (fallback == 1) {
    if ((st = launch_assemble(m, Us, R, nullptr, FO_F64, FO_JAC_NEWTON, false, s)) != FO_OK) return st;
    if (n_residuals) ++*n_residuals;
    if ((st = multidot(n, nullptr, 0, 0, R, part, dots, s)) != FO_OK) return st;
    FO_HIP_TRY(hipMemcpyAsync(&hv[1], dots, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  FO_HIP_TRY(hipStreamSynchronize(s));
  bool use_nn = bad == 0;
  if (use_nn && fallback == 1) {
    if ((st = launch_assemble(m, U, R, nullptr, FO_F64, FO_JAC_NEWTON, false, s)) != FO_OK) return st;
    if (n_residuals) ++*n_residuals;
    if ((st = multidot(n, nullptr, 0, 0, R, part, dots, s)) != FO_OK) return st;
    FO_HIP_TRY(hipMemcpyAsync(&hv[0], dots, sizeof(double), hipMemcpyDeviceToHost, s));
    FO_HIP_TRY(hipStreamSynchronize(s));
    use_nn = std::isfinite(hv[0]) && hv[0] <= hv[1];
  }
  if (!use_nn) FO_HIP_TRY(hipMemcpyAsync(U, Us, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FO_HIP_TRY(hipStreamSynchronize(s));
  if (used_network) *used_network = use_nn ? 1 : 0;
  return FO_OK;
}
}  // namespace fo

extern "C" size_t fo_learned_workspace_bytes(const fo_mesh *m) { return m ? llayout(m).total : 0; }

extern "C" fo_status fo_initial_guess_learned(const fo_mesh *m, const float *P, const float *norm, double *U,
                                              int32_t fallback, int32_t smooth_sweeps, void *ws, size_t ws_bytes,
                                              int32_t *used_network, void *stream) {
  return learned_guess(m, P, norm, U, fallback, smooth_sweeps, ws, ws_bytes, used_network, nullptr,
                       static_cast<hipStream_t>(stream));
}

// Workspace of fo_initial_guess_learned_noalloc: a library-owned array on each device,
// resolved to its device address once per device (the array's name in host code is a
// host-side stand-in, never a device address) and held until the process ends.
namespace {
__device__ __align__(256) unsigned char scratch[FO_LEARNED_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

fo_status scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return fo::fail(FO_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fo::fail(FO_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return FO_OK;
}
}  // namespace

extern "C" fo_status fo_initial_guess_learned_noalloc(const fo_mesh *m, const float *P, const float *norm, double *U,
                                                      int32_t fallback, int32_t smooth_sweeps, int32_t *used_network,
                                                      void *stream) {
  if (!m) return fail(FO_EINVAL, "fo_initial_guess_learned_noalloc: NULL mesh");
  const size_t need = llayout(m).total;
  if (need > FO_LEARNED_SCRATCH_BYTES)
    return fail(FO_EINVAL, "fo_initial_guess_learned_noalloc: mesh needs " + std::to_string(need) +
                               " bytes of workspace, more than the library's " +
                               std::to_string(size_t(FO_LEARNED_SCRATCH_BYTES)) + "-byte array");
  int dev = -1;
  FO_HIP_TRY(hipGetDevice(&dev));
  if (dev != m->device)
    return fail(FO_EINVAL, "fo_initial_guess_learned_noalloc: the mesh's device must be the current device");
  void *ws = nullptr;
  fo_status st = scratch_address(dev, &ws);
  if (st != FO_OK) return st;
  return learned_guess(m, P, norm, U, fallback, smooth_sweeps, ws, FO_LEARNED_SCRATCH_BYTES, used_network, nullptr,
                       static_cast<hipStream_t>(stream));
}

extern "C" fo_status fo_learned_targets(const fo_mesh *m, const double *U, const double *Us, float *T, void *stream) {
  if (!m || !U || !Us || !T) return fail(FO_EINVAL, "fo_learned_targets: NULL argument");
  if (m->view.L + 1 != NOUT / 2) return fail(FO_EINVAL, "fo_learned_targets: the network predicts 11 levels (L = 10)");
  const int64_t n = m->view.n_dofs;
  hipLaunchKernelGGL(targets_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     n, U, Us, T);
  FO_LAUNCH_CHECK("targets_kernel");
  return FO_OK;
}

extern "C" fo_status fo_feature_stats(const float *X, int64_t n_rows, float *norm, float *Xn, void *stream) {
  if (!X || !norm || n_rows < 2) return fail(FO_EINVAL, "fo_feature_stats: NULL argument or fewer than 2 rows");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(feature_stats_kernel, dim3(NIN), dim3(256), 0, s, X, n_rows, norm);
  FO_LAUNCH_CHECK("feature_stats_kernel");
  if (Xn) {
    const int64_t n = n_rows * NIN;
    hipLaunchKernelGGL(normalise_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, X, norm, Xn);
    FO_LAUNCH_CHECK("normalise_kernel");
  }
  return FO_OK;
}
