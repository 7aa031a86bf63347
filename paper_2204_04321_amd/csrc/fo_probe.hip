// Device probes for the roofline figures (measurement only; not part of the fo_stokes ABI):
// the FP64 vector FMA rate and the HBM streaming bandwidth this device reaches, to report
// kernel figures against measured as well as published peaks.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "fo_probe.h"

namespace {

constexpr int CHAINS = 16;  // independent FMA chains per thread (cover the FMA latency)

__global__ __launch_bounds__(256) void fma64_kernel(int iters, double seed, double *__restrict__ out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double a[CHAINS];
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) a[i] = seed + 1e-9 * double(gid) + double(i);
  const double m = 0.999999999, c = 1e-12;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = fma(a[i], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s += a[i];
  out[gid] = s;
}

// four 16-byte loads in flight per thread before the stores
__global__ __launch_bounds__(256) void copy_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                    int64_t n2) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n2; i += 4 * stride) {
    const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n2; i += stride) dst[i] = src[i];
}

// read-only stream: each thread sums its 16-byte chunks, one partial per thread
__global__ __launch_bounds__(256) void read_kernel(const double2 *__restrict__ src, int64_t n2,
                                                    double *__restrict__ out) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (; i + 3 * stride < n2; i += 4 * stride) {
    const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    s0 += (a.x + b.x) + (c.x + d.x);
    s1 += (a.y + b.y) + (c.y + d.y);
  }
  for (; i < n2; i += stride) { s0 += src[i].x; s1 += src[i].y; }
  out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s0 + s1;
}

// write-only stream of a constant, 16-byte stores
__global__ __launch_bounds__(256) void write_kernel(double2 *__restrict__ dst, int64_t n2, double v) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const double2 w = make_double2(v, v);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n2; i += stride) dst[i] = w;
}

}  // namespace

// FP64 FMAs: blocks x 256 threads, each runs `iters` x 8 dependent-chain FMAs and writes one
// double to out[blocks * 256].  Returns 0, or -1 on bad arguments / launch failure.
extern "C" int fo_probe_fma64(int blocks, int iters, double *out, void *stream) {
  if (blocks < 1 || iters < 1 || !out) return -1;
  hipLaunchKernelGGL(fma64_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), iters, 1.0, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}


// dst[0..n) = src[0..n) with 16-byte loads and stores (n even, both 16-byte aligned).
extern "C" int fo_probe_copy(const double *src, double *dst, int64_t n, int blocks, void *stream) {
  if (!src || !dst || n < 2 || (n & 1) || blocks < 1) return -1;
  hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const double2 *>(src), reinterpret_cast<double2 *>(dst), n / 2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// sum of src[0..n) in per-thread partials out[blocks * 256] (n even, 16-byte aligned); moves 8 n bytes.
extern "C" int fo_probe_read(const double *src, int64_t n, int blocks, double *out, void *stream) {
  if (!src || !out || n < 2 || (n & 1) || blocks < 1) return -1;
  hipLaunchKernelGGL(read_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const double2 *>(src), n / 2, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// dst[0..n) = v (n even, 16-byte aligned); moves 8 n bytes.
extern "C" int fo_probe_write(double *dst, int64_t n, double v, int blocks, void *stream) {
  if (!dst || n < 2 || (n & 1) || blocks < 1) return -1;
  hipLaunchKernelGGL(write_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<double2 *>(dst), n / 2, v);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
