// Launchers of the linear-algebra kernels used by the Newton driver.
#pragma once

#include "fo_internal.h"

namespace fo {
fo_status spmv(const fo_mesh *mesh, const void *vals, int dtype, const double *x, double *y, hipStream_t s);
fo_status colblock_factor(const fo_mesh *mesh, const void *vals, int dtype, float *fac, hipStream_t s);
fo_status colblock_apply(const fo_mesh *mesh, const float *fac, const double *r, double *z, hipStream_t s);
// z = P0 y + M^{-1} (r - JP y): the column smoother after the plane correction of the two-level
// preconditioner (W32: FP32 collapse weights [V][L+1][2][2], JP: FP32 J P0 by column, y: [2 V])
fo_status colblock_apply_correction(const fo_mesh *mesh, const float *fac, const float *W32, const float *JP,
                                    const double *y, const double *r, double *z, hipStream_t s);
int multidot_blocks(int64_t n);
// out[0..nv-1] = V_i . w, out[nv] = w . w (partial: multidot_blocks(n) * (nv + 1) doubles;
// n and ld even, FO_EINVAL otherwise)
fo_status multidot(int64_t n, const double *V, int64_t ld, int nv, const double *w, double *partial,
                   double *out, hipStream_t s);
int dot2_blocks(int64_t n);
// out[0] = a . w, out[1] = w . w (partial: 2 dot2_blocks(n) doubles; n even, FO_EINVAL otherwise)
fo_status dot2(int64_t n, const double *a, const double *w, double *partial, double *out, hipStream_t s);
// w += sign * sum_i h_i V_i (n and ld even, FO_EINVAL otherwise)
fo_status multiaxpy(int64_t n, const double *V, int64_t ld, int nv, const double *h, double *w, double sign,
                    hipStream_t s);
// x += alpha p, r -= alpha q with alpha = num[0] / den[0] read on the device
fo_status cg_step(int64_t n, const double *num, const double *den, const double *p, const double *q, double *x,
                  double *r, hipStream_t s);
fo_status axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
fo_status xpay(int64_t n, const double *x, double a, const double *y, double *z, hipStream_t s);
}  // namespace fo
