/* Device probes for the roofline figures: measurement infrastructure, not part of the
 * fo_stokes method ABI (libfo_probe.so, built beside libfo_stokes.so).  They give the FP64
 * vector FMA rate and the streaming HBM bandwidth the device actually reaches, so kernel
 * figures can be stated against measured as well as published peaks.  All pointers are
 * device memory owned by the caller; `stream` is a hipStream_t (NULL = default stream).
 * Each call only enqueues work; time it with events on the same stream.  Return 0, or -1
 * on invalid arguments or a failed launch. */
#ifndef FO_PROBE_H
#define FO_PROBE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* blocks x 256 threads; each thread runs `iters` steps of 16 independent FP64 FMA chains
 * (32 iters flops per thread) and writes one double to out[blocks * 256]. */
int fo_probe_fma64(int blocks, int iters, double *out, void *stream);

/* dst[0..n) = src[0..n) with 16-byte loads and stores over `blocks` x 256 threads (grid
 * stride); n even, src and dst 16-byte aligned and not overlapping.  Moves 16 n bytes. */
int fo_probe_copy(const double *src, double *dst, int64_t n, int blocks, void *stream);

/* Sum of src[0..n) into per-thread partials out[blocks * 256] (n even, src 16-byte
 * aligned): a read-only stream of 8 n bytes. */
int fo_probe_read(const double *src, int64_t n, int blocks, double *out, void *stream);

/* dst[0..n) = v with 16-byte stores (n even, dst 16-byte aligned): a write-only stream of
 * 8 n bytes. */
int fo_probe_write(double *dst, int64_t n, double v, int blocks, void *stream);

#ifdef __cplusplus
}
#endif
#endif
