/*
 * sbs_probe.h -- measurement helpers of libsbs: kernels that only move bytes,
 * for the bandwidth ceiling the solves are compared with and for calibrating
 * hardware counters.  They are not part of the method and compute nothing.
 * Same conventions as sbs.h (status codes, device pointers, void* stream,
 * asynchronous launches).
 */
#ifndef SBS_PROBE_H
#define SBS_PROBE_H

#include <stdint.h>

#include "sbs.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Grid-stride sweep over `bytes` (a multiple of 16) of contiguous device
 * memory, 16 bytes per lane per access, `unroll` (1, 2, 4, 8) accesses in
 * flight per lane, `wg_per_cu` workgroups of 256 threads per compute unit.
 *  mode 0: copy src -> dst (non-temporal stores);
 *  mode 1: read src only (dst must hold 16 bytes per launched thread; it is
 *          written only in the practically impossible case that a checksum
 *          matches a fixed constant);
 *  mode 2: write dst only.
 * Pointers 16-byte aligned.  Errors: SBS_ERR_INVALID_ARG, SBS_ERR_DEVICE.
 */
sbs_status sbs_probe_linear(int32_t mode, const void *src, void *dst,
                            int64_t bytes, int32_t unroll, int32_t wg_per_cu,
                            void *stream);

/*
 * The access pattern of the partitioned solve with no arithmetic, in place
 * on an interleaved (n, m) FP64 array x (x[i*m + j]): workgroups of S
 * consecutive systems, rows cut into blocks of lb (16, 32, 64) rows, each
 * lane loading its block of `vec` (1 or 2) adjacent systems (8- or 16-byte
 * accesses), one workgroup barrier, then non-temporal stores of the same
 * values to the same places (x is unchanged).  Needs n % lb == 0, m % S == 0,
 * S % vec == 0 and (S / vec) * (n / lb) <= 1024 threads (and within the
 * register budget of the shape).  16 bytes of HBM traffic per element.
 * Errors: SBS_ERR_INVALID_ARG, SBS_ERR_DEVICE.
 */
sbs_status sbs_probe_blocks(double *x, int64_t n, int64_t m, int32_t lb,
                            int32_t vec, int32_t S, int32_t wg_per_cu,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SBS_PROBE_H */
