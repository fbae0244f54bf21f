/* mpx_probe.h -- measurement aid of libmpx (not part of the arithmetic).
 *
 * Times the VALU instruction kinds the multicomponent kernels consist of, so
 * that the FP64 and FP32 vector peaks used for the rooflines can be measured
 * on the device rather than taken from a datasheet.
 *
 * mpx_probe_valu launches threads / 256 workgroups of 256 threads; each thread
 * runs 16 independent chains of 4 * iters dependent operations of one kind
 * (x := x + y, or x := fma(x, y, z)) and stores one value to out[thread]
 * (device buffer of `threads` doubles for the F64 kinds, floats for F32).
 * The caller times the launch on `stream` (asynchronous); lane-operations =
 * threads * iters * 64.  mpx_probe_threads() is the grid the probe is meant
 * for: 8 workgroups of 256 threads per compute unit.  Returns MPX_EINVAL for
 * a bad kind, iters < 1, threads not a positive multiple of 256 or a null
 * out; MPX_EDEVICE on a launch failure. */
#ifndef MPX_PROBE_H
#define MPX_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MPX_PROBE_F64_ADD = 0, MPX_PROBE_F64_FMA = 1, MPX_PROBE_F32_ADD = 2, MPX_PROBE_F32_FMA = 3 };

int64_t mpx_probe_threads(void);
int mpx_probe_valu(int kind, int64_t iters, void *out, int64_t threads, void *stream);

/* FP64 issue rate at low occupancy: one workgroup of 256 * waves_per_simd
 * threads per compute unit (waves_per_simd = 1..4), each thread running
 * `chains` (1, 2, 4, 8 or 16) independent chains of 8 * iters dependent
 * additions and storing one double to out[thread] (device buffer of out_len
 * doubles, at least mpx_probe_chains_threads(waves_per_simd)).  Lane-operations
 * = threads * iters * 8 * chains; the caller times the launch on `stream`.
 * mpx_probe_chains_threads returns 0 for waves_per_simd outside 1..4.
 * Returns MPX_EINVAL for bad chains, waves_per_simd, iters < 1, a null or too
 * short out; MPX_EDEVICE on a launch failure. */
int64_t mpx_probe_chains_threads(int waves_per_simd);
int mpx_probe_chains(int chains, int waves_per_simd, int64_t iters, void *out, int64_t out_len,
                     void *stream);

#ifdef __cplusplus
}
#endif

#endif
