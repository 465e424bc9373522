/*
 * bfx_probe.h -- peak probes of libbfx (measurement utilities, not part of the
 * FX method).  The hot-path kernels are priced against the device's dense MFMA
 * and HBM peaks; these calls measure what the device sustains, so that both
 * fractions can be reported.  They compute nothing that is checked.
 */
#ifndef BFX_PROBE_H
#define BFX_PROBE_H

#include "bfx.h"

#ifdef __cplusplus
extern "C" {
#endif

#define BFX_PROBE_MFMA_I8 0  /* v_mfma_i32_32x32x32_i8, int8 -> int32       */
#define BFX_PROBE_MFMA_F16 1 /* v_mfma_f32_32x32x16_f16, binary16 -> binary32 */

/* Enqueue the MFMA probe: nblocks workgroups of 8 waves, each wave issuing
 * 8 x iters MFMAs of `kind` into 8 independent accumulators (no memory
 * traffic).  d_sink: device int32[nblocks], written only in a case the data
 * never produces (it keeps the loop from being removed).  Time it with events
 * on `stream`; bfx_probe_mfma_ops gives its operation count (2 per
 * multiply-add).  BFX_EINVAL for a bad kind, iters <= 0, nblocks outside
 * [1, 2^20] or a NULL d_sink.                                               */
bfx_status bfx_probe_mfma(int32_t kind, int32_t iters, int32_t nblocks, int32_t *d_sink, bfx_stream stream);
int64_t bfx_probe_mfma_ops(int32_t kind, int32_t iters, int32_t nblocks);

/* Enqueue the read probe: nblocks workgroups of 256 lanes read the nbytes of
 * device buffer d_buf once (16-byte loads, grid-stride) and fold them to one
 * word per workgroup into d_sink (device int32[nblocks], written only where
 * the fold is non-zero).  d_buf 16-byte aligned, nbytes a positive multiple
 * of 16, nblocks in [1, 2^23]; BFX_EINVAL otherwise.                        */
bfx_status bfx_probe_read(const void *d_buf, int64_t nbytes, int32_t nblocks, int32_t *d_sink,
                          bfx_stream stream);

#define BFX_PROBE_LDS_TR16 2 /* ds_read_b64_tr_b16 (transposing, 8 bytes per lane)  */
#define BFX_PROBE_LDS_TR8 3  /* ds_read_b64_tr_b8                                   */
#define BFX_PROBE_LDS_B128 4 /* ds_read_b128 (16 bytes per lane, no transpose)      */

/* Enqueue the LDS read probe: nblocks workgroups of 8 waves, each wave issuing
 * 12 x iters LDS reads of `kind` inside a 16 KiB LDS buffer (the X-engines'
 * conflict-free transposing pattern for the tr kinds, consecutive 16-byte
 * chunks for b128) and folding the results into d_sink (device
 * int32[nblocks], written only in a case the data never produces).
 * bfx_probe_lds_bytes gives the bytes it reads.  BFX_EINVAL for a bad kind,
 * iters <= 0, nblocks outside [1, 2^20] or a NULL d_sink.                    */
bfx_status bfx_probe_lds(int32_t kind, int32_t iters, int32_t nblocks, int32_t *d_sink, bfx_stream stream);
int64_t bfx_probe_lds_bytes(int32_t kind, int32_t iters, int32_t nblocks);

#ifdef __cplusplus
}
#endif
#endif /* BFX_PROBE_H */
