/*
 * bfx.h -- C ABI of an MI355X (gfx950) FX-correlator hot path.
 *
 * The calls follow the gulp model of the Bifrost paper (Sec. 3.5: a block
 * reads a ring buffer one "gulp" at a time; a ring holds four gulps by
 * default):
 * each call consumes one gulp that already sits in caller-owned device memory
 * and enqueues its work on the caller's HIP stream.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Ownership: the caller owns every device buffer.  accumulate / dump /
 *   fengine / beamform never allocate or free device memory.  A plan owns
 *   host metadata only, except a batched plan, which also owns a small device
 *   work list (allocated by bfx_xengine_create_batched, freed by destroy).
 * - Asynchrony: calls enqueue on `stream` (a hipStream_t; NULL = the null
 *   stream) and return.  Argument errors are detected on the host and
 *   returned before anything is enqueued; a failing HIP launch is reported as
 *   BFX_EHIP.  Device-side faults surface at the caller's next synchronisation.
 * - Threads: a plan may be used by one thread at a time; different plans are
 *   independent.  Error details are kept per thread (bfx_last_error_detail).
 * - Layouts are fixed (no layout flags):
 *     voltages   [time][channel][input], time slowest, input fastest;
 *                input = 2*antenna + polarisation;
 *     ci8        two int8 per sample, real byte first (Sec. 6: "8+8");
 *     ci4        one byte per sample, real part in bits 7..4, imaginary part
 *                in bits 3..0, each 4-bit two's complement (Sec. 6: "4+4"
 *                complex signed integers; the nibble order is this library's
 *                convention -- the paper does not state one);
 *     cf16       two IEEE binary16 per sample, real first;
 *     visibility [channel][p][2] with p = i*(i+1)/2 + j, j <= i (row-major
 *                lower triangle including the autocorrelations), the pair
 *                (re, im) of V_ij = sum_t x_i(t) * conj(x_j(t)).
 */
#ifndef BFX_H
#define BFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bfx_status {
    BFX_OK = 0,
    BFX_EINVAL = -1,  /* bad argument: null/misaligned pointer, bad size, dtype */
    BFX_ERANGE = -2,  /* integration would overflow the int32 accumulator     */
    BFX_EHIP = -3,    /* a HIP runtime call failed (detail has hipGetErrorString) */
    BFX_ENOTSUP = -4, /* valid request this build does not implement         */
    BFX_ENOMEM = -5   /* host or device allocation at plan creation failed   */
} bfx_status;

typedef enum bfx_dtype {
    BFX_I8 = 1,   /* real int8 (F-engine input)               */
    BFX_CI4 = 2,  /* 4+4-bit complex, see layout above         */
    BFX_CI8 = 3,  /* 8+8-bit complex                           */
    BFX_CF16 = 4, /* binary16 complex                          */
    BFX_CF32 = 5, /* binary32 complex                          */
    BFX_CI32 = 6, /* int32 complex (integer visibilities)      */
    BFX_CF64 = 7  /* binary64 complex (running sums)           */
} bfx_dtype;

/* hipStream_t, passed as a plain pointer so that this header needs no HIP
 * include.  NULL selects the null stream.                                   */
typedef void *bfx_stream;

/* Flag for bfx_xengine_accumulate: write V instead of adding to d_acc. */
#define BFX_ACC_OVERWRITE 1u

typedef struct bfx_xengine bfx_xengine; /* opaque plan */

/* Human-readable name of a status code (static storage, never NULL). */
const char *bfx_strerror(bfx_status s);

/* Detail of the last error raised on the calling thread ("" if none).
 * Valid until the next bfx_* call on this thread.                          */
const char *bfx_last_error_detail(void);

/* ------------------------------------------------------------------------ */
/* X-engine (Sec. 2.2 linear-algebra module; Sec. 7 lists correlation as the
 * capability being added).  Per channel f it forms the Hermitian visibility
 * matrix V_f = sum_t x_t x_t^H over the time samples of a gulp, keeping the
 * lower triangle only.
 *
 * Input dtypes and results:
 *   BFX_CI4, BFX_CI8 -> int32 visibilities, bit-exact (int8 MFMA, int32
 *                       accumulation; the sums are exact integers);
 *   BFX_CF16         -> binary32 visibilities (FP16 MFMA, FP32 accumulation).
 */

/* Largest number of samples one integration (the samples accumulated since the
 * last BFX_ACC_OVERWRITE) may hold before an int32 visibility could overflow:
 *   ci8: floor((2^31-1) / (2*128^2)) = 65535
 *   ci4: floor((2^31-1) / (2*8^2))   = 16777215
 *   cf16: INT64_MAX (no integer bound).
 * Returns -1 for any other dtype.                                           */
int64_t bfx_xengine_max_ntime(bfx_dtype in);

/* Create a plan for one array of `ninput` inputs and `nchan` channels.
 * ninput must be a positive multiple of 4 (<= 8192), nchan positive
 * (<= 65536), `in` one of BFX_CI4, BFX_CI8, BFX_CF16.  Host-only: no device
 * memory is allocated.  On success *plan receives the new plan.            */
bfx_status bfx_xengine_create(bfx_xengine **plan, int32_t ninput, int32_t nchan, bfx_dtype in);

/* Create a batched plan: `nsub` (<= 4096) independent arrays (subarrays /
 * subbands) of ninput[k] inputs and nchan[k] channels, correlated by one
 * persistent launch (ci4 or ci8 input; at most 2^24 work items in all).
 * Inputs and outputs live in two arenas, subarrays in order k = 0, 1, ...:
 *   input arena:  subarray k's gulp is [ntime][nchan_k][ninput_k] contiguous
 *                 and occupies ntime * R_k bytes, R_k = its row bytes rounded
 *                 up to a multiple of 256 (so offsets scale with ntime);
 *   output arena: subarray k's [nchan_k][p][2] visibilities, each block
 *                 rounded up to a multiple of 256 bytes.
 * bfx_xengine_sub_offsets gives both offsets.  Allocates the device work
 * list and subarray table on the current device (BFX_ENOMEM / BFX_EHIP on
 * failure); accumulate on a batched plan must run on that device.  Results
 * are bit-identical to one plain plan per subarray.                         */
bfx_status bfx_xengine_create_batched(bfx_xengine **plan, int32_t nsub, const int32_t *ninput,
                                      const int32_t *nchan, bfx_dtype in);

/* Free a plan (NULL is accepted).  Waits for nothing: the caller must not
 * destroy a batched plan while work enqueued with it is still running.      */
bfx_status bfx_xengine_destroy(bfx_xengine *plan);

/* Bytes of one input gulp of `ntime` samples, and bytes of the visibility
 * buffer (the accumulator; int32 pairs or binary32 pairs).  For batched plans
 * these are arena sizes.  Return 0 on a bad argument.                       */
size_t bfx_xengine_in_bytes(const bfx_xengine *plan, int64_t ntime);
size_t bfx_xengine_out_bytes(const bfx_xengine *plan);

/* Subarray k of a batched plan (k = 0 for a plain plan): byte offset of its
 * [ntime][nchan_k][ninput_k] gulp inside the input arena, and byte offset of
 * its [nchan_k][p][2] visibilities inside the output arena.  Every offset is a
 * multiple of 256.                                                          */
bfx_status bfx_xengine_sub_offsets(const bfx_xengine *plan, int32_t k, int64_t ntime,
                                   int64_t *in_offset, int64_t *out_offset);

/* Samples accumulated since the last BFX_ACC_OVERWRITE (host bookkeeping). */
int64_t bfx_xengine_nacc(const bfx_xengine *plan);

/* ------------------------------------------------------------------------ */
/* Kernel variants and autotuning (the batched persistent launch of the gulp
 * model, Sec. 3.5, tuned per array shape).  A plan runs one of
 * bfx_xengine_num_variants(plan) <= BFX_XENGINE_VARIANTS kernel variants;
 * every variant computes the same result (integer paths: the same bits):
 *   0, 1  the plan's own MFMA type (int8 for ci4/ci8, binary16 for cf16), with
 *         four or eight waves issuing the stage copies into LDS;
 *   2, 3  ci4 plans (not batched): the same on FP8 MFMA -- every 4-bit
 *         value is exact in e4m3, products and sums are integers below 2^23
 *         and binary32 accumulates them exactly (Sec. 6: 4+4-bit voltages;
 *         Sec. 2.2: quantized types down to a few bits);
 *         cf16 plans: variants 0, 1 with each LDS stage read two stages
 *         ahead (the same arithmetic in the same order; gulps of at most 16
 *         samples run variant 0 or 1 instead).
 *
 * bfx_xengine_autotune times each variant on the plan's shape with `ntime`
 * samples (1 <= ntime <= min(bfx_xengine_max_ntime, 2^20)) on `stream` and
 * keeps the fastest.  It allocates (and frees) one input gulp, filled with
 * seeded pseudo-random samples spread like the workloads' (not a constant),
 * and one visibility buffer of device memory, waits for the stream, and
 * leaves nacc unchanged.  times_us, if not NULL, receives the best time of
 * each variant (host float[BFX_XENGINE_VARIANTS], microseconds; 0 for
 * variants the plan does not have).  If the environment
 * variable BFX_TUNE_CACHE names a file, the choice is appended to it as one
 * JSON line {"arch", "dtype", "shape", "variant", "us"}, and plans created
 * later for the same (device architecture, dtype, shape) start with the
 * cached variant (the last matching line wins); otherwise plans start with
 * variant 0.  Returns BFX_EINVAL for a bad ntime, BFX_EHIP if a device
 * allocation or launch fails (the plan keeps its variant).               */
#define BFX_XENGINE_VARIANTS 4
bfx_status bfx_xengine_autotune(bfx_xengine *plan, int64_t ntime, float *times_us, bfx_stream stream);

/* The plan's current variant (-1 for NULL), the number of variants it has
 * (-1 for NULL), and an explicit choice (BFX_EINVAL outside
 * [0, bfx_xengine_num_variants(plan))).                                     */
int32_t bfx_xengine_variant(const bfx_xengine *plan);
int32_t bfx_xengine_num_variants(const bfx_xengine *plan);
bfx_status bfx_xengine_set_variant(bfx_xengine *plan, int32_t variant);

/* Look up a tune-cache file without a device: the variant cached for
 * (arch, dtype, shape), or -1 if there is none (or the file cannot be read).
 * shape is "NxF" for a plan with N inputs and F channels, and
 * "b:N1xF1,N2xF2,..." for a batched plan; dtype is "ci4", "ci8" or "cf16". */
int32_t bfx_tune_cache_lookup(const char *path, const char *arch, const char *dtype, const char *shape);

/* Correlate one gulp.
 *   d_in   device, [ntime][nchan][ninput] samples of the plan's dtype (for a
 *          batched plan: the input arena), 16-byte aligned;
 *   ntime  samples in the gulp, >= 1;
 *   d_acc  device, the visibility buffer (bfx_xengine_out_bytes), 16-byte
 *          aligned; with BFX_ACC_OVERWRITE it is overwritten with this gulp's
 *          V, otherwise V is added to it.
 * Returns BFX_ERANGE, without enqueueing, when the integer bound
 * bfx_xengine_max_ntime would be exceeded by nacc + ntime.  Results do not
 * depend on launch shape or scheduling (integer sums are exact).
 * Graph capture: the bound is checked when a call is captured, and every
 * replay of the graph repeats the captured launches.  A call without
 * BFX_ACC_OVERWRITE is therefore accepted on a capturing stream only after an
 * overwrite call on this plan captured into the same graph (each replay then
 * restarts the integration); otherwise it returns BFX_ENOTSUP without
 * enqueueing.                                                               */
bfx_status bfx_xengine_accumulate(bfx_xengine *plan, const void *d_in, int64_t ntime, void *d_acc,
                                  uint32_t flags, bfx_stream stream);

/* Batched correlation for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results as a batched plan built from
 * (nsub, ninput, nchan, in) followed by bfx_xengine_accumulate with
 * BFX_ACC_OVERWRITE, but with no plan.  The subarray table and work list
 * are built on the device, per call, in a fixed scratch array in the
 * library's device memory (about 0.5 MiB on each device it runs on, held
 * until the process ends); nothing is allocated or freed.
 *   nsub      1 .. 16 subarrays (ninput[k] a positive multiple of 4 <= 8192,
 *             nchan[k] in [1, 65536]); at most 65536 work-list entries in all
 *             (BFX_ENOTSUP beyond: use a batched plan);
 *   in        BFX_CI4 or BFX_CI8;
 *   d_in      device input arena laid out as for bfx_xengine_create_batched;
 *   ntime     1 .. bfx_xengine_max_ntime(in) samples;
 *   d_acc     device visibility arena (same layout and size as the plan's);
 *   flags     must be BFX_ACC_OVERWRITE (no integration state is kept
 *             between calls; BFX_ENOTSUP otherwise).
 * Every call on one device uses that device's one scratch array: calls that
 * overlap on one device (other streams, other host threads) race, and each
 * call leaves its work list there for the next to overwrite.  Argument errors
 * are returned before anything is enqueued.                                 */
bfx_status bfx_xengine_accumulate_batched_noalloc(int32_t nsub, const int32_t *ninput, const int32_t *nchan,
                                                  bfx_dtype in, const void *d_in, int64_t ntime, void *d_acc,
                                                  uint32_t flags, bfx_stream stream);

/* Hand over an integration (Sec. 4.1 accumulate block).
 *   d_acc    device visibility buffer filled by accumulate;
 *   d_out    device, may be NULL or == d_acc (no copy); otherwise the
 *            visibilities are copied there (same dtype and size);
 *   d_run64  device, may be NULL; otherwise [nchan][p][2] binary64 running
 *            sum, updated as d_run64 += (double)d_acc.
 * Does not change nacc: start the next integration with BFX_ACC_OVERWRITE.  */
bfx_status bfx_xengine_dump(bfx_xengine *plan, const void *d_acc, void *d_out, double *d_run64,
                            bfx_stream stream);

/* Correlate one binary16 gulp and fold it straight into a binary64 running
 * sum (the X-engine's cross-multiply, Sec. 2.2 and 7, with the dump of the
 * Sec. 4.1 accumulate block fused into its store):
 *   d_run64[k] += (double)V_k,
 * V the binary32 visibilities that bfx_xengine_accumulate with
 * BFX_ACC_OVERWRITE would write -- so the result has the same bits as that
 * call followed by bfx_xengine_dump(plan, d_acc, NULL, d_run64) -- without
 * writing and reading back the binary32 buffer.
 *   plan     a single-array BFX_CF16 plan (BFX_ENOTSUP otherwise);
 *   d_in     device cf16 gulp [ntime][nchan][ninput], 16-byte aligned;
 *   ntime    1 .. 65535 samples (one launch; BFX_ERANGE beyond: longer
 *            integrations accumulate into a binary32 buffer and dump it);
 *   d_run64  device binary64 [nchan][p][2] running sum (2 x out_bytes),
 *            16-byte aligned, read and written.
 * Does not change the plan's accumulation count.  Argument errors are
 * returned before anything is enqueued.                                     */
bfx_status bfx_xengine_accumulate_run64(bfx_xengine *plan, const void *d_in, int64_t ntime, double *d_run64,
                                        bfx_stream stream);

/* ------------------------------------------------------------------------ */
/* F-engine (Sec. 2.2 FFT and quantize modules; Sec. 6: 204.8 MS/s real
 * samples become 4096 channels, i.e. a real transform of 2N points keeps the
 * N channels below Nyquist).
 *   d_in     device int8 [nspec*nfft][ninput]: real samples, inputs fastest;
 *   nfft     transform length, a power of two in [64, 8192];
 *   ninput   positive, even;
 *            (this build implements nfft = 4096 with ninput a multiple of
 *            8 and returns BFX_ENOTSUP for the other valid shapes);
 *   nspec    number of non-overlapping frames per input (rectangular window);
 *   d_scale  device float[nfft/2], per-channel requantization scale (ignored
 *            for BFX_CF32 output);
 *   d_out    device [nspec][nfft/2][ninput] of `out`:
 *              BFX_CI8:  q = clamp(round_half_even(scale_k * X), -127, 127)
 *                        for the real and imaginary parts separately;
 *              BFX_CF32: the unscaled spectrum X in binary32.
 * X_s[k][i] = sum_{n<nfft} x[s*nfft+n][i] exp(-2 pi i k n / nfft),
 * k = 0 .. nfft/2-1 (bin 0 = DC, Nyquist dropped, no normalisation).
 * Computed in binary32.  The ci8 output can be fed straight to an X-engine
 * plan with ninput inputs and nfft/2 channels.                              */
bfx_status bfx_fengine(const int8_t *d_in, int32_t ninput, int32_t nfft, int64_t nspec,
                       const float *d_scale, void *d_out, bfx_dtype out, bfx_stream stream);

/* ------------------------------------------------------------------------ */
/* Phase-and-sum beamformer with square-law detection and integration (Sec. 6
 * DRX pipeline; Sec. 4.1 detect and accumulate blocks).
 *   d_x    device cf16 [ntime][nchan][ninput];
 *   d_w    device cf16 [nchan][nbeam][ninput] steering weights, applied
 *          without conjugation: y[b][f][t] = sum_i w[f][b][i] * x[t][f][i];
 *   d_out  device float [nbeam][nchan][ntime/navg]:
 *          P[b][f][u] = sum_{t=u*navg}^{u*navg+navg-1} |y[b][f][t]|^2.
 * ntime must be a positive multiple of navg (<= 2^30); ninput a positive
 * multiple of 32 (<= 8192); nbeam in [1, 256].  binary16 products, binary32
 * accumulation of y and of P.  This build integrates navg = 1, 2, 4, 8, 16 or
 * 32 samples and returns BFX_ENOTSUP for other valid navg, and for shapes
 * needing more than (2^32-1)/256 workgroups (ceil(nchan/8)*8 *
 * ceil(ntime/256) * ceil(nbeam/32)); split such a gulp in time.             */
bfx_status bfx_beamform_detect(const void *d_x, const void *d_w, int32_t ninput, int32_t nchan,
                               int32_t nbeam, int64_t ntime, int32_t navg, float *d_out,
                               bfx_stream stream);

/* ------------------------------------------------------------------------ */
/* T-engine: channelized spectra back to complex voltages (Sec. 6: the TBN
 * pipeline's T-engine -- convert to floating point, reduce the bandwidth,
 * shift along the channel axis, inverse transform, complex mixer for
 * sub-channel tuning, quantize to 8+8 -- and the DRX T-engine, whose inverse
 * transform runs on the GPU and whose output is quantized to 4+4).
 *   d_in     device ci8 spectra [nspec][nchan][ninput] (layout above);
 *   chan0    first channel of the band, chan0 + nfft <= nchan;
 *   nfft     band width in channels = output samples per frame, a power of
 *            two in [64, 8192]; ninput positive and even (this build
 *            transforms nfft = 4096 with ninput a multiple of 8 and returns
 *            BFX_ENOTSUP for the other valid shapes);
 *   mix_num, mix_den  mixer frequency mix_num / mix_den cycles per output
 *            sample (0 <= mix_num, 1 <= mix_den <= 2^31-1);
 *   d_out    device [nspec*nfft][ninput] samples of `out`: BFX_CI8 (real byte
 *            first) or BFX_CI4 (real nibble high), 16-byte aligned.
 * With X_k = d_in[s][chan0 + k][i] and t = s*nfft + n:
 *   z[n]  = (1/nfft) sum_{k<nfft} X_k exp(+2 pi i (k - nfft/2) n / nfft)
 *           (the band centre chan0 + nfft/2 maps to zero frequency),
 *   z'[n] = z[n] exp(+2 pi i ((mix_num * t) mod mix_den) / mix_den),
 *   q     = clamp(round_half_even(scale * z'), -L, L) for the real and
 *           imaginary parts, L = 127 (ci8) or 7 (ci4; -8 is never written).
 * Computed in binary32 (the mixer phase index is exact integer arithmetic);
 * a code may differ by one from the exact result where scale * z' lies within
 * the binary32 error of a half-integer.                                      */
bfx_status bfx_tengine(const int8_t *d_in, int32_t nchan, int32_t ninput, int64_t nspec, int32_t chan0,
                       int32_t nfft, int64_t mix_num, int64_t mix_den, float scale, void *d_out, bfx_dtype out,
                       bfx_stream stream);

/* ------------------------------------------------------------------------ */
/* Phase-and-sum beamformer on 4+4-bit voltages with integer weights (Sec. 6:
 * the DRX pipeline's GPU beamformer consumes the 4+4 complex samples
 * directly), square-law detection and integration (Sec. 4.1 detect and
 * accumulate blocks).  Exact integer arithmetic up to one final conversion:
 *   d_x     device ci4 [ntime][nchan][ninput] (layout above);
 *   d_w     device int8 [nchan][nbeam][ninput][2] weights (re, im), any int8
 *           value, applied without conjugation;
 *   d_scale device float[nbeam], per-beam scale of the weights (the physical
 *           weight of beam b is scale_b * w);
 *   d_out   device float [nbeam][nchan][ntime/navg]:
 *             y[b][f][t] = sum_i w[f][b][i] x[t][f][i]        (exact integers)
 *             S[b][f][u] = sum_{t=u*navg}^{u*navg+navg-1} |y[b][f][t]|^2 (exact)
 *             P[b][f][u] = (float)((double)scale_b * (double)scale_b * (double)S),
 *           each conversion and product rounded to nearest even, in that order.
 * ninput a positive multiple of 64 (<= 8192), nchan in [1, 65536], nbeam in
 * [1, 256], ntime a positive multiple of navg (<= 2^30).  d_x and d_w 16-byte
 * aligned, d_scale and d_out 4-byte aligned.  This build integrates navg = 1,
 * 2, 4, ..., 64 samples and returns BFX_ENOTSUP for other valid navg, and for
 * shapes needing more than (2^32-1)/256 workgroups (ceil(nchan/8)*8 *
 * ceil(ntime/256) * ceil(nbeam/32)).  int8 MFMA with int32 accumulation:
 * every partial sum is bounded by 2 * 8192 * 128 * 128 < 2^31.              */
bfx_status bfx_beamform_ci4(const void *d_x, const int8_t *d_w, const float *d_scale, int32_t ninput,
                            int32_t nchan, int32_t nbeam, int64_t ntime, int32_t navg, float *d_out,
                            bfx_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* BFX_H */
