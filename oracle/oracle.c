/*
 * oracle.c -- plain, slow CPU reference for the FX-correlator hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the GPU path.
 *
 * Everything here is the textbook definition written out as loops, in int64
 * for integer data and in double precision for floating point:
 *
 *   - unpack of 4+4-bit and 8+8-bit complex signed integers
 *     (paper Sec. 6, packet capture and TBN pipeline: voltages travel as
 *      "4+4" complex signed integers and are unpacked to "8+8");
 *   - the X-engine product V_f = sum_t x_t x_t^H per channel
 *     (paper Sec. 2.2 linear-algebra module; Sec. 7 lists correlation as the
 *      capability being built; the product itself is the standard FX
 *      correlator definition V_ij = sum_t x_i(t) conj(x_j(t)));
 *   - a direct DFT of real frames (paper Sec. 2.2 FFT module; Sec. 6: the
 *     F-engine turns 204.8 MS/s into 4096 channels, i.e. a real transform of
 *     2N points keeps N channels);
 *   - requantization to 8-bit (paper Sec. 2.2 quantize module; Sec. 4.1
 *     quantize block);
 *   - phase-and-sum beamforming with square-law detection and integration
 *     (paper Sec. 6 DRX pipeline; Sec. 4.1 detect and accumulate blocks).
 *
 * Where the paper is silent, the reading taken is written next to the code.
 * Optional OpenMP over the outermost (channel / spectrum) loop does not change
 * any arithmetic: every output element is computed by exactly one thread in the
 * same order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Unpack.  Reading: one byte per 4+4 sample, real part in the high nibble,
 * imaginary part in the low nibble, each a 4-bit two's-complement integer.
 * 8+8 samples are two int8 bytes, real first.                               */

static int nibble_value(int nib)
{
    int v = nib & 15;
    if (v >= 8) v -= 16;
    return v;
}

int orc_unpack_ci4(const uint8_t *in, int64_t n, int32_t *re, int32_t *im)
{
    if (!in || !re || !im || n < 0) return ORC_EINVAL;
    for (int64_t k = 0; k < n; ++k) {
        int b = in[k];
        re[k] = nibble_value(b >> 4);
        im[k] = nibble_value(b);
    }
    return ORC_OK;
}

int orc_unpack_ci8(const int8_t *in, int64_t n, int32_t *re, int32_t *im)
{
    if (!in || !re || !im || n < 0) return ORC_EINVAL;
    for (int64_t k = 0; k < n; ++k) {
        re[k] = in[2 * k];
        im[k] = in[2 * k + 1];
    }
    return ORC_OK;
}

/* Read sample (t, f, i) of a [t][f][i] voltage array.  dtype 4 = ci4 (one
 * byte per sample), dtype 8 = ci8 (two bytes per sample).                    */
static void sample_at(const void *in, int dtype, int64_t t, int32_t nchan,
                      int32_t ninput, int32_t f, int32_t i, int64_t *re, int64_t *im)
{
    int64_t idx = (t * nchan + f) * (int64_t)ninput + i;
    if (dtype == 4) {
        int b = ((const uint8_t *)in)[idx];
        *re = nibble_value(b >> 4);
        *im = nibble_value(b);
    } else {
        const int8_t *p = (const int8_t *)in;
        *re = p[2 * idx];
        *im = p[2 * idx + 1];
    }
}

/* ------------------------------------------------------------------------ */
/* Integer X-engine.  For channels f0..f0+nf-1 and time samples t0..t0+nt-1:
 *
 *   V_ij = sum_t x_i(t) * conj(x_j(t))
 *   Re V_ij = sum_t re_i re_j + im_i im_j
 *   Im V_ij = sum_t im_i re_j - re_i im_j
 *
 * full == 0: lower triangle j <= i, packed row-major, p = i(i+1)/2 + j,
 *            out is [nf][N(N+1)/2][2] int64.
 * full != 0: every (i, j), out is [nf][N][N][2] int64.                      */
int orc_xengine_int(const void *in, int dtype, int64_t ntime, int32_t nchan,
                    int32_t ninput, int32_t f0, int32_t nf, int64_t t0, int64_t nt,
                    int full, int64_t *out, int nthreads)
{
    if (!in || !out || (dtype != 4 && dtype != 8)) return ORC_EINVAL;
    if (ntime < 0 || nchan <= 0 || ninput <= 0) return ORC_EINVAL;
    if (f0 < 0 || nf < 0 || f0 + nf > nchan) return ORC_EINVAL;
    if (t0 < 0 || nt < 0 || t0 + nt > ntime) return ORC_EINVAL;
    const int64_t N = ninput;
    const int64_t per_chan = full ? N * N : N * (N + 1) / 2;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int32_t ff = 0; ff < nf; ++ff) {
        int32_t f = f0 + ff;
        int64_t *o = out + (int64_t)ff * per_chan * 2;
        for (int64_t i = 0; i < N; ++i) {
            int64_t jmax = full ? N - 1 : i;
            for (int64_t j = 0; j <= jmax; ++j) {
                int64_t acc_re = 0, acc_im = 0;
                for (int64_t t = t0; t < t0 + nt; ++t) {
                    int64_t ar, ai, br, bi;
                    sample_at(in, dtype, t, nchan, ninput, f, (int32_t)i, &ar, &ai);
                    sample_at(in, dtype, t, nchan, ninput, f, (int32_t)j, &br, &bi);
                    acc_re += ar * br + ai * bi;
                    acc_im += ai * br - ar * bi;
                }
                int64_t p = full ? i * N + j : i * (i + 1) / 2 + j;
                o[2 * p] = acc_re;
                o[2 * p + 1] = acc_im;
            }
        }
    }
    return ORC_OK;
}

/* The same product on decoded double-precision voltages (used for the FP16
 * X-engine: every FP16 value is exact in double, so this is the exact sum up
 * to double rounding).  re/im are [nt][nf][N]; out is [nf][P][2] double.     */
int orc_xengine_f64(const double *re, const double *im, int64_t nt, int32_t nf,
                    int32_t ninput, int full, double *out, int nthreads)
{
    if (!re || !im || !out || nt < 0 || nf <= 0 || ninput <= 0) return ORC_EINVAL;
    const int64_t N = ninput;
    const int64_t per_chan = full ? N * N : N * (N + 1) / 2;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int32_t f = 0; f < nf; ++f) {
        double *o = out + (int64_t)f * per_chan * 2;
        for (int64_t i = 0; i < N; ++i) {
            int64_t jmax = full ? N - 1 : i;
            for (int64_t j = 0; j <= jmax; ++j) {
                double acc_re = 0.0, acc_im = 0.0;
                for (int64_t t = 0; t < nt; ++t) {
                    int64_t a = (t * nf + f) * N + i;
                    int64_t b = (t * nf + f) * N + j;
                    acc_re += re[a] * re[b] + im[a] * im[b];
                    acc_im += im[a] * re[b] - re[a] * im[b];
                }
                int64_t p = full ? i * N + j : i * (i + 1) / 2 + j;
                o[2 * p] = acc_re;
                o[2 * p + 1] = acc_im;
            }
        }
    }
    return ORC_OK;
}

/* Running sum of dumps: run[k] += dump[k] in double (integration across
 * dumps, paper Sec. 4.1 accumulate block).                                  */
int orc_accumulate_f64(double *run, const double *dump, int64_t n)
{
    if (!run || !dump || n < 0) return ORC_EINVAL;
    for (int64_t k = 0; k < n; ++k) run[k] += dump[k];
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Direct DFT of real frames.  x is [nspec*nfft][ninput] int8 (time-major,
 * inputs innermost).  Frame s of input i is x[s*nfft + n][i], n < nfft.
 *
 *   X_s[k][i] = sum_n x[s*nfft+n][i] * exp(-2 pi i k n / nfft),
 *   k = 0 .. nfft/2 - 1 (the Nyquist bin is dropped; bin 0 is DC),
 *   forward sign, no normalisation, rectangular window, no overlap.
 *
 * Twiddles come from a double table indexed by the exact integer (k*n) mod
 * nfft, so no phase error accumulates with n.  out is
 * [nspec][nfft/2][ninput][2] double.                                        */
int orc_dft_real(const int8_t *x, int32_t ninput, int32_t nfft, int64_t nspec,
                 double *out, int nthreads)
{
    if (!x || !out || ninput <= 0 || nfft <= 1 || (nfft & 1) || nspec < 0)
        return ORC_EINVAL;
    double *c = (double *)malloc(sizeof(double) * (size_t)nfft);
    double *s = (double *)malloc(sizeof(double) * (size_t)nfft);
    if (!c || !s) { free(c); free(s); return ORC_EINVAL; }
    const double two_pi = 6.283185307179586476925286766559;
    for (int32_t m = 0; m < nfft; ++m) {
        c[m] = cos(two_pi * (double)m / (double)nfft);
        s[m] = sin(two_pi * (double)m / (double)nfft);
    }
    const int32_t nchan = nfft / 2;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int64_t sp = 0; sp < nspec; ++sp) {
        for (int32_t k = 0; k < nchan; ++k) {
            for (int32_t i = 0; i < ninput; ++i) {
                double acc_re = 0.0, acc_im = 0.0;
                for (int32_t n = 0; n < nfft; ++n) {
                    double v = (double)x[(sp * nfft + n) * (int64_t)ninput + i];
                    int64_t m = ((int64_t)k * n) % nfft;
                    acc_re += v * c[m];
                    acc_im -= v * s[m];
                }
                int64_t o = ((sp * nchan + k) * (int64_t)ninput + i) * 2;
                out[o] = acc_re;
                out[o + 1] = acc_im;
            }
        }
    }
    free(c);
    free(s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Requantize to 8+8.  Reading: a caller-supplied per-channel scale, round half
 * to even, saturate to the symmetric range [-127, 127] (so -128 is never
 * produced).  The paper's quantize module (Sec. 2.2) fixes no rounding rule;
 * the definition taken is the exact one, q = sat(rint_even(scale * v)) on the
 * double spectrum value v and the binary32 scale widened to double.  A binary32
 * implementation can round the other way only where scale * v lies within its
 * own error of a half-integer.
 * X is [nspec][nchan][ninput][2] double, out is [nspec][nchan][ninput][2] int8. */
static int8_t requant_one(double v, float scale)
{
    double r = rint((double)scale * v); /* default rounding mode: half to even */
    if (r > 127.0) r = 127.0;
    if (r < -127.0) r = -127.0;
    if (r != r) r = 0.0; /* NaN never arises from finite input */
    return (int8_t)r;
}

int orc_requantize(const double *X, const float *scale, int64_t nspec, int32_t nchan,
                   int32_t ninput, int8_t *out)
{
    if (!X || !scale || !out || nspec < 0 || nchan <= 0 || ninput <= 0) return ORC_EINVAL;
    for (int64_t sp = 0; sp < nspec; ++sp)
        for (int32_t k = 0; k < nchan; ++k)
            for (int32_t i = 0; i < ninput; ++i) {
                int64_t o = ((sp * nchan + k) * (int64_t)ninput + i) * 2;
                out[o] = requant_one(X[o], scale[k]);
                out[o + 1] = requant_one(X[o + 1], scale[k]);
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase-and-sum beamformer with square-law detection and integration.
 *
 *   y[b][f][t]  = sum_i w[f][b][i] * x[t][f][i]          (no conjugation)
 *   P[b][f][u]  = sum_{t = u*navg}^{u*navg+navg-1} |y[b][f][t]|^2
 *
 * xre/xim are [ntime][nchan][ninput], wre/wim [nchan][nbeam][ninput] (decoded
 * FP16 values, exact in double); out is [nbeam][nchan][ntime/navg] double.   */
int orc_beamform_detect(const double *xre, const double *xim, const double *wre,
                        const double *wim, int64_t ntime, int32_t nchan, int32_t ninput,
                        int32_t nbeam, int32_t navg, double *out, int nthreads)
{
    if (!xre || !xim || !wre || !wim || !out) return ORC_EINVAL;
    if (ntime < 0 || nchan <= 0 || ninput <= 0 || nbeam <= 0 || navg <= 0) return ORC_EINVAL;
    if (ntime % navg) return ORC_EINVAL;
    const int64_t nout = ntime / navg;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int32_t f = 0; f < nchan; ++f) {
        for (int32_t b = 0; b < nbeam; ++b) {
            for (int64_t u = 0; u < nout; ++u) {
                double power = 0.0;
                for (int64_t t = u * navg; t < (u + 1) * navg; ++t) {
                    double yr = 0.0, yi = 0.0;
                    for (int32_t i = 0; i < ninput; ++i) {
                        int64_t wx = ((int64_t)f * nbeam + b) * ninput + i;
                        int64_t xx = (t * nchan + f) * (int64_t)ninput + i;
                        yr += wre[wx] * xre[xx] - wim[wx] * xim[xx];
                        yi += wre[wx] * xim[xx] + wim[wx] * xre[xx];
                    }
                    power += yr * yr + yi * yi;
                }
                out[((int64_t)b * nchan + f) * nout + u] = power;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase-and-sum beamformer on 4+4-bit voltages with 8-bit integer weights
 * (paper Sec. 6, DRX pipeline: the GPU beamformer takes the 4+4 complex
 * samples directly, without unpacking them first), square-law detection and
 * integration (Sec. 4.1 detect and accumulate blocks).
 *
 *   y[b][f][t] = sum_i w[f][b][i] * x[t][f][i]         (complex, no conjugation,
 *                                                       exact in int64)
 *   S[b][f][u] = sum_{t = u*navg}^{u*navg+navg-1} |y[b][f][t]|^2   (int64)
 *   P[b][f][u] = fl32( fl64( fl64(scale_b * scale_b) * fl64(S) ) )
 *
 * Reading: the weights are integers w_int with a per-beam binary32 scale
 * scale_b (physical weight scale_b * w_int), so the physical power is
 * scale_b^2 * S.  The binary32 result is defined by the rounding steps above:
 * scale_b^2 is exact in double; S is converted to double (exact below 2^53),
 * the product rounded to double, then to binary32.
 *
 * x: ci4 bytes [ntime][nchan][ninput]; w: int8 [nchan][nbeam][ninput][2]
 * (re, im); scale: float[nbeam]; power: float [nbeam][nchan][ntime/navg];
 * y (optional, may be NULL): int64 [nbeam][nchan][ntime][2].               */
int orc_beamform_ci4(const uint8_t *x, const int8_t *w, const float *scale, int64_t ntime,
                     int32_t nchan, int32_t ninput, int32_t nbeam, int32_t navg,
                     float *power, int64_t *y, int nthreads)
{
    if (!x || !w || !scale || !power) return ORC_EINVAL;
    if (ntime < 0 || nchan <= 0 || ninput <= 0 || nbeam <= 0 || navg <= 0) return ORC_EINVAL;
    if (ntime % navg) return ORC_EINVAL;
    const int64_t nout = ntime / navg;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int32_t f = 0; f < nchan; ++f) {
        for (int32_t b = 0; b < nbeam; ++b) {
            for (int64_t u = 0; u < nout; ++u) {
                int64_t s = 0;
                for (int64_t t = u * navg; t < (u + 1) * navg; ++t) {
                    int64_t yr = 0, yi = 0;
                    for (int32_t i = 0; i < ninput; ++i) {
                        int64_t wx = (((int64_t)f * nbeam + b) * ninput + i) * 2;
                        int64_t wr = w[wx], wi = w[wx + 1];
                        int byte = x[(t * nchan + f) * (int64_t)ninput + i];
                        int64_t xr = nibble_value(byte >> 4), xi = nibble_value(byte);
                        yr += wr * xr - wi * xi;
                        yi += wr * xi + wi * xr;
                    }
                    if (y) {
                        int64_t o = (((int64_t)b * nchan + f) * ntime + t) * 2;
                        y[o] = yr;
                        y[o + 1] = yi;
                    }
                    s += yr * yr + yi * yi;
                }
                double sb2 = (double)scale[b] * (double)scale[b];
                power[((int64_t)b * nchan + f) * nout + u] = (float)(sb2 * (double)s);
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* T-engine: channelized spectra back to a time series (paper Sec. 6, TBN
 * pipeline and DRX T-engine): complex samples are converted to floating
 * point, reduced in bandwidth to nfft channels starting at chan0, shifted
 * along the channel axis so the centre of the kept band sits at zero
 * frequency, inverse transformed, multiplied by a complex mixer for
 * sub-channel tuning, and quantized to 8+8 or 4+4 bit complex integers.
 *
 *   X_k   = x[s][chan0 + k][i],  k = 0 .. nfft-1          (ci8 input)
 *   z[n]  = (1/nfft) sum_k X_k exp(+2 pi i (k - nfft/2) n / nfft)
 *   z'[n] = z[n] exp(+2 pi i ((mix_num * t) mod mix_den) / mix_den),
 *           t = s * nfft + n (the mixer phase runs on across frames)
 *   q     = clamp(rint_half_even(scale * z'), -L, L) per component,
 *           L = 127 (out_bits 8) or 7 (out_bits 4).
 *
 * Readings (the paper names the steps, not their conventions): the inverse
 * transform is normalised by 1/nfft (the convention of the library inverse FFT
 * the paper's TBN pipeline calls); the shift maps channel chan0 + nfft/2 to
 * zero frequency; the mixer frequency is the exact fraction mix_num/mix_den
 * cycles per output sample; quantization is symmetric (4+4 never uses -8).
 * Phases are reduced exactly in integers before cos/sin in double.
 * Output: int32 [nspec * nfft][ninput][2] codes (the caller packs them).    */
int orc_tengine(const int8_t *x, int32_t nchan, int32_t ninput, int64_t nspec, int32_t chan0,
                int32_t nfft, int64_t mix_num, int64_t mix_den, float scale, int out_bits,
                int32_t *q, double *z_out, int nthreads)
{
    if (!x || !q || nchan <= 0 || ninput <= 0 || nspec < 0 || nfft <= 0 || (nfft & 1)) return ORC_EINVAL;
    if (chan0 < 0 || chan0 + nfft > nchan || mix_den <= 0 || mix_num < 0) return ORC_EINVAL;
    if (out_bits != 8 && out_bits != 4) return ORC_EINVAL;
    const double two_pi = 6.283185307179586476925286766559;
    const double lim = out_bits == 8 ? 127.0 : 7.0;
    double *c = (double *)malloc(sizeof(double) * nfft);
    double *sn = (double *)malloc(sizeof(double) * nfft);
    if (!c || !sn) { free(c); free(sn); return ORC_EINVAL; }
    for (int32_t m = 0; m < nfft; ++m) {
        c[m] = cos(two_pi * m / nfft);
        sn[m] = sin(two_pi * m / nfft);
    }
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int64_t sp = 0; sp < nspec; ++sp) {
        for (int32_t i = 0; i < ninput; ++i) {
            for (int32_t n = 0; n < nfft; ++n) {
                double zr = 0.0, zi = 0.0;
                for (int32_t k = 0; k < nfft; ++k) {
                    int64_t ix = ((sp * nchan + chan0 + k) * (int64_t)ninput + i) * 2;
                    double xr = x[ix], xi = x[ix + 1];
                    /* phase index (k - nfft/2) n mod nfft, non-negative */
                    int64_t m = (((int64_t)(k - nfft / 2) * n) % nfft + nfft) % nfft;
                    zr += xr * c[m] - xi * sn[m];
                    zi += xr * sn[m] + xi * c[m];
                }
                zr /= nfft;
                zi /= nfft;
                int64_t t = sp * nfft + n;
                int64_t pm = (int64_t)(((unsigned __int128)mix_num * (unsigned __int128)t) % (unsigned __int128)mix_den);
                double ph = two_pi * (double)pm / (double)mix_den;
                double cr = cos(ph), ci = sin(ph);
                double ur = zr * cr - zi * ci, ui = zr * ci + zi * cr;
                int64_t o = (t * ninput + i) * 2;
                if (z_out) { z_out[o] = ur; z_out[o + 1] = ui; }
                double a = rint((double)scale * ur), b = rint((double)scale * ui);
                if (a > lim) a = lim;
                if (a < -lim) a = -lim;
                if (b > lim) b = lim;
                if (b < -lim) b = -lim;
                q[o] = (int32_t)a;
                q[o + 1] = (int32_t)b;
            }
        }
    }
    free(c);
    free(sn);
    return ORC_OK;
}
