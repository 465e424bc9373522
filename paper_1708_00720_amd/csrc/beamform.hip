// Phase-and-sum beamformer with square-law detection and time integration
// (the DRX beamformer of Sec. 6; detect and accumulate blocks of Sec. 4.1):
//   y[b][f][t] = sum_i w[f][b][i] x[t][f][i]     (no conjugation)
//   P[b][f][u] = sum_{t in window u} |y[b][f][t]|^2,   windows of navg samples.
//
// Formulation.  Per channel this is a complex (beams x inputs) by
// (inputs x time) product.  As a real product on MFMA,
//   [Re y; Im y] = W' X',  X'[2i+c][t] = component c of x[t][f][i],
//   W' row 2b   = (Re w_bi, -Im w_bi) over columns (2i, 2i+1),
//   W' row 2b+1 = (Im w_bi,  Re w_bi).
// A cf16 voltage row x[t][f][:] with (re, im) interleaved is column t of X'
// with K contiguous: the MFMA B fragment (8 consecutive K of one column per
// lane) is one 16-byte global load, so voltages stream from HBM into
// registers with no LDS pass.  A cf16 weight (re in the low half, im in the
// high half of a dword) becomes a W' element pair by flipping the sign bit of
// the high half (row 2b) or swapping halves (row 2b+1).
//
// Tiles.  Work unit = (channel, 256 samples, 32 beams); 4 waves of 64 samples
// (two 32-sample MFMA tiles) x 64 real rows (32 beams): v_mfma_f32_32x32x16_f16,
// FP32 accumulation, 4 x 16 accumulators per lane.  Weights of 32 beams x 512
// inputs (64 KiB) are staged in LDS per K chunk, rows XOR-swizzled in 16-byte
// chunks so the A-fragment reads (8 beams per 8-lane group) are conflict free.
// Voltage loads are double-buffered four K steps (32 inputs) ahead.
//
// Detection.  In the 32x32 output layout the (Re, Im) rows of a beam are
// adjacent registers of one lane, so |y|^2 is lane-local; a window of navg
// (a power of two <= 32) consecutive samples is navg consecutive lanes,
// summed by a ds_swizzle butterfly.  Work units are assigned so that all
// units of a channel share an XCD (its weights are read from HBM once).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "bfx_internal.h"

namespace bfx {
namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int kBeams = 32;      // beams per unit (64 real MFMA rows)
constexpr int kKChunk = 512;    // complex inputs per LDS weight chunk
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kTB = 256;        // samples per unit
constexpr int kTWave = kTB / kWaves;  // 64 samples = 2 MFMA tiles per wave
constexpr int kU = 4;           // K steps (8 inputs each) per load batch
constexpr int kLdsBytes = kBeams * kKChunk * 4;  // 64 KiB

// LDS byte offset of 16-byte chunk c (4 inputs) of beam row b.
__device__ inline uint32_t w_off(int b, int c) { return (uint32_t)(b * (kKChunk * 4) + ((c ^ (b & 7)) << 4)); }

// Lane-xor exchange within 32-lane groups (ds_swizzle bitmask mode: and 0x1F,
// or 0, xor K).
template <int K>
__device__ inline float swz_xor(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x1F | (K << 10)));
}

// Sum over aligned groups of 2^L consecutive lanes (L <= 5).
template <int L>
__device__ inline float group_sum(float p) {
    if constexpr (L >= 1) p += swz_xor<1>(p);
    if constexpr (L >= 2) p += swz_xor<2>(p);
    if constexpr (L >= 3) p += swz_xor<4>(p);
    if constexpr (L >= 4) p += swz_xor<8>(p);
    if constexpr (L >= 5) p += swz_xor<16>(p);
    return p;
}

struct Unit {
    int f, tb, bg;
};

__device__ inline bool unit_of(int B, int ntb, int nbg, int nchan, Unit &u) {
    const int s = B >> 3;
    const int per = ntb * nbg;
    const int cl = s / per;
    const int r = s - cl * per;
    u.bg = r / ntb;
    u.tb = r - u.bg * ntb;
    u.f = cl * 8 + (B & 7);
    return u.f < nchan;
}

// Load the B fragments (two 32-sample tiles) of kU K steps starting at input
// `i0` (relative to the channel row) into xb.
__device__ __forceinline__ void load_x(v4u (&xb)[kU][2], const uint8_t *row0, const uint8_t *row1,
                                       int i0) {
#pragma unroll
    for (int s = 0; s < kU; ++s) {
        xb[s][0] = *(const v4u *)(row0 + (int64_t)(i0 + 8 * s) * 4);
        xb[s][1] = *(const v4u *)(row1 + (int64_t)(i0 + 8 * s) * 4);
    }
}

// kU K steps of the wave's 64 x 64 tile.  The W' fragment of row m comes
// from the raw cf16 weights of beam m/2: row parity 0 flips the sign of the
// imaginary halves, parity 1 swaps the halves (one v_perm + one xor per dword
// with per-lane constants `sel`, `flip`).
__device__ __forceinline__ void mma_batch(const v4u (&xb)[kU][2], const uint8_t *lds, int kstep0,
                                          int brow0, int brow1, int h, uint32_t sel,
                                          uint32_t flip, v16f (&acc)[2][2]) {
#pragma unroll
    for (int s = 0; s < kU; ++s) {
        const int c = 2 * (kstep0 + s) + h;  // 16-byte chunk (4 inputs) of this lane
        v4u a[2];
        a[0] = *(const v4u *)(lds + w_off(brow0, c));
        a[1] = *(const v4u *)(lds + w_off(brow1, c));
        v8h af[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            v4u t;
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] = __builtin_amdgcn_perm(a[r][q], a[r][q], sel) ^ flip;
            af[r] = __builtin_bit_cast(v8h, t);
        }
        const v8h b0 = __builtin_bit_cast(v8h, xb[s][0]);
        const v8h b1 = __builtin_bit_cast(v8h, xb[s][1]);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[0], b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[0], b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[1], b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[1], b1, acc[1][1], 0, 0, 0);
    }
}

template <int LOGNAVG>
__global__ __launch_bounds__(kThreads, 2) void beamform_kernel(
    const uint8_t *__restrict__ x, const uint8_t *__restrict__ w, int ninput, int nchan, int nbeam,
    int ntime, int ntb, int nbg, float *__restrict__ out) {
    constexpr int kNavg = 1 << LOGNAVG;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    Unit u;
    if (!unit_of(blockIdx.x, ntb, nbg, nchan, u)) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int h = lane >> 5;      // K half of the MFMA fragment
    const int m = lane & 31;
    const int brow0 = m >> 1;     // beam (within the unit) of A row m, row block 0
    const int brow1 = 16 + (m >> 1);
    const uint32_t sel = (m & 1) ? 0x01000302u : 0x03020100u;  // swap halves / identity
    const uint32_t flip = (m & 1) ? 0u : 0x80000000u;           // negate Im w on Re rows

    // this lane's two sample rows (clamped: rows past ntime only feed windows
    // that are never stored)
    const int tw = u.tb * kTB + wave * kTWave;
    const int t0 = min(tw + m, ntime - 1);
    const int t1 = min(tw + 32 + m, ntime - 1);
    const int64_t rstride = (int64_t)nchan * ninput * 4;
    const uint8_t *xr0 = x + (int64_t)t0 * rstride + (int64_t)u.f * ninput * 4 + 16 * h;
    const uint8_t *xr1 = x + (int64_t)t1 * rstride + (int64_t)u.f * ninput * 4 + 16 * h;

    v16f acc[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = v16f{0.0f};

    const int beam0 = u.bg * kBeams;
    for (int kc = 0; kc < ninput; kc += kKChunk) {
        const int nin = min(kKChunk, ninput - kc);  // multiple of 32
        __syncthreads();  // the previous chunk's weights are consumed
        // stage the weights of 32 beams x nin inputs (zero past nbeam)
        for (int e = tid; e < kBeams * (kKChunk / 4); e += kThreads) {
            const int b = e / (kKChunk / 4);
            const int c = e - b * (kKChunk / 4);
            v4u v = v4u{0u, 0u, 0u, 0u};
            if (beam0 + b < nbeam && 4 * c < nin)
                v = *(const v4u *)(w + (((int64_t)u.f * nbeam + beam0 + b) * ninput + kc + 4 * c) * 4);
            *(v4u *)(lds + w_off(b, c)) = v;
        }
        __syncthreads();

        // one batch of kU K steps per iteration; the next batch's voltages
        // are in flight while this one is multiplied
        const int nbatch = nin / (8 * kU);  // nin % 32 == 0
        v4u xa[kU][2], xb[kU][2];
        load_x(xa, xr0, xr1, kc);
        for (int bt = 0; bt < nbatch; ++bt) {
            if (bt + 1 < nbatch) load_x(xb, xr0, xr1, kc + (bt + 1) * 8 * kU);
            mma_batch(xa, lds, bt * kU, brow0, brow1, h, sel, flip, acc);
#pragma unroll
            for (int s2 = 0; s2 < kU; ++s2) {
                xa[s2][0] = xb[s2][0];
                xa[s2][1] = xb[s2][1];
            }
        }
    }

    // detect: lane holds sample tw + 32*tt + m of beams
    //   beam0 + 16*r + 4*(q/2) + 2*h + (q%2), from registers v = 2q, 2q+1
    const int nwin = ntime >> LOGNAVG;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int t = tw + 32 * tt + m;
            const int uwin = t >> LOGNAVG;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float a = acc[r][tt][2 * q], b = acc[r][tt][2 * q + 1];
                const float p = group_sum<LOGNAVG>(a * a + b * b);
                const int beam = beam0 + 16 * r + 4 * (q >> 1) + 2 * h + (q & 1);
                if ((m & (kNavg - 1)) == 0 && beam < nbeam && uwin < nwin)
                    out[((int64_t)beam * nchan + u.f) * nwin + uwin] = p;
            }
        }
    }
}

typedef void (*BfKernel)(const uint8_t *, const uint8_t *, int, int, int, int, int, int, float *);
const BfKernel kKernels[6] = {beamform_kernel<0>, beamform_kernel<1>, beamform_kernel<2>,
                              beamform_kernel<3>, beamform_kernel<4>, beamform_kernel<5>};

std::once_flag g_init_once;
hipError_t g_init_err = hipSuccess;

void init_once() {
    for (BfKernel k : kKernels) {
        g_init_err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (g_init_err != hipSuccess) return;
    }
}

}  // namespace

bool beamform_supported(int32_t navg) { return navg >= 1 && navg <= 32 && (navg & (navg - 1)) == 0; }

hipError_t launch_beamform(const void *x, const void *w, int32_t ninput, int32_t nchan,
                           int32_t nbeam, int64_t ntime, int32_t navg, float *out, hipStream_t s) {
    std::call_once(g_init_once, init_once);
    if (g_init_err != hipSuccess) return g_init_err;
    int lognavg = 0;
    while ((1 << lognavg) < navg) ++lognavg;
    const int ntb = (int)((ntime + kTB - 1) / kTB);
    const int nbg = (nbeam + kBeams - 1) / kBeams;
    const int64_t units = ((int64_t)nchan + 7) / 8 * 8 * ntb * nbg;
    hipLaunchKernelGGL(kKernels[lognavg], dim3((unsigned)units), dim3(kThreads), kLdsBytes, s,
                       (const uint8_t *)x, (const uint8_t *)w, ninput, nchan, nbeam, (int)ntime,
                       ntb, nbg, out);
    return hipGetLastError();
}

}  // namespace bfx
