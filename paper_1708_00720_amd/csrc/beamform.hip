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
// with K contiguous, so a B fragment of v_mfma_f32_16x16x32_f16 (8
// consecutive K of one column per lane) is 16 contiguous bytes of one row.
// A cf16 weight (re in the low half, im in the high half of a dword) becomes
// a W' element pair by flipping the sign bit of the high half (row 2b) or
// swapping halves (row 2b+1).
//
// Data path.  Voltages reach LDS with global_load_lds_dwordx4 in stages of 16
// samples x one K chunk of up to 256 inputs: each sample's slice of a row
// (up to 1 KiB, contiguous in HBM) is fetched whole by consecutive lanes, so
// every DRAM page opened is read out in one burst (loading fragments straight
// into registers reads each row in 32-byte pieces spread over the K loop).
// Three stages rotate; the DMA two stages ahead is issued behind the barrier
// that releases the current one.  The 16-byte chunks of a row are XOR-
// swizzled by the row index so the 16 rows of a B fragment read hit distinct
// banks.
//
// Tiles.  Work unit = (channel, 256 samples, 32 beams); wave w owns beams
// 8w..8w+7 (16 real MFMA rows) for all 256 samples (16 tiles of 16 samples,
// 16 x 4 FP32 accumulators per lane: the longer the unit, the fewer times a
// chunk's weights and its first stages are waited for).  Its W' fragments for the whole K chunk
// (16 K steps x 8 binary16 per lane) are expanded from the cf16 weights into
// registers once per chunk; the K loop then runs on LDS reads and MFMAs only.
// Two workgroups share a CU.
//
// Detection.  In the 16x16 output layout a lane holds rows 4g..4g+3 of one
// sample column (g = lane / 16): the (Re, Im) rows of beams 2g and 2g+1, so
// |y|^2 is lane-local; a window of navg (a power of two <= 32) consecutive
// samples is navg consecutive lanes of a 16-lane group (two adjacent tiles for
// navg = 32), summed by a ds_swizzle butterfly.  Work units are assigned so
// that all units of a channel share an XCD (its weights are read from HBM
// once).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "bfx_internal.h"

namespace bfx {
namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int kBeams = 32;      // beams per unit: 4 waves x 8 beams
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kS = 16;          // samples per stage (one MFMA column tile)
constexpr int kNT = 16;         // stages per unit and K chunk
constexpr int kTB = kS * kNT;   // samples per unit
constexpr int kKC = 256;        // complex inputs per K chunk
constexpr int kKS = kKC / 16;   // MFMA K steps (32 real K = 16 inputs) per chunk
constexpr int kStageBytes = kS * kKC * 4;  // 16 KiB
constexpr int kSlots = 3;       // LDS stages in flight
constexpr int kLdsBytes = kSlots * kStageBytes;

// Lane-xor exchange within 32-lane groups (ds_swizzle bitmask mode: and 0x1F,
// or 0, xor K).
template <int K>
__device__ inline float swz_xor(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x1F | (K << 10)));
}

// Sum over aligned groups of 2^L consecutive lanes (L <= 4).
template <int L>
__device__ inline float group_sum(float p) {
    if constexpr (L >= 1) p += swz_xor<1>(p);
    if constexpr (L >= 2) p += swz_xor<2>(p);
    if constexpr (L >= 3) p += swz_xor<4>(p);
    if constexpr (L >= 4) p += swz_xor<8>(p);
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

// 16 bytes from global memory straight into LDS at m0 + 16 * lane.
__device__ inline void dma16(const void *src, uint32_t lds_wave_base) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_wave_base)), "v"(src)
                 : "memory", "m0");
}

// Row swizzle of the 16-byte chunks (a row of cpr chunks, cpr a multiple of 8).
__device__ inline int row_swz(int r, int cpr) { return r & ((cpr & 15) ? 7 : 15); }

// Issue this wave's share of the DMA of one stage: rows t0..t0+15 (clamped:
// rows past ntime only feed windows that are never stored), inputs kc..kc+nin.
__device__ __forceinline__ void stage_dma(const uint8_t *xrow0, int64_t rstride, int t0, int ntime, int nin,
                                          uint32_t lds_stage, int wave, int lane) {
    const int cpr = nin / 4;       // 16-byte chunks per row
    const int ninstr = cpr / 4;    // 1 KiB wave instructions per stage (16 rows)
    for (int j = wave; j < ninstr; j += kWaves) {
        const int c = 64 * j + lane;
        const int r = c / cpr;
        const int p = c - r * cpr;
        const int t = min(t0 + r, ntime - 1);
        dma16(xrow0 + (int64_t)t * rstride + 16 * (p ^ row_swz(r, cpr)), lds_stage + 1024 * j);
    }
}

// Wait until at most N vector-memory operations of this wave are in flight
// (N <= 15; expcnt and lgkmcnt left at their maxima).
template <int N>
__device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(N | 0x0F70); }

// The same with a wave-uniform run-time count n in 0..4.
__device__ inline void wait_vm_n(int n) {
    switch (n) {
        case 0: wait_vm<0>(); break;
        case 1: wait_vm<1>(); break;
        case 2: wait_vm<2>(); break;
        case 3: wait_vm<3>(); break;
        default: wait_vm<4>(); break;
    }
}

template <int LOGNAVG>
__global__ __launch_bounds__(kThreads, 2) void beamform_kernel(
    const uint8_t *__restrict__ x, const uint8_t *__restrict__ w, int ninput, int nchan, int nbeam,
    int ntime, int ntb, int nbg, float *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;
    Unit u;
    if (!unit_of(blockIdx.x, ntb, nbg, nchan, u)) return;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int m = lane & 15;  // A row / B and D column of this lane
    const int g = lane >> 4;  // K quarter of the A and B fragments; D rows 4g..4g+3
    const int beam_a = u.bg * kBeams + 8 * wave + (m >> 1);   // beam of W' row m
    const uint32_t sel = (m & 1) ? 0x01000302u : 0x03020100u;  // swap halves / identity
    const uint32_t flip = (m & 1) ? 0u : 0x80000000u;           // negate Im w on Re rows

    const int64_t rstride = (int64_t)nchan * ninput * 4;
    const int tu = u.tb * kTB;
    const uint8_t *xf = x + (int64_t)u.f * ninput * 4;

    v4f acc[kNT];
#pragma unroll
    for (int st = 0; st < kNT; ++st) acc[st] = v4f{0.0f, 0.0f, 0.0f, 0.0f};

    for (int kc = 0; kc < ninput; kc += kKC) {
        const int nin = min(kKC, ninput - kc);  // multiple of 32
        const int nks = nin / 16;
        const int rowb = nin * 4;               // LDS bytes per stage row
        const int ninstr = nin / 16;            // DMA instructions per stage
        const int nmine = wave < ninstr ? (ninstr - wave + kWaves - 1) / kWaves : 0;  // this wave's
        // W' fragments of this chunk (zero past nbeam), complete before any
        // DMA of the chunk is issued
        v8h wf[kKS];
        const uint8_t *wrow = w + (((int64_t)u.f * nbeam + beam_a) * ninput + kc + 4 * g) * 4;
#pragma unroll
        for (int ks = 0; ks < kKS; ++ks) {
            v4u a = v4u{0u, 0u, 0u, 0u};
            if (ks < nks && beam_a < nbeam) a = *(const v4u *)(wrow + 64 * ks);
            v4u t;
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] = __builtin_amdgcn_perm(a[q], a[q], sel) ^ flip;
            wf[ks] = __builtin_bit_cast(v8h, t);
        }
        // every wave is done with the previous chunk's stages
        __syncthreads();
#pragma unroll
        for (int st = 0; st < kSlots - 1; ++st)
            stage_dma(xf + (int64_t)kc * 4, rstride, tu + kS * st, ntime, nin, lds_base + st * kStageBytes,
                      wave, lane);
        const int swz = row_swz(m, nin / 4);
#pragma unroll
        for (int st = 0; st < kNT; ++st) {
            // this stage has landed everywhere (the next one may still be in
            // flight), and the slot of the previous one is free
            if (st + 1 < kNT) wait_vm_n(nmine);
            else wait_vm<0>();
            __syncthreads();
            if (st + kSlots - 1 < kNT)
                stage_dma(xf + (int64_t)kc * 4, rstride, tu + kS * (st + kSlots - 1), ntime, nin,
                          lds_base + ((st + kSlots - 1) % kSlots) * kStageBytes, wave, lane);
            const uint8_t *srow = lds + (st % kSlots) * kStageBytes + m * rowb;
            if (nks == kKS) {
                // full chunk: reads in batches of eight ahead of their MFMAs
#pragma unroll
                for (int k0 = 0; k0 < kKS; k0 += 8) {
                    v8h b[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        b[k] = *(const v8h *)(srow + 16 * ((4 * (k0 + k) + g) ^ swz));
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        acc[st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wf[k0 + k], b[k], acc[st], 0, 0, 0);
                }
            } else {
                // partial chunk (nks even): K steps in pairs, none past nks
#pragma unroll
                for (int k0 = 0; k0 < kKS; k0 += 2) {
                    if (k0 < nks) {
                        const v8h b0 = *(const v8h *)(srow + 16 * ((4 * k0 + g) ^ swz));
                        const v8h b1 = *(const v8h *)(srow + 16 * ((4 * k0 + 4 + g) ^ swz));
                        acc[st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wf[k0], b0, acc[st], 0, 0, 0);
                        acc[st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wf[k0 + 1], b1, acc[st], 0, 0, 0);
                    }
                }
            }
        }
    }

    // detect: lane holds sample tu + 16*st + m of beams 8*wave + 2g (registers
    // 0, 1) and 8*wave + 2g + 1 (registers 2, 3)
    const int nwin = ntime >> LOGNAVG;
    const int bw = u.bg * kBeams + 8 * wave + 2 * g;
    // navg 16 and 32: each window of the unit is summed in all 16 lanes of a
    // group; lane m keeps window m, and the unit's windows leave as one store
    // per beam pair (16 or 8 consecutive windows of each beam) instead of one
    // per window
    float w0 = 0.0f, w1 = 0.0f;
#pragma unroll
    for (int st = 0; st < kNT; ++st) {
        if (LOGNAVG == 5 && (st & 1)) continue;
        float p0 = acc[st][0] * acc[st][0] + acc[st][1] * acc[st][1];
        float p1 = acc[st][2] * acc[st][2] + acc[st][3] * acc[st][3];
        if constexpr (LOGNAVG == 5) {
            p0 += acc[st + 1][0] * acc[st + 1][0] + acc[st + 1][1] * acc[st + 1][1];
            p1 += acc[st + 1][2] * acc[st + 1][2] + acc[st + 1][3] * acc[st + 1][3];
        }
        constexpr int L = LOGNAVG < 4 ? LOGNAVG : 4;
        p0 = group_sum<L>(p0);
        p1 = group_sum<L>(p1);
        if constexpr (LOGNAVG >= 4) {
            if (m == (st >> (LOGNAVG - 4))) {
                w0 = p0;
                w1 = p1;
            }
        } else {
            const int t = tu + kS * st + m;
            const int uwin = t >> LOGNAVG;
            if ((m & ((1 << L) - 1)) == 0 && uwin < nwin) {
                if (bw < nbeam) out[((int64_t)bw * nchan + u.f) * nwin + uwin] = p0;
                if (bw + 1 < nbeam) out[((int64_t)(bw + 1) * nchan + u.f) * nwin + uwin] = p1;
            }
        }
    }
    if constexpr (LOGNAVG >= 4) {
        static_assert(kNT == 16, "at most one window per lane of a 16-lane group");
        constexpr int kW = kNT >> (LOGNAVG - 4);  // windows per unit: 16 or 8
        const int uwin = (tu >> LOGNAVG) + m;
        if (m < kW && uwin < nwin) {
            if (bw < nbeam) out[((int64_t)bw * nchan + u.f) * nwin + uwin] = w0;
            if (bw + 1 < nbeam) out[((int64_t)(bw + 1) * nchan + u.f) * nwin + uwin] = w1;
        }
    }
}

typedef void (*BfKernel)(const uint8_t *, const uint8_t *, int, int, int, int, int, int, float *);
const BfKernel kKernels[6] = {beamform_kernel<0>, beamform_kernel<1>, beamform_kernel<2>,
                              beamform_kernel<3>, beamform_kernel<4>, beamform_kernel<5>};

DeviceInit g_init;

hipError_t set_attributes() {
    for (BfKernel k : kKernels) {
        const hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 kLdsBytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

bool beamform_supported(int32_t navg) { return navg >= 1 && navg <= 32 && (navg & (navg - 1)) == 0; }

// Workgroups of one launch: channels (padded to the XCD count) x 256-sample
// units x 32-beam groups.
int64_t beamform_units(int32_t nchan, int32_t nbeam, int64_t ntime) {
    const int64_t ntb = (ntime + kTB - 1) / kTB;
    const int64_t nbg = (nbeam + kBeams - 1) / kBeams;
    return ((int64_t)nchan + 7) / 8 * 8 * ntb * nbg;
}

hipError_t launch_beamform(const void *x, const void *w, int32_t ninput, int32_t nchan,
                           int32_t nbeam, int64_t ntime, int32_t navg, float *out, hipStream_t s) {
    const hipError_t e = g_init.ensure(set_attributes, nullptr);
    if (e != hipSuccess) return e;
    int lognavg = 0;
    while ((1 << lognavg) < navg) ++lognavg;
    const int ntb = (int)((ntime + kTB - 1) / kTB);
    const int nbg = (nbeam + kBeams - 1) / kBeams;
    const int64_t units = beamform_units(nchan, nbeam, ntime);
    if (units > kMaxWorkgroups256) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kKernels[lognavg], dim3((unsigned)units), dim3(kThreads), kLdsBytes, s,
                       (const uint8_t *)x, (const uint8_t *)w, ninput, nchan, nbeam, (int)ntime,
                       ntb, nbg, out);
    return hipGetLastError();
}

}  // namespace bfx
