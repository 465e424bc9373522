// Binary16 X-engine for gfx950: cf16 voltages -> binary32 visibilities.
//
// Per channel f the kernel forms V = sum_t x_t x_t^H, lower triangle (the FX
// correlator's cross-multiply, Sec. 2.2 linear-algebra module and Sec. 7),
// with binary16 products and binary32 accumulation on MFMA.
//
// Formulation.  Each complex input i is two real rows of a matrix Y
// (row 2i = Re x_i, row 2i+1 = Im x_i, columns = time), and the kernel forms
// the real product C = Y Y^T on the lower block triangle.  Per complex pair
//   Re V_ij = C[2i][2j] + C[2i+1][2j+1],   Im V_ij = C[2i+1][2j] - C[2i][2j+1],
// which is exactly 4 real MACs per complex MAC: no redundant work.  The cf16
// row [t][f][i] in memory, (re, im) interleaved, already is row t of Y^T, so
// the LDS stage needs no de-interleave: ds_read_b64_tr_b16 turns 4 time rows
// x 16 real rows into per-real-row K(time)-contiguous MFMA fragments.
//
// Tiles.  Work decomposition, LDS ring and persistent loop are those of the
// integer kernels (xe_common.h); a stage holds 16 time rows of 256 complex
// inputs = one K step of v_mfma_f32_32x32x16_f16.  A wave's tile is 64 complex
// rows x 32 complex columns = 128 x 64 real: 4 x 2 sub-blocks of 32 x 32
// binary32 accumulators (128 registers), 8 MFMAs per stage.
//
// Epilogue.  In the 32x32 MFMA output layout (lane l, register v hold real row
// 8*(v/4) + 4*(l/32) + v%4, real column l%32) the four real products of a
// complex pair sit in two adjacent registers of two adjacent lanes.  Each
// lane swaps the four registers of a quad with its neighbour (DPP) and forms
// both rows' results from its own and the neighbour's values: even lanes keep
// the even complex row of the quad, odd lanes the odd one, so every lane
// stores.
//
// Accuracy.  binary16 x binary16 products are exact in binary32; the error is
// the binary32 summation over T samples: |dV_ij| <= ~T u sum_t |x_i||x_j|
// <= ~T u sqrt(V_ii V_jj) (u = 2^-24, Cauchy-Schwarz).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "bfx_internal.h"
#include "xe_common.h"

namespace bfx {
namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

using F16Fmt = RowFmt<4>;  // 1 KiB rows, 16 rows per stage
static_assert(F16Fmt::kT == 16, "one 16-sample MFMA step per stage");

struct F16Acc {
    v16f c[4][2];  // [row sub-block of 16 complex][column sub-block of 16 complex]
};

// Per-lane LDS byte offset (within a stage) of the first transposing read of
// the fragment of complex inputs ioff..ioff+15 (real rows 2*ioff..2*ioff+31).
// tr_b16: lanes 4r..4r+3 of a 16-lane group name the four 8-byte quarters of
// time row r (r = 0..3); lane j receives 16-bit element j of rows 0..3.  Group
// G covers real rows +16*(G&1) and times +8*(G>>1) (the MFMA K half).  The
// swizzle only depends on t % 4, which is the same for the second read (4 rows
// further), so that one is at a fixed distance.
__device__ inline int frag_base16(int ioff, int lane) {
    using F = F16Fmt;
    const int G = (lane >> 4) & 3;
    const int k = lane & 15;
    const int t = 8 * (G >> 1) + (k >> 2);
    const int byte = 4 * ioff + 32 * (G & 1) + 8 * (k & 3);
    return t * F::kRow + 16 * ((byte >> 4) ^ F::swz(t)) + (byte & 15);
}

__device__ __forceinline__ v8h read_frag16(const uint8_t *p) {
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)p);
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(p + 4 * F16Fmt::kRow));
    const v4h l = __builtin_bit_cast(v4h, lo);
    const v4h h = __builtin_bit_cast(v4h, hi);
    return v8h{l[0], l[1], l[2], l[3], h[0], h[1], h[2], h[3]};
}

// Epilogue modes (the loop's `overwrite` argument).
constexpr int kAddF32 = 0, kStoreF32 = 1, kAddF64 = 2;

struct F16Consumer {
    static constexpr int kWaves = 8;
    static constexpr int kThreads = 64 * kWaves;
    typedef F16Acc Acc;
    struct Raw {
        v8h a[4], b[2];  // row and column fragments of one stage
    };
    static constexpr int kLdsReads = 12;  // LDS instructions of one stage's reads (6 fragments x 2)
    struct Bases {
        int fb[6];  // 4 row fragments, 2 column fragments
    };
    __device__ static __forceinline__ WaveJob job(const Task &tk, int wave, int ninput) {
        return make_job_half(tk, wave, ninput);
    }
    __device__ static __forceinline__ void zero(Acc &acc) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc.c[r][c] = v16f{0.0f};
    }
    __device__ static __forceinline__ void bind(const WaveJob &job, int lane, Bases &b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) b.fb[r] = frag_base16(job.rrow + 16 * r, lane);
#pragma unroll
        for (int c = 0; c < 2; ++c) b.fb[4 + c] = frag_base16(job.crow + 16 * c, lane);
    }
    __device__ static __forceinline__ void read(const uint8_t *st, const Bases &b, Raw &raw) {
#pragma unroll
        for (int r = 0; r < 4; ++r) raw.a[r] = read_frag16(st + b.fb[r]);
#pragma unroll
        for (int c = 0; c < 2; ++c) raw.b[c] = read_frag16(st + b.fb[4 + c]);
    }
    // The MFMA operands are the raw reads themselves: nothing is formed ahead.
    struct Pre {};
    __device__ static __forceinline__ void prep(const Raw &, Pre &) {}
    // MFMA k of the stage: column fragment k / 4, row fragment k % 4.
    __device__ static __forceinline__ void mfma_k(int k, const Raw &raw, Acc &acc) {
        const int c = k >> 2, r = k & 3;
        acc.c[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(raw.a[r], raw.b[c], acc.c[r][c], 0, 0, 0);
    }
    static constexpr int kHead = 2;
    __device__ static __forceinline__ void head(const Pre &, const Raw &raw, Acc &acc) {
#pragma unroll
        for (int k = 0; k < kHead; ++k) mfma_k(k, raw, acc);
    }
    __device__ static __forceinline__ void tail(const Pre &, const Raw &raw, const Raw &, Pre &, Acc &acc) {
#pragma unroll
        for (int k = kHead; k < 8; ++k) mfma_k(k, raw, acc);
    }

    // Swap with the neighbouring lane (DPP quad_perm [1,0,3,2]).
    __device__ static __forceinline__ float swap_lane(float x) {
        return __builtin_bit_cast(
            float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
    }

    // mode: kAddF32 adds V to the binary32 buffer, kStoreF32 stores it,
    // kAddF64 adds (double)V to a binary64 running sum (16-byte elements).
    __device__ static __forceinline__ void epilogue(const WaveJob &j, const Item &it, const Acc &acc,
                                                    int lane, int mode) {
        const int ninput = it.ninput;
        uint8_t *obase = (uint8_t *)it.out + (int64_t)j.ochan * it.out_chan_bytes;
        const int g = lane >> 5;
        const int odd = lane & 1;
        const int il = j.rblk * kBlk + 2 * g + odd;                  // row of d = 0
        const int jl = j.cblk * kBlk + 32 * j.ch + ((lane & 31) >> 1);  // column of c = 0
        const uint32_t es = mode == kAddF64 ? 16 : 8;                 // bytes per complex element
        const uint32_t base = (uint32_t)(il * (il + 1) / 2 + jl) * es;
        const uint32_t step = (uint32_t)il * es;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int R0 = j.rblk * kBlk + 16 * r;                // first complex row
                const int C0 = j.cblk * kBlk + 32 * j.ch + 16 * c;    // first complex column
                if (R0 + 15 < C0 || R0 >= ninput || C0 >= ninput) continue;  // dead sub-block
                const bool interior = R0 >= C0 + 15 && R0 + 15 < ninput;
                const v16f &v = acc.c[r][c];
                const int jj = jl + 16 * c;
                auto dst = [&](int s) {
                    const int d = 16 * r + 4 * s;
                    return obase + base + (uint32_t)(16 * c) * es + (uint32_t)d * step +
                           (uint32_t)(d * (d + 1) / 2) * es;
                };
                auto ok = [&](int s) {
                    const int i = il + 16 * r + 4 * s;
                    return interior || (i < ninput && jj <= i);
                };
                float2 res[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    // a_k: this lane's register 4s+k; b_k: the same register
                    // of the neighbouring lane.  Registers 4s, 4s+1 are the
                    // even complex row's real row, 4s+2, 4s+3 the next real
                    // row; even lanes hold real column 2j, odd lanes 2j+1.
                    //   even lane (row 2i'):   Re = a0 + b1, Im = a1 - b0;
                    //   odd lane (row 2i'+1):  Re = b2 + a3, Im = b3 - a2.
                    // Both are formed and the lane keeps its own: a select
                    // between the registers themselves would become a
                    // per-lane indexed read of the accumulator vector.
                    const float a0 = v[4 * s], a1 = v[4 * s + 1], a2 = v[4 * s + 2], a3 = v[4 * s + 3];
                    const float b0 = swap_lane(a0), b1 = swap_lane(a1), b2 = swap_lane(a2), b3 = swap_lane(a3);
                    const float ere = a0 + b1, eim = a1 - b0;
                    const float ore = b2 + a3, oim = b3 - a2;
                    res[s] = float2{odd ? ore : ere, odd ? oim : eim};
                }
                if (mode == kAddF64) {
                    // the binary32 result, converted exactly, into the running
                    // sum: all old values first, then the sums, then the stores
                    double2 old[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        old[s] = double2{0.0, 0.0};
                        if (ok(s)) old[s] = *(const double2 *)dst(s);
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        old[s] = double2{old[s].x + (double)res[s].x, old[s].y + (double)res[s].y};
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        if (ok(s)) *(double2 *)dst(s) = old[s];
                    continue;
                }
                if (mode == kAddF32) {
                    // all old values first, then the sums, then the stores
                    float2 old[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        old[s] = float2{0.0f, 0.0f};
                        if (ok(s)) old[s] = *(const float2 *)dst(s);
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s = 0; s < 4; ++s) res[s] = float2{res[s].x + old[s].x, res[s].y + old[s].y};
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    if (ok(s)) *(float2 *)dst(s) = res[s];
            }
        }
    }
};

template <int DW>
__global__ __launch_bounds__(F16Consumer::kThreads, 1) void xengine_f16_kernel(SingleArray w, int nt,
                                                                  int total_flat, int overwrite) {
    xe_loop<F16Fmt, F16Consumer, DW>(w, nt, total_flat, overwrite);
}

// The same with each stage's reads issued two stages ahead (items of at least
// two stages).
template <int DW>
__global__ __launch_bounds__(F16Consumer::kThreads, 1) void xengine_f16_ra2_kernel(SingleArray w, int nt,
                                                                      int total_flat, int overwrite) {
    xe_loop_ra2<F16Fmt, F16Consumer, DW>(w, nt, total_flat, overwrite);
}

// Kernel variants a plan chooses between (index = variant): four or eight
// DMA waves, reads one (0, 1) or two (2, 3) stages ahead.
typedef void (*F16Kernel)(SingleArray, int, int, int);
constexpr int kF16Variants = 4;
const F16Kernel kF16[kF16Variants] = {xengine_f16_kernel<4>, xengine_f16_kernel<8>, xengine_f16_ra2_kernel<4>,
                                      xengine_f16_ra2_kernel<8>};

DeviceInit g_init;

hipError_t set_attributes() {
    for (int v = 0; v < kF16Variants; ++v) {
        const hipError_t e = hipFuncSetAttribute((const void *)kF16[v], hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 kLdsBytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_xengine_f16(const void *in, int64_t nt, int32_t nchan, int32_t ninput, void *out,
                              F16Out mode, int variant, hipStream_t s) {
    if (variant < 0 || variant >= kF16Variants) return hipErrorInvalidValue;
    const int m = mode == F16Out::kAdd ? kAddF32 : mode == F16Out::kStore ? kStoreF32 : kAddF64;
    int num_cus = 0;
    const hipError_t e = g_init.ensure(set_attributes, &num_cus);
    if (e != hipSuccess) return e;
    SingleArray w;
    w.in = (const uint8_t *)in;
    w.out = out;
    w.bps = 4;
    w.t_stride = (int64_t)nchan * ninput * 4;
    w.out_chan_bytes = (int64_t)ninput * (ninput + 1) / 2 * (m == kAddF64 ? 16 : 8);
    w.nchan = nchan;
    w.ninput = ninput;
    w.nb = (ninput + kBlk - 1) / kBlk;
    w.nitems = tri_items(w.nb);
    w.npk = w.nb == 1 ? 4 : 1;
    w.ngroups = (nchan + w.npk - 1) / w.npk;
    const int64_t total_flat = ((int64_t)w.ngroups + 7) / 8 * 8 * w.nitems;
    const int64_t grid = persistent_grid(num_cus, total_flat);
    // reads two stages ahead need items of two stages at least
    if (variant >= 2 && (nt + F16Fmt::kT - 1) / F16Fmt::kT < 2) variant -= 2;
    hipLaunchKernelGGL(kF16[variant], dim3((unsigned)grid), dim3(F16Consumer::kThreads), kLdsBytes, s, w,
                       (int)nt, (int)total_flat, m);
    return hipGetLastError();
}

}  // namespace bfx
