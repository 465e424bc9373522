// Integer phase-and-sum beamformer on 4+4-bit voltages, with square-law
// detection and time integration.  The DRX pipeline of Sec. 6 beamforms the
// 4+4 complex samples directly, without an unpacking pass; the detect and
// accumulate blocks are those of Sec. 4.1.
//
//   y[b][f][t] = sum_i w[f][b][i] x[t][f][i]          (complex, no conjugation)
//   S[b][f][u] = sum_{t in window u} |y[b][f][t]|^2   (exact integers)
//   P[b][f][u] = fl32(fl64(fl64(scale_b)^2) * fl64(S))
//
// Weights are int8 pairs (re, im) with a per-beam binary32 scale, so y and S
// are exact integers and the only rounding is in the final conversion, taken
// in the steps above: the result is the same bits whatever the launch shape.
//
// Formulation.  Per channel a (beams x inputs) by (inputs x time) complex
// product, as four real products on v_mfma_i32_16x16x64_i8 with int32
// accumulation and no negated operand (so the whole int8 weight range is
// exact):
//   RR = W_re X_re,  II = W_im X_im,  IM = W_re X_im + W_im X_re,
//   Re y = RR - II,  Im y = IM.
// A voltage row x[t][f][:] is one B column with K = inputs contiguous: lane
// (column n, K group q) takes 16 consecutive bytes of one row.  The ci4 byte
// is split in registers into 16*re (the high nibble kept in place) and 16*im
// (the low nibble shifted up), as int8 bytes; the products carry a factor 16
// that the epilogue shifts out exactly (RR, II, IM are multiples of 16).
//
// Data path.  Work unit = (channel, 256 samples, 32 beams); four waves, wave
// w owns samples 64w .. 64w+63 of the unit (four tiles of 16) for all 32
// beams (two M tiles).  A stage is 16 samples of every wave (64 time rows) x
// one K chunk of up to 256 inputs, 256 bytes per LDS row; it reaches LDS with
// global_load_lds_dwordx4 (each 1 KiB wave instruction is 4 whole rows).  The
// 16-byte chunks of a row are XOR-swizzled by the row index, so the 16 rows
// of one fragment read hit distinct banks.  Three stages rotate; the stage two
// ahead is issued behind the barrier that releases the current one, across
// K-chunk boundaries.  The weights of a K chunk (two M tiles x (re, im) x 4
// K steps) are loaded into registers when the chunk starts.
//
// Detection.  In the 16x16 output layout a lane holds rows 4g..4g+3 (beams)
// of one sample column, so |y|^2 is lane-local; a window of navg <= 16
// samples is navg consecutive lanes of a 16-lane group, summed in int64 by a
// ds_swizzle butterfly; navg = 32 and 64 also add the wave's adjacent tiles.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfx_internal.h"

namespace bfx {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kBeams = 32;             // beams per unit: two M tiles of 16
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kTiles = 4;              // 16-sample tiles per wave and unit
constexpr int kTB = 16 * kTiles * kWaves;  // samples per unit (256)
constexpr int kRows = 16 * kWaves;     // time rows per stage
constexpr int kKC = 256;               // inputs per K chunk (one LDS row)
constexpr int kKS = kKC / 64;          // MFMA K steps per chunk
constexpr int kStageBytes = kRows * kKC;  // 16 KiB
constexpr int kSlots = 3;
constexpr int kLdsBytes = kSlots * kStageBytes;
constexpr int kDmaPerWave = kStageBytes / 1024 / kWaves;  // 4

struct Unit {
    int f, tb, bg;
};

// Flat unit id B -> (channel, 256-sample block, beam group); units of one
// channel sit at B % 8 == f % 8 and so share an XCD and its L2 (the channel's
// weights are fetched from HBM once).
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

__device__ inline void dma16(const void *src, uint32_t lds_wave_base) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_wave_base)), "v"(src)
                 : "memory", "m0");
}

// Wait until at most N vector-memory operations of this wave are in flight
// (gfx9 encoding: vmcnt in bits 3:0 and 15:14; expcnt and lgkmcnt at their
// maxima).
template <int N>
__device__ inline void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

// Wait until this wave's LDS reads have returned (lgkmcnt = 0).
__device__ inline void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Workgroup barrier without a memory fence: the DMA into LDS is ordered by
// the explicit vmcnt waits, and every LDS read of a stage has returned (its
// MFMAs consumed it) before the wave reaches the next barrier.
__device__ inline void block_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Lane exchange by xor within 32-lane groups (ds_swizzle bitmask mode).
template <int K>
__device__ inline int swz_xor(int v) { return __builtin_amdgcn_ds_swizzle(v, 0x1F | (K << 10)); }

template <int K>
__device__ inline int64_t swz_xor64(int64_t v) {
    const int lo = swz_xor<K>((int)(uint32_t)v);
    const int hi = swz_xor<K>((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int K>
__device__ inline double swz_xor_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = swz_xor<K>((int)(uint32_t)b);
    const int hi = swz_xor<K>((int)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over aligned groups of 2^L consecutive lanes (L <= 4), in int64.
template <int L>
__device__ inline int64_t group_sum64(int64_t p) {
    if constexpr (L >= 1) p += swz_xor64<1>(p);
    if constexpr (L >= 2) p += swz_xor64<2>(p);
    if constexpr (L >= 3) p += swz_xor64<4>(p);
    if constexpr (L >= 4) p += swz_xor64<8>(p);
    return p;
}

// This wave's share of the DMA of stage i (K chunk i / kTiles, tile i %
// kTiles).  LDS row R = 16 v + r holds time tu + 64 v + 16 s + r of wave v
// (clamped to the last sample: rows past ntime feed windows never stored),
// bytes kc .. kc + 255 of the channel's row, its 16-byte chunk c at slot
// c ^ (R & 15).  Slots beyond the chunk's inputs fetch chunk 0 of the row
// (never read).
__device__ __forceinline__ void stage_dma(const uint8_t *xf, int64_t rstride, int tu, int ntime, int ninput,
                                          int i, uint32_t lds_stage, int wave, int lane) {
    const int kc = (i / kTiles) * kKC;
    const int s = i % kTiles;
    const int cpr = min(kKC, ninput - kc) / 16;
#pragma unroll
    for (int j = 0; j < kDmaPerWave; ++j) {
        const int ins = wave * kDmaPerWave + j;  // 1 KiB = LDS rows 4 ins .. 4 ins + 3
        const int R = 4 * ins + (lane >> 4);
        const int c = (lane & 15) ^ (R & 15);
        const int t = min(tu + 64 * (R >> 4) + 16 * s + (R & 15), ntime - 1);
        const int cc = c < cpr ? c : 0;
        dma16(xf + (int64_t)t * rstride + kc + 16 * cc, lds_stage + 1024 * ins);
    }
}

// Lane exchange with the lane 32 away (v_permlane32_swap).
__device__ inline int xor32(int v, int lane) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return lane < 32 ? r[1] : r[0];
}

__device__ inline double xor32_f64(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = xor32((int)(uint32_t)b, lane);
    const int hi = xor32((int)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// ci4 bytes 16 re + (im & 15) -> R = 16 re (the high nibble in place) and
// X' = 16 re + (im + 8) (bit 3 flipped: the low nibble becomes im + 8 in
// 0..15), both exact int8.  Against weights w, X' gives 16 sum(re w) +
// sum(im w) + 8 sum(w): the last term is a per-beam constant.
__device__ __forceinline__ void split_ci4_offset(const v4i raw, v4i &r, v4i &xo) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r[k] = (int)((uint32_t)raw[k] & 0xF0F0F0F0u);
        xo[k] = (int)((uint32_t)raw[k] ^ 0x08080808u);
    }
}

__device__ __forceinline__ void split_ci4(const v4i raw, v4i &re, v4i &im) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        re[k] = (int)((uint32_t)raw[k] & 0xF0F0F0F0u);
        im[k] = (int)(((uint32_t)raw[k] << 4) & 0xF0F0F0F0u);
    }
}

template <int LOGNAVG>
__global__ __launch_bounds__(kThreads, 2) void beamform_ci4_kernel(
    const uint8_t *__restrict__ x, const int8_t *__restrict__ w, const float *__restrict__ scale,
    int ninput, int nchan, int nbeam, int ntime, int ntb, int nbg, float *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;
    Unit u;
    if (!unit_of(blockIdx.x, ntb, nbg, nchan, u)) return;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int m = lane & 15;  // A row (beam within an M tile) / B column (sample)
    const int q = lane >> 4;  // K group of 16 inputs; output rows 4q..4q+3

    const int64_t rstride = (int64_t)nchan * ninput;
    const int tu = u.tb * kTB;
    const uint8_t *xf = x + (int64_t)u.f * ninput;
    const int nchunk = (ninput + kKC - 1) / kKC;
    const int nst = nchunk * kTiles;

    v4i rr[kTiles][2], ii[kTiles][2], im[kTiles][2];
#pragma unroll
    for (int s = 0; s < kTiles; ++s)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) rr[s][mt] = ii[s][mt] = im[s][mt] = v4i{0, 0, 0, 0};

    // LDS row of this lane's B fragments, and its swizzle
    const int R = 16 * wave + m;
    const int swz = R & 15;

#pragma unroll
    for (int i = 0; i < kSlots - 1; ++i)
        if (i < nst) stage_dma(xf, rstride, tu, ntime, ninput, i, lds_base + i * kStageBytes, wave, lane);

    v4i wre[kKS][2], wim[kKS][2];
    for (int ch = 0; ch < nchunk; ++ch) {
        const int kc = ch * kKC;
        const int nks = min(kKC, ninput - kc) / 64;
        // weights of this K chunk: beam bg*32 + 16 mt + m, inputs
        // kc + 64 ks + 16 q .. +15, de-interleaved into re and im bytes
#pragma unroll
        for (int ks = 0; ks < kKS; ++ks)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const int beam = u.bg * kBeams + 16 * mt + m;
                v4i a = v4i{0, 0, 0, 0}, b = v4i{0, 0, 0, 0};
                if (ks < nks && beam < nbeam) {
                    const int8_t *p = w + (((int64_t)u.f * nbeam + beam) * ninput + kc + 64 * ks + 16 * q) * 2;
                    a = *(const v4i *)p;
                    b = *(const v4i *)(p + 16);
                }
                wre[ks][mt] = v4i{(int)__builtin_amdgcn_perm(a[1], a[0], 0x06040200u),
                                  (int)__builtin_amdgcn_perm(a[3], a[2], 0x06040200u),
                                  (int)__builtin_amdgcn_perm(b[1], b[0], 0x06040200u),
                                  (int)__builtin_amdgcn_perm(b[3], b[2], 0x06040200u)};
                wim[ks][mt] = v4i{(int)__builtin_amdgcn_perm(a[1], a[0], 0x07050301u),
                                  (int)__builtin_amdgcn_perm(a[3], a[2], 0x07050301u),
                                  (int)__builtin_amdgcn_perm(b[1], b[0], 0x07050301u),
                                  (int)__builtin_amdgcn_perm(b[3], b[2], 0x07050301u)};
            }
#pragma unroll
        for (int s = 0; s < kTiles; ++s) {
            const int i = ch * kTiles + s;
            // stage i has landed everywhere; the slot of stage i - 1 is free
            if (i + 1 < nst) wait_vm<kDmaPerWave>();
            else wait_vm<0>();
            block_barrier();
            if (i + kSlots - 1 < nst)
                stage_dma(xf, rstride, tu, ntime, ninput, i + kSlots - 1,
                          lds_base + ((i + kSlots - 1) % kSlots) * kStageBytes, wave, lane);
            const uint8_t *srow = lds + (i % kSlots) * kStageBytes + R * kKC;
            v4i raw[kKS];
#pragma unroll
            for (int ks = 0; ks < kKS; ++ks)
                if (ks < nks) raw[ks] = *(const v4i *)(srow + 16 * ((4 * ks + q) ^ swz));
#pragma unroll
            for (int ks = 0; ks < kKS; ++ks) {
                if (ks < nks) {
                    v4i xr, xi;
                    split_ci4(raw[ks], xr, xi);
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        rr[s][mt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wre[ks][mt], xr, rr[s][mt], 0, 0, 0);
                        ii[s][mt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wim[ks][mt], xi, ii[s][mt], 0, 0, 0);
                        im[s][mt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wre[ks][mt], xi, im[s][mt], 0, 0, 0);
                        im[s][mt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wim[ks][mt], xr, im[s][mt], 0, 0, 0);
                    }
                }
            }
        }
    }

    // detect and integrate: lane holds sample tu + 64 wave + 16 s + m of beams
    // bg*32 + 16 mt + 4q + v
    constexpr int L = LOGNAVG < 4 ? LOGNAVG : 4;
    constexpr int kTilesPerWin = LOGNAVG > 4 ? 1 << (LOGNAVG - 4) : 1;
    const int nwin = ntime >> LOGNAVG;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        // navg >= 16: window w of beam 16 mt + 4q + v is summed in all 16
        // lanes of group q; lane m = kW v + w keeps it (kW = 4, 2, 1 windows per
        // beam), so the group's windows leave as one store with 4 kW lanes
        // active (kW consecutive windows of each of its four beams) instead of
        // one store per window with one lane in 16
        constexpr int kW = kTiles / kTilesPerWin;
        float keep = 0.0f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int beam = u.bg * kBeams + 16 * mt + 4 * q + v;
            const double sb = (double)(beam < nbeam ? scale[beam] : 0.0f);
            const double sb2 = sb * sb;
#pragma unroll
            for (int s0 = 0; s0 < kTiles; s0 += kTilesPerWin) {
                int64_t acc = 0;
#pragma unroll
                for (int s = s0; s < s0 + kTilesPerWin; ++s) {
                    const int yr = (rr[s][mt][v] - ii[s][mt][v]) >> 4;
                    const int yi = im[s][mt][v] >> 4;
                    acc += (int64_t)yr * yr + (int64_t)yi * yi;
                }
                acc = group_sum64<L>(acc);
                if constexpr (LOGNAVG >= 4) {
                    if (m == kW * v + s0 / kTilesPerWin) keep = (float)(sb2 * (double)acc);
                } else {
                    const int t = tu + 64 * wave + 16 * s0 + m;
                    const int uwin = t >> LOGNAVG;
                    if ((m & ((1 << L) - 1)) == 0 && uwin < nwin && beam < nbeam)
                        out[((int64_t)beam * nchan + u.f) * nwin + uwin] = (float)(sb2 * (double)acc);
                }
            }
        }
        if constexpr (LOGNAVG >= 4) {
            static_assert(kTiles == 4, "at most four windows per beam and wave");
            const int beam = u.bg * kBeams + 16 * mt + 4 * q + m / kW;
            const int uwin = ((tu + 64 * wave) >> LOGNAVG) + m % kW;
            if (m < 4 * kW && uwin < nwin && beam < nbeam)
                out[((int64_t)beam * nchan + u.f) * nwin + uwin] = keep;
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent kernel for up to 512 inputs (the paper's 256 dual-polarisation
// antennas and below).  All weights of a (channel, 32-beam group) fit in the
// registers of the waves that use them (8 K steps of 64 inputs), so a work
// item covers 1024 samples with its weights loaded once, and the LDS ring runs
// on across items: no pipeline restart between items.
//
// Item = (channel, beam group, 1024 samples), walked by a persistent grid of
// one workgroup per CU (items of one channel on one XCD, as above).  Eight
// waves: wave w takes M tile w >> 2 (16 beams) and time quarter w & 3, the 256
// consecutive samples 256 (w & 3) .. of the item, one 16-sample tile per
// stage.  A stage is 64 time rows (16 per quarter) x 512 bytes (every input of
// the row), 32 KiB; four stages rotate, three in flight.  The 16-byte chunks
// of row R sit at chunk ^ (R & 15), so the 16 rows a wave reads per K step
// fall on distinct bank groups.
//
// The product is taken transposed, D[sample][beam] = X W^T (the operands of
// v_mfma_i32_16x16x64_i8 have the same lane layout on both sides), so a lane
// holds four consecutive samples of one beam: windows of up to 4 samples are
// lane-local, 8 and 16 add the lanes 16 and 32 away, 32 and 64 add
// consecutive stages.  From 16 samples a window on, a lane gathers its beam's
// windows of consecutive stages in registers and stores them once per item
// (4, 2 or 1 windows).  The nibble split takes two operations per word
// instead of three: R = 16 re (mask) and X' = 16 re + im + 8 (flip bit 3),
//   P1 = R Wre, P2 = X' Wre, Q1 = R Wim, Q2 = X' Wim,
//   Re y = P1/16 - (Q2 - Q1 - 8 S_im),  Im y = Q1/16 + (P2 - P1 - 8 S_re),
// with S_re, S_im the sums of the beam's weight components over the inputs,
// computed once per item.  Every term is an exact int32.
//
// Weights travel through LDS too, so that their transfer is counted by the
// same vector-memory waits as the ring: the (32 beams x 512 inputs x 2) bytes
// of the next item are fetched into a 32 KiB buffer at stage 8 of the current
// item, counted in with the ring's waits from stage 12 on, and read into
// registers (de-interleaved) after the MFMAs of the current item's last stage.
// Beam row b sits at 1 KiB * b with chunk c at c ^ (b & 15), so the 16 beams
// a wave reads per K step fall on distinct bank groups.
constexpr int kPWaves = 8;
constexpr int kPThreads = 64 * kPWaves;
constexpr int kPRow = 512;                        // LDS bytes per time row
constexpr int kPStage = 64 * kPRow;               // 32 KiB
constexpr int kPSlots = 4;
constexpr int kPWBytes = kBeams * 1024;           // weight buffer, 32 KiB
constexpr int kPLds = kPSlots * kPStage + kPWBytes;  // 160 KiB
constexpr int kPDma = kPStage / 1024 / kPWaves;   // 4 DMA instructions per wave and stage
constexpr int kPWDma = kPWBytes / 1024 / kPWaves;  // 4 per wave for the weights
constexpr int kPItemT = 1024;                     // samples per item
constexpr int kPStages = kPItemT / 64;            // 16 stages per item
constexpr int kPKS = kPRow / 64;                  // K steps of 64 inputs
constexpr int kPWStage = 8;                       // stage of an item that fetches the next item's weights
constexpr int kPMaxInput = kPRow;
static_assert(kPWStage + kPSlots < kPStages, "the next item's weights land before the item's last stage");

__device__ const uint4 kZero16 = {0u, 0u, 0u, 0u};

// Item cursor shared by the producer and the consumer side.
struct PItem {
    int B;      // flat item id
    bool valid;
    Unit u;
};

__device__ __forceinline__ void pitem_first(PItem &c, int start, int grid, int total, int ntb, int nbg,
                                            int nchan) {
    c.B = start;
    c.valid = false;
    while (c.B < total && !(c.valid = unit_of(c.B, ntb, nbg, nchan, c.u))) c.B += grid;
}

__device__ __forceinline__ void pitem_next(PItem &c, int grid, int total, int ntb, int nbg, int nchan) {
    pitem_first(c, c.B + grid, grid, total, ntb, nbg, nchan);
}

// dma16 from a wave-uniform base plus a 32-bit per-lane offset (the
// scalar-base form of the instruction): the base moves with the stage, the
// offsets stay in registers for the whole launch.
__device__ inline void dma16_at(const uint8_t *base, uint32_t off, uint32_t lds_wave_base) {
    const uint64_t b = (uint64_t)(uintptr_t)base;
    const uint64_t ub = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, %2"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_wave_base)), "v"(off), "s"(ub)
                 : "memory", "m0");
}

// This wave's share of a stage: LDS row R = 2 (kPDma wave + j) + lane / 32
// (j < kPDma), all in the time quarter wave / 2, holds sample
// T0 + 256 (R >> 4) + 16 k + (R & 15) of the item, its physical chunk
// lane % 32 the logical chunk (lane % 32) ^ (R & 15); chunks past the row's
// inputs fetch chunk 0.  The lane's byte offset of row R within the stage,
// (R & 15) rstride + 16 chunk, is below 2^29 (rstride <= 65536 x 512).
static_assert(16 % (2 * kPDma) == 0, "a wave's DMA rows lie in one 16-row group");
__device__ __forceinline__ uint32_t pstage_off(int64_t rstride, int ninput, int wave, int lane, int j) {
    const int R = 2 * (kPDma * wave + j) + (lane >> 5);
    const int c = (lane & 31) ^ (R & 15);
    const int cc = c < (ninput >> 4) ? c : 0;
    return (uint32_t)((R & 15) * rstride + 16 * cc);
}

// Stage k of item u.  Rows past the last sample (only in an item that ends
// early) are clamped to it.
__device__ __forceinline__ void pstage_dma(const uint8_t *x, int64_t rstride, int ninput, int ntime,
                                           const PItem &it, int k, const uint32_t (&doff)[kPDma],
                                           uint32_t lds_stage, int wave, int lane) {
    if (!it.valid) {
#pragma unroll
        for (int j = 0; j < kPDma; ++j) dma16(&kZero16, lds_stage + 1024 * (kPDma * wave + j));
        return;
    }
    const uint8_t *xf = x + (int64_t)it.u.f * ninput;
    const int t16 = it.u.tb * kPItemT + 256 * ((2 * kPDma * wave) >> 4) + 16 * k;  // the rows' first sample
    if (t16 + 16 <= ntime) {
        const uint8_t *base = xf + (int64_t)t16 * rstride;
#pragma unroll
        for (int j = 0; j < kPDma; ++j) dma16_at(base, doff[j], lds_stage + 1024 * (kPDma * wave + j));
        return;
    }
    const int nck = ninput >> 4;
#pragma unroll
    for (int j = 0; j < kPDma; ++j) {
        const int R = 2 * (kPDma * wave + j) + (lane >> 5);
        const int c = (lane & 31) ^ (R & 15);
        const int cc = c < nck ? c : 0;
        const int64_t t = min(t16 + (R & 15), ntime - 1);
        dma16(xf + t * rstride + 16 * cc, lds_stage + 1024 * (kPDma * wave + j));
    }
}

// This wave's share of the weights of item u: beam rows b = kPWDma wave + j.
__device__ __forceinline__ void pweights_dma(const int8_t *w, int ninput, int nbeam, const Unit &u,
                                             uint32_t lds_w, int wave, int lane) {
    const int nck = ninput >> 3;  // 16-byte chunks of one beam row
    const int8_t *w0 = w + (int64_t)u.f * nbeam * ninput * 2;
#pragma unroll
    for (int j = 0; j < kPWDma; ++j) {
        const int b = kPWDma * wave + j;
        const int beam = u.bg * kBeams + b;
        const int c = lane ^ (b & 15);
        const bool ok = c < nck && beam < nbeam;
        const int64_t off = ok ? ((int64_t)beam * ninput * 2 + 16 * c) : 0;
        dma16(w0 + off, lds_w + 1024 * b);
    }
}

template <int LOGNAVG>
__global__ __launch_bounds__(kPThreads, 1) void beamform_ci4_persistent_kernel(
    const uint8_t *__restrict__ x, const int8_t *__restrict__ w, const float *__restrict__ scale,
    int ninput, int nchan, int nbeam, int ntime, int ntb, int nbg, int total, float *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;
    const uint32_t lds_w = lds_base + kPSlots * kPStage;
    const uint8_t *wbuf = lds + kPSlots * kPStage;
    const int grid = gridDim.x;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int m = lane & 15;      // A row (beam in the M tile) / B column (sample in the tile)
    const int q = lane >> 4;      // K group of 16 inputs; output rows 4q .. 4q+3
    const int mt = wave >> 2;     // M tile
    const int qw = wave & 3;      // time quarter
    const int64_t rstride = (int64_t)nchan * ninput;
    const int nks = ninput >> 6;
    const int R = 16 * qw + m;    // LDS row of this lane's B fragments
    uint32_t doff[kPDma];         // this lane's DMA offsets within a stage
#pragma unroll
    for (int j = 0; j < kPDma; ++j) doff[j] = pstage_off(rstride, ninput, wave, lane, j);

    PItem cit;  // consumer's item
    pitem_first(cit, blockIdx.x, grid, total, ntb, nbg, nchan);
    if (!cit.valid) return;
    PItem pit = cit;  // producer's item
    int pk = 0;       // producer's stage within pit

    auto produce = [&](uint32_t slot_base) __attribute__((always_inline)) {
        pstage_dma(x, rstride, ninput, ntime, pit, pk, doff, slot_base, wave, lane);
        if (pit.valid && ++pk == kPStages) {
            pk = 0;
            pitem_next(pit, grid, total, ntb, nbg, nchan);
        }
    };

    // prologue: the first item's weights, then stages 0 .. 3
    pweights_dma(w, ninput, nbeam, cit.u, lds_w, wave, lane);
#pragma unroll
    for (int i = 0; i < kPSlots; ++i) produce(lds_base + i * kPStage);
    wait_vm<(kPSlots - 1) * kPDma>();  // weights and stage 0
    block_barrier();

    v4i wre[kPKS], wim[kPKS];
    auto load_weights = [&]() __attribute__((always_inline)) {
        const uint8_t *row = wbuf + 1024 * (16 * mt + m);
#pragma unroll
        for (int ks = 0; ks < kPKS; ++ks) {
            v4i a = v4i{0, 0, 0, 0}, b = v4i{0, 0, 0, 0};
            if (ks < nks) {
                const int c = 8 * ks + 2 * q;
                a = *(const v4i *)(row + 16 * (c ^ m));
                b = *(const v4i *)(row + 16 * ((c + 1) ^ m));
            }
            wre[ks] = v4i{(int)__builtin_amdgcn_perm(a[1], a[0], 0x06040200u),
                          (int)__builtin_amdgcn_perm(a[3], a[2], 0x06040200u),
                          (int)__builtin_amdgcn_perm(b[1], b[0], 0x06040200u),
                          (int)__builtin_amdgcn_perm(b[3], b[2], 0x06040200u)};
            wim[ks] = v4i{(int)__builtin_amdgcn_perm(a[1], a[0], 0x07050301u),
                          (int)__builtin_amdgcn_perm(a[3], a[2], 0x07050301u),
                          (int)__builtin_amdgcn_perm(b[1], b[0], 0x07050301u),
                          (int)__builtin_amdgcn_perm(b[3], b[2], 0x07050301u)};
        }
    };
    // (every K step unguarded when the item has all kPKS of them: a
    // branch per step would keep the compiler from overlapping them)
    const bool full = nks == kPKS;
    auto read_frags = [&](const uint8_t *stage, v4i (&f)[kPKS]) __attribute__((always_inline)) {
        const uint8_t *row = stage + kPRow * R;
        if (full) {
#pragma unroll
            for (int ks = 0; ks < kPKS; ++ks) f[ks] = *(const v4i *)(row + 16 * ((4 * ks + q) ^ m));
        } else {
#pragma unroll
            for (int ks = 0; ks < kPKS; ++ks)
                if (ks < nks) f[ks] = *(const v4i *)(row + 16 * ((4 * ks + q) ^ m));
        }
    };

    // Per-item constants of this lane's beam (bg*32 + 16 mt + m): its squared
    // scale, and 8 x the sums of its weights' real and imaginary parts over
    // all inputs (the offset that X' carries into P2 and Q2).
    const int nwin = ntime >> LOGNAVG;
    double sb2 = 0.0;
    int c8im = 0, m8re = 0;  // 8 S_im and -8 S_re
    float *ob = out;         // the beam's row of windows in this item's channel
    bool bok = false;        // the lane's beam exists
    auto item_consts = [&]() __attribute__((always_inline)) {
        const int beam = cit.u.bg * kBeams + 16 * mt + m;
        bok = beam < nbeam;
        ob = out + ((int64_t)beam * nchan + cit.u.f) * nwin;
        const double sb = (double)(bok ? scale[beam] : 0.0f);
        sb2 = sb * sb;
        int sre = 0, sim = 0;
#pragma unroll
        for (int ks = 0; ks < kPKS; ++ks)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sre = __builtin_amdgcn_sdot4(wre[ks][k], 0x01010101, sre, false);
                sim = __builtin_amdgcn_sdot4(wim[ks][k], 0x01010101, sim, false);
            }
        // the four K groups of the beam are the lanes m, m+16, m+32, m+48
        sre += swz_xor<16>(sre);
        sim += swz_xor<16>(sim);
        sre += xor32(sre, lane);
        sim += xor32(sim, lane);
        m8re = -8 * sre;
        c8im = 8 * sim;
    };

    v4i fa[kPKS], fb[kPKS];
#pragma unroll
    for (int ks = 0; ks < kPKS; ++ks) fa[ks] = fb[ks] = v4i{0, 0, 0, 0};
    load_weights();
    item_consts();
    read_frags(lds, fa);

    constexpr int kTilesPerWin = LOGNAVG > 4 ? 1 << (LOGNAVG - 4) : 1;
    double part = 0.0;
    float kw[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // a lane's windows of the item (navg >= 16)
    // every beam row of windows starts 16-byte (8-byte) aligned
    const bool row16 = (nwin & 3) == 0 && ((uintptr_t)out & 15) == 0;
    const bool row8 = (nwin & 1) == 0 && ((uintptr_t)out & 7) == 0;
    PItem cnext = cit;  // the consumer's next item
    pitem_next(cnext, grid, total, ntb, nbg, nchan);
    int ck = 0;         // consumer's stage within cit
    unsigned i = 0;     // consumer's stage in the workgroup's sequence

    // One stage: reads of stage i+1 into nxt, MFMAs and detection of stage i
    // from cur.  Returns whether a stage follows.
    auto step = [&](v4i (&cur)[kPKS], v4i (&nxt)[kPKS]) __attribute__((always_inline)) {
        const bool last = ck + 1 == kPStages;
        const bool more = !last || cnext.valid;
        if (more) {
            // Stage i+1 has landed.  Younger than it: kPSlots - 2 stages of
            // DMA, and the next item's weights while they were fetched behind
            // it (issued at stage kPWStage behind stage kPWStage + kPSlots).
            if (cnext.valid && ck > kPWStage && ck < kPWStage + kPSlots)
                wait_vm<(kPSlots - 2) * kPDma + kPWDma>();
            else
                wait_vm<(kPSlots - 2) * kPDma>();
            wait_lds();  // every read of stage i has returned: its slot is refilled now
            block_barrier();
            produce(lds_base + (i % kPSlots) * kPStage);
            if (ck == kPWStage && cnext.valid) pweights_dma(w, ninput, nbeam, cnext.u, lds_w, wave, lane);
            read_frags(lds + ((i + 1) % kPSlots) * kPStage, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);
        // D[sample][beam] = X W^T over the stage's 16 samples: P1 = R Wre,
        // P2 = X' Wre, Q1 = R Wim, Q2 = X' Wim (R = 16 re, X' = 16 re + im + 8)
        v4i p1 = v4i{0, 0, 0, 0}, p2 = p1, q1 = p1, q2 = p1;
        auto kstep = [&](int ks) __attribute__((always_inline)) {
            v4i r, xo;
            split_ci4_offset(cur[ks], r, xo);
            p1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(r, wre[ks], p1, 0, 0, 0);
            q2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(xo, wim[ks], q2, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(xo, wre[ks], p2, 0, 0, 0);
            q1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(r, wim[ks], q1, 0, 0, 0);
        };
        if (full) {
#pragma unroll
            for (int ks = 0; ks < kPKS; ++ks) kstep(ks);
        } else {
#pragma unroll
            for (int ks = 0; ks < kPKS; ++ks)
                if (ks < nks) kstep(ks);
        }
        __builtin_amdgcn_sched_barrier(0);
        // the next item's weights (in LDS since its stage kPWStage + kPSlots)
        if (last && more) load_weights();
        // Detect and integrate.  Lane: beam bg*32 + 16 mt + m, samples
        // T0 + 256 qw + 16 ck + 4q + v (v = 0..3), so windows of up to 4
        // samples are lane-local, 8 and 16 add the lanes 16 and 32 away, 32
        // and 64 add consecutive stages.
        const int tw = cit.u.tb * kPItemT + 256 * qw + 16 * ck;  // the wave's first sample
        const int t0 = tw + 4 * q;
        // |y|^2 in binary64: with at most 512 inputs |Re y|, |Im y| < 2^20, so
        // every sample's power is an integer below 2^41 and a window's sum
        // (up to 64 samples) one below 2^47, exact in binary64 whatever the
        // order of the additions.
        double dr[4], di[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            dr[v] = (double)((p1[v] >> 4) + (q1[v] - q2[v]) + c8im);
            di[v] = (double)((q1[v] >> 4) + (p2[v] - p1[v]) + m8re);
        }
        if constexpr (LOGNAVG == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (bok && t0 + v < nwin) ob[t0 + v] = (float)(sb2 * __builtin_fma(dr[v], dr[v], di[v] * di[v]));
        } else if constexpr (LOGNAVG == 1) {
            const int u0 = t0 >> 1;
            double e[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int a = 2 * h, b = 2 * h + 1;
                e[h] = __builtin_fma(dr[a], dr[a], di[a] * di[a]);
                e[h] = __builtin_fma(dr[b], dr[b], __builtin_fma(di[b], di[b], e[h]));
            }
            if (bok && u0 < nwin) ob[u0] = (float)(sb2 * e[0]);
            if (bok && u0 + 1 < nwin) ob[u0 + 1] = (float)(sb2 * e[1]);
        } else {
            double sum = di[0] * di[0];
            sum = __builtin_fma(dr[0], dr[0], sum);
#pragma unroll
            for (int v = 1; v < 4; ++v) sum = __builtin_fma(dr[v], dr[v], __builtin_fma(di[v], di[v], sum));
            if constexpr (LOGNAVG >= 3) sum += swz_xor_f64<16>(sum);
            if constexpr (LOGNAVG >= 4) sum += xor32_f64(sum, lane);
            part += sum;
            constexpr int kLeadMask = LOGNAVG >= 4 ? 3 : LOGNAVG == 3 ? 1 : 0;
            if constexpr (LOGNAVG >= 4) {
                // Windows of 16 samples and more: one per kTilesPerWin stages
                // and beam, its sum in every lane of the beam.  Lane (q, m)
                // shifts in the kW consecutive windows kW q .. kW q + kW - 1 of
                // the wave's quarter and stores them at the item's last stage:
                // one store of 4 kW bytes per lane and item instead of a 4-byte
                // store per window to 16 beam rows.
                constexpr int kW = 4 / kTilesPerWin;  // windows per lane and item: 4, 2, 1
                if ((ck % kTilesPerWin) == kTilesPerWin - 1) {
                    const float pw = (float)(sb2 * part);
                    part = 0.0;
                    if (ck / kTilesPerWin < kW * (q + 1)) {
#pragma unroll
                        for (int k = 0; k + 1 < kW; ++k) kw[k] = kw[k + 1];
                        kw[kW - 1] = pw;
                    }
                }
                if (last && bok) {
                    const int u = ((cit.u.tb * kPItemT + 256 * qw) >> LOGNAVG) + kW * q;
                    if (kW == 4 && row16 && u + 4 <= nwin) {
                        *(float4 *)(ob + u) = make_float4(kw[0], kw[1], kw[2], kw[3]);
                    } else if (kW == 2 && row8 && u + 2 <= nwin) {
                        *(float2 *)(ob + u) = make_float2(kw[0], kw[1]);
                    } else {
#pragma unroll
                        for (int v = 0; v < kW; ++v)
                            if (u + v < nwin) ob[u + v] = kw[v];
                    }
                }
            } else {
                // a window ends in this stage
                const int u = t0 >> LOGNAVG;
                if ((q & kLeadMask) == 0 && bok && u < nwin) ob[u] = (float)(sb2 * part);
                part = 0.0;
            }
        }
        if (last) {
            cit = cnext;
            pitem_next(cnext, grid, total, ntb, nbg, nchan);
            ck = 0;
            if (more) item_consts();
        } else {
            ++ck;
        }
        ++i;
        return more;
    };
    while (step(fa, fb) && step(fb, fa)) {
    }
    wait_vm<0>();  // no DMA may still target LDS when the workgroup retires
}

typedef void (*BfKernel)(const uint8_t *, const int8_t *, const float *, int, int, int, int, int, int,
                         float *);
const BfKernel kKernels[7] = {beamform_ci4_kernel<0>, beamform_ci4_kernel<1>, beamform_ci4_kernel<2>,
                              beamform_ci4_kernel<3>, beamform_ci4_kernel<4>, beamform_ci4_kernel<5>,
                              beamform_ci4_kernel<6>};
typedef void (*BfPKernel)(const uint8_t *, const int8_t *, const float *, int, int, int, int, int, int, int,
                          float *);
const BfPKernel kPKernels[7] = {beamform_ci4_persistent_kernel<0>, beamform_ci4_persistent_kernel<1>,
                                beamform_ci4_persistent_kernel<2>, beamform_ci4_persistent_kernel<3>,
                                beamform_ci4_persistent_kernel<4>, beamform_ci4_persistent_kernel<5>,
                                beamform_ci4_persistent_kernel<6>};

DeviceInit g_init;
bool g_persistent_ok[kMaxDevices];  // the device gives a workgroup kPLds bytes of LDS

hipError_t set_attributes() {
    for (BfKernel k : kKernels) {
        const hipError_t e =
            hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
    }
    int dev = 0, lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && optin > lds)
        lds = optin;
    g_persistent_ok[dev] = lds >= kPLds;
    if (!g_persistent_ok[dev]) return hipSuccess;
    for (BfPKernel k : kPKernels) {
        e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, kPLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

bool beamform_ci4_supported(int32_t navg) { return navg >= 1 && navg <= 64 && (navg & (navg - 1)) == 0; }

int64_t beamform_ci4_units(int32_t nchan, int32_t nbeam, int64_t ntime) {
    const int64_t ntb = (ntime + kTB - 1) / kTB;
    const int64_t nbg = (nbeam + kBeams - 1) / kBeams;
    return ((int64_t)nchan + 7) / 8 * 8 * ntb * nbg;
}

hipError_t launch_beamform_ci4(const void *x, const int8_t *w, const float *scale, int32_t ninput,
                               int32_t nchan, int32_t nbeam, int64_t ntime, int32_t navg, float *out,
                               hipStream_t s) {
    int num_cus = 0;
    const hipError_t e = g_init.ensure(set_attributes, &num_cus);
    if (e != hipSuccess) return e;
    int dev = 0;
    const hipError_t ed = hipGetDevice(&dev);
    if (ed != hipSuccess) return ed;
    int lognavg = 0;
    while ((1 << lognavg) < navg) ++lognavg;
    const int nbg = (nbeam + kBeams - 1) / kBeams;
    const int64_t units = beamform_ci4_units(nchan, nbeam, ntime);
    if (units > kMaxWorkgroups256) return hipErrorInvalidConfiguration;
    if (ninput <= kPMaxInput && g_persistent_ok[dev]) {
        // items of 1024 samples: never more than the 256-sample units above
        const int ntb = (int)((ntime + kPItemT - 1) / kPItemT);
        const int64_t total = ((int64_t)nchan + 7) / 8 * 8 * ntb * nbg;
        int64_t grid = (int64_t)(num_cus > 0 ? num_cus : 256) / 8 * 8;
        if (grid < 8) grid = 8;
        if (grid > total) grid = total;
        hipLaunchKernelGGL(kPKernels[lognavg], dim3((unsigned)grid), dim3(kPThreads), kPLds, s,
                           (const uint8_t *)x, w, scale, ninput, nchan, nbeam, (int)ntime, ntb, nbg, (int)total,
                           out);
        return hipGetLastError();
    }
    const int ntb = (int)((ntime + kTB - 1) / kTB);
    hipLaunchKernelGGL(kKernels[lognavg], dim3((unsigned)units), dim3(kThreads), kLdsBytes, s,
                       (const uint8_t *)x, w, scale, ninput, nchan, nbeam, (int)ntime, ntb, nbg, out);
    return hipGetLastError();
}

}  // namespace bfx
