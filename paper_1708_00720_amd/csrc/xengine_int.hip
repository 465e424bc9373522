// Integer X-engine for gfx950: packed ci4 / ci8 voltages -> int32 visibilities.
//
// Per channel f the kernel forms V = sum_t x_t x_t^H and keeps the lower
// triangle (the FX correlator's cross-multiply; the paper's linear-algebra
// module, Sec. 2.2, and its planned correlation capability, Sec. 7).  The
// contraction over time runs on int8 MFMA with int32 accumulation, so the
// result is the exact integer sum.
//
// Split into real products (a = Re x, b = Im x, sums over t):
//   Re V_ij = sum a_i a_j + b_i b_j
//   Im V_ij = P_ij - Q_ij,  P_ij = sum b_i a_j,  Q_ij = sum a_i b_j
// Accumulators per output tile (Re, P, Q) and no negated operand:
// the full int8 range (including -128) is exact.
//
// Work decomposition, LDS ring and persistent loop: xe_common.h.  Per stage a
// wave issues all of its transposing reads first: ds_read_b64_tr_b8 (ci4: 8
// samples of one input per lane) or ds_read_b64_tr_b16 (ci8: 4 (re,im) pairs
// per lane) turn input-major rows into the K(time)-contiguous layout MFMA
// wants.  ci4 is split in registers into 16*re and 16*im bytes (the nibble
// kept in the high half of the byte is that value times 16 as int8),
// interleaved with the MFMAs of the previous 32-sample step; its products carry
// a factor 256 that the epilogue shifts out exactly.  ci8 (re, im) pairs are
// de-interleaved with v_perm.  MFMA: v_mfma_i32_32x32x32_i8, two waves per
// SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "bfx_internal.h"
#include "xe_common.h"

namespace bfx {
namespace {

// Stage layout plus the number of 32-sample MFMA steps per stage.
template <bool CI4>
struct Fmt : RowFmt<CI4 ? 1 : 2> {
    static constexpr int kKK = RowFmt<CI4 ? 1 : 2>::kT / 32;
};

// A wave's 64x32 tile: two 32x32 sub-blocks (row halves r = 0, 1), each with
// three int32 accumulators: Re V = sum a a + b b, P = sum b a, Q = sum a b
// (Im V = P - Q).  The two MFMAs into a Re accumulator of one 32-sample step
// are six MFMAs apart, longer than an MFMA's latency.
struct Acc {
    v16i rr[2], p[2], q[2];
};

// Packed-voltage fragment of a 32-input sub-block for one 32-sample step:
// lane l holds input (l % 32) of the sub-block at the 16 samples of k-group
// l / 32, as 16*re and 16*im bytes (ci4) or re / im bytes (ci8).
struct Frag {
    v4i re, im;
};

// Per-lane LDS byte offset (within a stage) of the first transposing read of
// the 32-input sub-block starting at LDS input `ioff`.  The remaining reads of
// the fragment are at fixed distances (whole rows), because the swizzle only
// depends on the row index modulo 8 (ci4) or 4 (ci8), which is the same for
// all reads of a lane.
template <bool CI4>
__device__ inline int frag_base(int ioff, int lane) {
    using F = Fmt<CI4>;
    const int G = (lane >> 4) & 3;
    const int k = lane & 15;
    if (CI4) {
        // tr_b8: lanes 2r, 2r+1 of a 16-lane group name the two 8-byte halves
        // of row r (r = 0..7); lane j receives byte j of rows 0..7.
        const int r8 = k >> 1;
        const int c = (ioff >> 4) + (G & 1);
        const int t = 16 * (G >> 1) + r8;
        return t * F::kRow + 16 * (c ^ F::swz(t)) + 8 * (k & 1);
    } else {
        // tr_b16: lanes 4r..4r+3 of a 16-lane group name the four 8-byte
        // quarters of row r (r = 0..3); lane j receives 16-bit element j of
        // rows 0..3, here the (re, im) pair of one input at 4 samples.
        const int r4 = k >> 2;
        const int q = k & 3;
        const int c = ((ioff + 16 * (G & 1)) >> 3) + (q >> 1);
        const int t = 16 * (G >> 1) + r4;
        return t * F::kRow + 16 * (c ^ F::swz(t)) + 8 * (q & 1);
    }
}

// Raw transposed reads of one fragment (before the ci4 nibble split or the
// ci8 (re, im) de-interleave).
template <bool CI4>
struct RawFrag {
    v2i w[CI4 ? 2 : 4];
};

template <bool CI4>
__device__ __forceinline__ RawFrag<CI4> read_frag(const uint8_t *p /* stage + frag_base */, int kk) {
    using F = Fmt<CI4>;
    RawFrag<CI4> r;
    if constexpr (CI4) {
        r.w[0] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)(p + kk * 32 * F::kRow));
        r.w[1] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)(p + (kk * 32 + 8) * F::kRow));
    } else {
#pragma unroll
        for (int rd = 0; rd < 4; ++rd)
            r.w[rd] = __builtin_bit_cast(
                v2i, __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(p + (kk * 32 + 4 * rd) * F::kRow)));
    }
    return r;
}

template <bool CI4>
__device__ __forceinline__ Frag split_frag(const RawFrag<CI4> &r) {
    Frag fr;
    if constexpr (CI4) {
        const uint32_t w[4] = {(uint32_t)r.w[0].x, (uint32_t)r.w[0].y, (uint32_t)r.w[1].x,
                               (uint32_t)r.w[1].y};
        fr.re = v4i{(int)(w[0] & 0xF0F0F0F0u), (int)(w[1] & 0xF0F0F0F0u),
                    (int)(w[2] & 0xF0F0F0F0u), (int)(w[3] & 0xF0F0F0F0u)};
        fr.im = v4i{(int)((w[0] << 4) & 0xF0F0F0F0u), (int)((w[1] << 4) & 0xF0F0F0F0u),
                    (int)((w[2] << 4) & 0xF0F0F0F0u), (int)((w[3] << 4) & 0xF0F0F0F0u)};
    } else {
        uint32_t re[4], im[4];
#pragma unroll
        for (int rd = 0; rd < 4; ++rd) {
            re[rd] = perm((uint32_t)r.w[rd].y, (uint32_t)r.w[rd].x, 0x06040200u);
            im[rd] = perm((uint32_t)r.w[rd].y, (uint32_t)r.w[rd].x, 0x07050301u);
        }
        fr.re = v4i{(int)re[0], (int)re[1], (int)re[2], (int)re[3]};
        fr.im = v4i{(int)im[0], (int)im[1], (int)im[2], (int)im[3]};
    }
    return fr;
}

// The eight MFMAs of one 32-sample step of a 64x32 tile (row fragments a0,
// a1, column fragment b), split for the stage's head (the first kHead) and
// tail (the rest).
__device__ __forceinline__ void mfma_k(int k, const Frag &a0, const Frag &a1, const Frag &b, Acc &acc) {
    switch (k) {
        case 0: acc.rr[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.re, b.re, acc.rr[0], 0, 0, 0); break;
        case 1: acc.rr[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.re, b.re, acc.rr[1], 0, 0, 0); break;
        case 2: acc.p[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.im, b.re, acc.p[0], 0, 0, 0); break;
        case 3: acc.p[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.im, b.re, acc.p[1], 0, 0, 0); break;
        case 4: acc.q[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.re, b.im, acc.q[0], 0, 0, 0); break;
        case 5: acc.q[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.re, b.im, acc.q[1], 0, 0, 0); break;
        case 6: acc.rr[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.im, b.im, acc.rr[0], 0, 0, 0); break;
        default: acc.rr[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.im, b.im, acc.rr[1], 0, 0, 0); break;
    }
}

// Raw transposing reads of one stage of a wave's 64x32 tile: per 32-sample
// step the two row fragments and the column fragment.
template <bool CI4>
struct StageRaw {
    RawFrag<CI4> r[Fmt<CI4>::kKK][3];
};

// Operands of a stage's first 32-sample step, formed from its raw reads
// during the previous stage.
struct StagePre {
    Frag f[3];
};

template <bool CI4>
__device__ __forceinline__ void read_stage(const uint8_t *stage, const int (&fb)[3], StageRaw<CI4> &raw) {
#pragma unroll
    for (int kk = 0; kk < Fmt<CI4>::kKK; ++kk)
#pragma unroll
        for (int f = 0; f < 3; ++f) raw.r[kk][f] = read_frag<CI4>(stage + fb[f], kk);
}

// MFMAs of a stage that run before its DMA and reads are issued.
constexpr int kHead = 2;

// MFMAs K0..7 of one step: the first KLEAD back to back, each later one
// followed by a slice of the VALU work the caller placed in the same
// scheduling region (NVALU operations in all).  A lead gives transposing
// reads issued just before the step time to return before the VALU work that
// consumes them stalls the MFMA issue behind it.
template <int K0, int KLEAD, int NVALU>
__device__ __forceinline__ void mfma_run(const Frag &a0, const Frag &a1, const Frag &b, Acc &acc) {
#pragma unroll
    for (int k = K0; k < 8; ++k) mfma_k(k, a0, a1, b, acc);
    constexpr int kRest = 8 - K0 - KLEAD;
    constexpr int kPer = (NVALU + kRest - 1) / kRest;
    __builtin_amdgcn_sched_group_barrier(kSchedMfma, KLEAD, 0);
#pragma unroll
    for (int i = 0; i < kRest; ++i) {
        __builtin_amdgcn_sched_group_barrier(kSchedMfma, 1, 0);
        __builtin_amdgcn_sched_group_barrier(kSchedValu, kPer, 0);
    }
}

// The rest of a stage's MFMA work, from registers: the remaining MFMAs of the
// first step, then the later steps, each step's split interleaved with the
// MFMAs of the step before; the last step carries the split of the next
// stage's first step (whose reads were issued after the head).  Every MFMA is
// unconditional (a dead sub-block of a diagonal or ragged pair, or an idle
// wave, computes values that are never stored): conditional MFMAs force
// accumulator copies at every merge point.
template <bool CI4>
__device__ __forceinline__ void stage_tail(const StagePre &pre, const StageRaw<CI4> &raw,
                                           const StageRaw<CI4> &nraw, StagePre &npre, Acc &acc) {
    constexpr int KK = Fmt<CI4>::kKK;
    constexpr int kSplitValu = CI4 ? 36 : 24;  // VALU operations of one step's split
    static_assert(KK == 1 || KK == 2, "one or two 32-sample steps per stage");
    if constexpr (KK == 1) {
#pragma unroll
        for (int f = 0; f < 3; ++f) npre.f[f] = split_frag<CI4>(nraw.r[0][f]);
        mfma_run<kHead, 3, kSplitValu>(pre.f[0], pre.f[1], pre.f[2], acc);
        __builtin_amdgcn_sched_barrier(0);
    } else {
        Frag mid[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) mid[f] = split_frag<CI4>(raw.r[1][f]);
        mfma_run<kHead, 0, kSplitValu>(pre.f[0], pre.f[1], pre.f[2], acc);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int f = 0; f < 3; ++f) npre.f[f] = split_frag<CI4>(nraw.r[0][f]);
        mfma_run<0, 2, kSplitValu>(mid[0], mid[1], mid[2], acc);
        __builtin_amdgcn_sched_barrier(0);
    }
    // ci4: pin the next stage's operands here; otherwise the split is sunk
    // past the loop's exit test into the next stage, in front of its first
    // MFMAs.  (For ci8 the pinned registers cost more than the overlap gains.)
    if constexpr (CI4) {
#pragma unroll
        for (int f = 0; f < 3; ++f) asm volatile("" : "+v"(npre.f[f].re), "+v"(npre.f[f].im));
    }
}

// Store a wave's finished 64x32 tile.  32x32 output layout of
// v_mfma_*_32x32: lane l, register v hold row 8*(v/4) + 4*(l/32) + v%4,
// column l%32.  Row i of the packed triangle starts at element i(i+1)/2, so
// with i = i0 + d the element offset is tri(i0) + d*i0 + tri(d) + j: one
// multiply-add per register from per-lane bases (32-bit: a channel holds
// fewer than 2^31 bytes of visibilities).  Interior tiles (every element
// inside the triangle and the array) store without a per-element test.
// When adding to the stored values, a sub-block's 16 old values are all
// loaded, then added, then stored: no store waits on a load issued after an
// earlier store (a wait for one load's data also waits for every store
// before it).
// Four int32 at an 8-byte-aligned address (one 16-byte store).
typedef int v4i8a __attribute__((ext_vector_type(4), aligned(8)));

// Swap with the neighbouring lane (DPP quad_perm [1,0,3,2]).
__device__ __forceinline__ int swap_lane(int x) { return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false); }

template <bool CI4>
__device__ __forceinline__ void store_sub(uint8_t *obase, int irow0, int jcol0, const v16i &re, const v16i &pp,
                                          const v16i &qq, int lane, int ninput, int overwrite) {
    const int g = lane >> 5;
    const int jj = jcol0 + (lane & 31);
    const int i0 = irow0 + 4 * g;
    const uint32_t base = (uint32_t)((i0 * (i0 + 1) / 2 + jj) * 8);
    const uint32_t step = (uint32_t)(i0 * 8);
    // every row >= every column and inside the array?
    const bool interior = irow0 >= jcol0 + 31 && irow0 + 31 < ninput;
    auto dof = [](int v) { return 8 * (v >> 2) + (v & 3); };
    auto dst = [&](int v) {
        const int d = dof(v);
        return (int2 *)(obase + base + (uint32_t)d * step + (uint32_t)(d * (d + 1) / 2 * 8));
    };
    auto ok = [&](int v) {
        const int i = i0 + dof(v);
        return i < ninput && jj <= i;
    };
    int2 res[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        int vr = re[v];
        int vi = pp[v] - qq[v];
        if (CI4) { vr >>= 8; vi >>= 8; }
        res[v] = int2{vr, vi};
    }
    if (!overwrite) {
        int2 old[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            old[v] = int2{0, 0};
            if (interior || ok(v)) old[v] = *dst(v);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < 16; ++v) res[v] = int2{res[v].x + old[v].x, res[v].y + old[v].y};
        __builtin_amdgcn_sched_barrier(0);
    }
    if (interior) {
        // Neighbouring lanes hold neighbouring columns of the same rows.  Each
        // lane pair swaps registers v and v+1 (rows d and d+1) with DPP, so the
        // even lane stores columns (jj, jj+1) of row d and the odd lane columns
        // (jj-1, jj) of row d+1: 16 bytes each, half the store instructions.
        // Every select below has one swapped operand, so none becomes a
        // per-lane indexed read of the accumulators.
        const bool odd = lane & 1;
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
            const int2 a = res[v], b = res[v + 1];
            const int sax = swap_lane(a.x), say = swap_lane(a.y);
            const int sbx = swap_lane(b.x), sby = swap_lane(b.y);
            const v4i8a out = odd ? v4i8a{sbx, sby, b.x, b.y} : v4i8a{a.x, a.y, sax, say};
            *(v4i8a *)(odd ? (uint8_t *)dst(v + 1) - 8 : (uint8_t *)dst(v)) = out;
        }
    } else {
#pragma unroll
        for (int v = 0; v < 16; ++v)
            if (ok(v)) *dst(v) = res[v];
    }
}

template <bool CI4>
__device__ __forceinline__ void epilogue(const WaveJob &j, const Item &it, const Acc &acc, int lane,
                                         int overwrite) {
    uint8_t *obase = (uint8_t *)it.out + (int64_t)j.ochan * it.out_chan_bytes;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (!((j.live >> (2 * r + j.ch)) & 1u)) continue;
        store_sub<CI4>(obase, j.rblk * kBlk + 32 * r, j.cblk * kBlk + 32 * j.ch, acc.rr[r], acc.p[r], acc.q[r],
                       lane, it.ninput, overwrite);
    }
}

__device__ inline void zero_acc(Acc &acc) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        acc.rr[r] = v16i{0};
        acc.p[r] = v16i{0};
        acc.q[r] = v16i{0};
    }
}

// Eight waves, two per SIMD: wave w works on 32 columns of block pair w % 4
// (a 64x32 tile with the four accumulators of two 32x32 sub-blocks).
template <bool CI4>
struct IntConsumer {
    static constexpr int kWaves = 8;
    static constexpr int kThreads = 64 * kWaves;
    typedef bfx::Acc Acc;
    typedef StageRaw<CI4> Raw;
    typedef StagePre Pre;
    struct Bases {
        int fb[3];
    };
    __device__ static __forceinline__ WaveJob job(const Task &tk, int wave, int ninput) {
        return make_job_half(tk, wave, ninput);
    }
    __device__ static __forceinline__ void zero(Acc &acc) { zero_acc(acc); }
    __device__ static __forceinline__ void bind(const WaveJob &job, int lane, Bases &b) {
        b.fb[0] = frag_base<CI4>(job.rrow, lane);
        b.fb[1] = frag_base<CI4>(job.rrow + 32, lane);
        b.fb[2] = frag_base<CI4>(job.crow, lane);
    }
    __device__ static __forceinline__ void read(const uint8_t *st, const Bases &b, Raw &raw) {
        read_stage<CI4>(st, b.fb, raw);
    }
    __device__ static __forceinline__ void prep(const Raw &raw, Pre &pre) {
#pragma unroll
        for (int f = 0; f < 3; ++f) pre.f[f] = split_frag<CI4>(raw.r[0][f]);
    }
    __device__ static __forceinline__ void head(const Pre &pre, const Raw &raw, Acc &acc) {
#pragma unroll
        for (int k = 0; k < kHead; ++k) mfma_k(k, pre.f[0], pre.f[1], pre.f[2], acc);
    }
    __device__ static __forceinline__ void tail(const Pre &pre, const Raw &raw, const Raw &nraw, Pre &npre,
                                                Acc &acc) {
        stage_tail<CI4>(pre, raw, nraw, npre, acc);
    }
    __device__ static __forceinline__ void epilogue(const WaveJob &j, const Item &it, const Acc &acc,
                                                    int lane, int overwrite) {
        bfx::epilogue<CI4>(j, it, acc, lane, overwrite);
    }
};

// ---------------------------------------------------------------------------
// ci4 on FP8 MFMA (kernel variants 2 and 3 of a ci4 plan).  Every 4-bit
// two's-complement value v in [-8, 7] is exact in FP8 e4m3, so the four real
// products run on v_mfma_scale_f32_32x32x64_f8f6f4 (e4m3 operands, unit
// scales, binary32 accumulation).  Products are integers of magnitude <= 64
// and a launch sums at most kLaunchMaxTime = 65535 samples, so every partial
// sum is an integer below 2^23 and binary32 holds it exactly: the result is
// the same bits as the int8 path.  On this device FP8 runs at the int8 rate
// and the nibble-to-e4m3 conversion (two byte-table lookups and a sign
// select) costs more vector work than the int8 split, so these variants are
// slower; they are the exact narrow-float alternative the autotuner also
// times.
//
// A stage holds 64 time rows = one K step of 64.  Lane l of a 32-input
// fragment holds input l % 32 at 32 samples of time half l / 32, from four
// ds_read_b64_tr_b8 (8 rows each); A and B fragments use the same time order,
// so their K positions pair up.
using Q8Fmt = RowFmt<1>;
static_assert(Q8Fmt::kT == 64, "one 64-sample FP8 MFMA step per stage");
typedef int v8i __attribute__((ext_vector_type(8)));

struct Q8Acc {
    v16f rr[2], p[2], q[2];
};

struct Q8Frag {
    v8i re, im;
};

__device__ inline int q8_frag_base(int ioff, int lane) {
    using F = Q8Fmt;
    const int G = (lane >> 4) & 3;
    const int k = lane & 15;
    const int c = (ioff >> 4) + (G & 1);
    const int t = 32 * (G >> 1) + (k >> 1);
    return t * F::kRow + 16 * (c ^ F::swz(t)) + 8 * (k & 1);
}

// e4m3 codes of the low nibbles (two's complement) of the four bytes of n:
// 0..7 -> 0x00 0x38 0x40 0x44 0x48 0x4A 0x4C 0x4E, -8..-1 -> 0xD0 0xCE 0xCC
// 0xCA 0xC8 0xC4 0xC0 0xB8 (two 8-entry byte tables, selected by bit 3).
__device__ __forceinline__ uint32_t e4m3_of_nibbles(uint32_t n) {
    const uint32_t sel = n & 0x07070707u;
    const uint32_t pos = perm(0x4E4C4A48u, 0x44403800u, sel);
    const uint32_t neg = perm(0xB8C0C4C8u, 0xCACCCED0u, sel);
    const uint32_t m = perm(0xFFFFFFFFu, 0u, ((n >> 1) & 0x04040404u));  // 0xFF where bit 3 is set
    return (neg & m) | (pos & ~m);
}

struct Q8Consumer {
    static constexpr int kWaves = 8;
    static constexpr int kThreads = 64 * kWaves;
    typedef Q8Acc Acc;
    struct Raw {
        v2i w[3][4];  // fragments a0, a1, b; four transposing reads each
    };
    struct Pre {
        Q8Frag f[3];
    };
    struct Bases {
        int fb[3];
    };
    __device__ static __forceinline__ WaveJob job(const Task &tk, int wave, int ninput) {
        return make_job_half(tk, wave, ninput);
    }
    __device__ static __forceinline__ void zero(Acc &acc) {
#pragma unroll
        for (int r = 0; r < 2; ++r) acc.rr[r] = acc.p[r] = acc.q[r] = v16f{0.0f};
    }
    __device__ static __forceinline__ void bind(const WaveJob &job, int lane, Bases &b) {
        b.fb[0] = q8_frag_base(job.rrow, lane);
        b.fb[1] = q8_frag_base(job.rrow + 32, lane);
        b.fb[2] = q8_frag_base(job.crow, lane);
    }
    __device__ static __forceinline__ void read(const uint8_t *st, const Bases &b, Raw &raw) {
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int rd = 0; rd < 4; ++rd)
                raw.w[f][rd] = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                    (lds_v2i *)(st + b.fb[f] + 8 * rd * Q8Fmt::kRow));
    }
    __device__ static __forceinline__ Q8Frag split(const v2i (&w)[4]) {
        Q8Frag fr;
#pragma unroll
        for (int rd = 0; rd < 4; ++rd)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t x = (uint32_t)(h ? w[rd].y : w[rd].x);
                fr.re[2 * rd + h] = (int)e4m3_of_nibbles(x >> 4);
                fr.im[2 * rd + h] = (int)e4m3_of_nibbles(x);
            }
        return fr;
    }
    __device__ static __forceinline__ void prep(const Raw &raw, Pre &pre) {
#pragma unroll
        for (int f = 0; f < 3; ++f) pre.f[f] = split(raw.w[f]);
    }
    __device__ static __forceinline__ void mfma_k(int k, const Pre &p, Acc &acc) {
        const Q8Frag &a0 = p.f[0], &a1 = p.f[1], &b = p.f[2];
        switch (k) {
            case 0: acc.rr[0] = mfma8(a0.re, b.re, acc.rr[0]); break;
            case 1: acc.rr[1] = mfma8(a1.re, b.re, acc.rr[1]); break;
            case 2: acc.p[0] = mfma8(a0.im, b.re, acc.p[0]); break;
            case 3: acc.p[1] = mfma8(a1.im, b.re, acc.p[1]); break;
            case 4: acc.q[0] = mfma8(a0.re, b.im, acc.q[0]); break;
            case 5: acc.q[1] = mfma8(a1.re, b.im, acc.q[1]); break;
            case 6: acc.rr[0] = mfma8(a0.im, b.im, acc.rr[0]); break;
            default: acc.rr[1] = mfma8(a1.im, b.im, acc.rr[1]); break;
        }
    }
    __device__ static __forceinline__ v16f mfma8(const v8i &a, const v8i &b, const v16f &c) {
        // e4m3 A and B (format 0), scales 2^0 (E8M0 127)
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
    }
    __device__ static __forceinline__ void head(const Pre &pre, const Raw &, Acc &acc) {
#pragma unroll
        for (int k = 0; k < kHead; ++k) mfma_k(k, pre, acc);
    }
    __device__ static __forceinline__ void tail(const Pre &pre, const Raw &, const Raw &nraw, Pre &npre,
                                                Acc &acc) {
        // the remaining MFMAs, each followed by a share of the next stage's
        // conversion (48 dwords of e4m3 codes)
#pragma unroll
        for (int f = 0; f < 3; ++f) npre.f[f] = split(nraw.w[f]);
#pragma unroll
        for (int k = kHead; k < 8; ++k) mfma_k(k, pre, acc);
        __builtin_amdgcn_sched_group_barrier(kSchedMfma, 1, 0);
#pragma unroll
        for (int i = kHead + 1; i < 8; ++i) {
            __builtin_amdgcn_sched_group_barrier(kSchedValu, 70, 0);
            __builtin_amdgcn_sched_group_barrier(kSchedMfma, 1, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    __device__ static __forceinline__ void epilogue(const WaveJob &j, const Item &it, const Acc &acc, int lane,
                                                    int overwrite) {
        // exact integers in binary32 -> int32, then the integer epilogue
        uint8_t *obase = (uint8_t *)it.out + (int64_t)j.ochan * it.out_chan_bytes;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (!((j.live >> (2 * r + j.ch)) & 1u)) continue;
            v16i rr, pp, qq;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                rr[v] = (int)acc.rr[r][v];
                pp[v] = (int)acc.p[r][v];
                qq[v] = (int)acc.q[r][v];
            }
            store_sub<false>(obase, j.rblk * kBlk + 32 * r, j.cblk * kBlk + 32 * j.ch, rr, pp, qq, lane,
                             it.ninput, overwrite);
        }
    }
};

template <int DW>
__global__ __launch_bounds__(Q8Consumer::kThreads, 1) void xengine_q8_kernel(SingleArray w, int nt,
                                                                 int total_flat, int overwrite) {
    xe_loop<Q8Fmt, Q8Consumer, DW>(w, nt, total_flat, overwrite);
}

// The consumer the integer kernels run.
template <bool CI4>
using IntKernelConsumer = IntConsumer<CI4>;

template <bool CI4, int DW>
__global__ __launch_bounds__(IntKernelConsumer<CI4>::kThreads, 1) void xengine_int_kernel(SingleArray w, int nt,
                                                                  int total_flat, int overwrite) {
    xe_loop<Fmt<CI4>, IntKernelConsumer<CI4>, DW>(w, nt, total_flat, overwrite);
}

// Work source of a batched plan: flat id B is work-list entry B, naming a
// subarray, an item and a channel (entries for XCD x sit at B % 8 == x; a
// negative entry pads the per-XCD queues to equal length).  The subarray
// record gives the gulp's place in the arena and the channel's output.
struct BatchArray {
    static constexpr bool kTable = false;
    __device__ __forceinline__ void fill_table(uint2 *, int, int) const {}
    const uint8_t *arena;
    uint8_t *out;
    const BatchUnit *units;
    const int2 *work;
    int64_t ntime;  // samples per gulp (arena layout)
    int64_t t0;     // first time row of this launch
    int bps;

    __device__ __forceinline__ bool get(int B, Item &it) const {
        const int2 e = work[B];
        if (e.x < 0) return false;
        const BatchUnit &u = units[e.x & ((1 << kBatchSubBits) - 1)];
        const int field = (e.x & ~kBatchPacked) >> kBatchSubBits;
        const bool packed = e.x & kBatchPacked;
        it.item = packed ? 0 : field;
        it.npack = packed ? field : 0;
        it.ninput = u.ninput;
        it.nb = u.nb;
        it.t_stride = u.t_stride;
        it.chan_bytes = (int64_t)u.ninput * bps;
        it.out_chan_bytes = (int64_t)u.ninput * (u.ninput + 1) / 2 * 8;
        it.base = arena + ntime * u.in_row_off + t0 * u.t_stride + (int64_t)e.y * it.chan_bytes;
        it.out = out + u.out_off + (int64_t)e.y * it.out_chan_bytes;
        return true;
    }
};

template <bool CI4, int DW>
__global__ __launch_bounds__(IntKernelConsumer<CI4>::kThreads, 1) void xengine_batched_kernel(BatchArray w, int nt,
                                                                      int total_flat,
                                                                      int overwrite) {
    xe_loop<Fmt<CI4>, IntKernelConsumer<CI4>, DW>(w, nt, total_flat, overwrite);
}

// Kernel variants a plan chooses between (index = variant): the number of
// waves that issue the stage DMA.
typedef void (*SingleKernel)(SingleArray, int, int, int);
typedef void (*BatchKernel)(BatchArray, int, int, int);
// ci8 plans: the int8 kernel with four or eight DMA waves; ci4 plans also
// the FP8 kernel (variants 2, 3).
const SingleKernel kSingle[2][kXengineVariants] = {
    {xengine_int_kernel<false, 4>, xengine_int_kernel<false, 8>, nullptr, nullptr},
    {xengine_int_kernel<true, 4>, xengine_int_kernel<true, 8>, xengine_q8_kernel<4>, xengine_q8_kernel<8>}};
const BatchKernel kBatched[2][kBatchedVariants] = {
    {xengine_batched_kernel<false, 4>, xengine_batched_kernel<false, 8>},
    {xengine_batched_kernel<true, 4>, xengine_batched_kernel<true, 8>}};

DeviceInit g_init;

hipError_t set_attributes() {
    for (int c = 0; c < 2; ++c) {
        for (int v = 0; v < kXengineVariants; ++v) {
            if (!kSingle[c][v]) continue;
            const hipError_t e = hipFuncSetAttribute((const void *)kSingle[c][v],
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
            if (e != hipSuccess) return e;
        }
        for (int v = 0; v < kBatchedVariants; ++v) {
            const hipError_t e = hipFuncSetAttribute((const void *)kBatched[c][v],
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace

int64_t xengine_items(int32_t ninput, int32_t nchan) {
    const int nb = (ninput + kBlk - 1) / kBlk;
    return nb == 1 ? ((int64_t)nchan + 3) / 4 : (int64_t)nchan * tri_items(nb);
}

int xengine_num_variants(bfx_dtype in, bool batched) {
    if (batched) return kBatchedVariants;
    return in == BFX_CI4 || in == BFX_CF16 ? 4 : 2;
}

hipError_t launch_xengine_int(bool ci4, const void *in, int64_t nt, int32_t nchan, int32_t ninput,
                              int32_t *out, bool overwrite, int variant, hipStream_t s) {
    if (variant < 0 || variant >= kXengineVariants || !kSingle[ci4][variant]) return hipErrorInvalidValue;
    int num_cus = 0;
    const hipError_t e = g_init.ensure(set_attributes, &num_cus);
    if (e != hipSuccess) return e;
    SingleArray w;
    w.in = (const uint8_t *)in;
    w.out = out;
    w.bps = ci4 ? 1 : 2;
    w.t_stride = (int64_t)nchan * ninput * w.bps;
    w.out_chan_bytes = (int64_t)ninput * (ninput + 1) / 2 * 8;
    w.nchan = nchan;
    w.ninput = ninput;
    w.nb = (ninput + kBlk - 1) / kBlk;
    w.nitems = tri_items(w.nb);
    w.npk = w.nb == 1 ? 4 : 1;
    w.ngroups = (nchan + w.npk - 1) / w.npk;
    const int64_t total_flat = ((int64_t)w.ngroups + 7) / 8 * 8 * w.nitems;
    const int64_t grid = persistent_grid(num_cus, total_flat);
    hipLaunchKernelGGL(kSingle[ci4][variant], dim3((unsigned)grid), dim3(IntKernelConsumer<true>::kThreads),
                       kLdsBytes, s, w, (int)nt, (int)total_flat, (int)overwrite);
    return hipGetLastError();
}

hipError_t launch_xengine_batched(bool ci4, const void *arena, int64_t ntime, int64_t t0,
                                  int64_t nt, const BatchUnit *d_units, const int2 *d_work,
                                  int64_t nwork, void *out, bool overwrite, int variant, hipStream_t s) {
    if (variant < 0 || variant >= kBatchedVariants) return hipErrorInvalidValue;
    int num_cus = 0;
    const hipError_t e = g_init.ensure(set_attributes, &num_cus);
    if (e != hipSuccess) return e;
    BatchArray w;
    w.arena = (const uint8_t *)arena;
    w.out = (uint8_t *)out;
    w.units = d_units;
    w.work = d_work;
    w.ntime = ntime;
    w.t0 = t0;
    w.bps = ci4 ? 1 : 2;
    const int64_t grid = persistent_grid(num_cus, nwork);
    hipLaunchKernelGGL(kBatched[ci4][variant], dim3((unsigned)grid), dim3(IntKernelConsumer<true>::kThreads),
                       kLdsBytes, s, w, (int)nt, (int)nwork, (int)overwrite);
    return hipGetLastError();
}

}  // namespace bfx
