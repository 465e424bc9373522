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
// Three accumulators per output tile (Re, P, Q) and no negated operand: the
// full int8 range (including -128) is exact.
//
// Work decomposition.  Inputs are grouped in blocks of 64.  One workgroup
// (8 waves, two per SIMD) holds up to four input blocks of one channel in LDS
// and produces up to four 64x64 block pairs (I >= J) of the triangle, each
// split between two waves (64 rows x 32 columns each).  The block pairs of
// a channel are packed into work items in closed form (decode_item): 2x2
// super-tiles below the diagonal, diagonal super-tiles that borrow a pair from
// the odd last block row, and the rest of that row in groups of three.  The
// grid is persistent (one workgroup per CU); workgroup b walks the flat work
// ids b, b + grid, ...  Flat id B maps channel f to ids with B % 8 == f % 8, so
// with round-robin dispatch over the 8 XCDs all items of a channel run on one
// XCD and share its L2.
//
// Data path.  A ring of kRing LDS stages of 16 KiB receives raw time rows of
// the four blocks (256 inputs) straight from HBM with global_load_lds_dwordx4
// (no staging registers), kRing-1 stages ahead of the MFMA work and across
// work-item boundaries; every wave issues two of each stage's 16 DMA
// instructions and waits on its own vector-memory counter before the stage
// barrier.  Each row's 16-byte chunks are XOR-swizzled by the row index so the
// transposing reads below are free of bank conflicts.  Per stage a wave issues
// all of its transposing reads first: ds_read_b64_tr_b8 (ci4: 8 samples of one
// input per lane) or ds_read_b64_tr_b16 (ci8: 4 (re,im) pairs per lane) turn
// input-major rows into the K(time)-contiguous layout MFMA wants.  ci4 is split
// in registers into 16*re and 16*im bytes (the nibble kept in the high half of
// the byte is that value times 16 as int8), interleaved with the MFMAs of the
// previous 32-sample step; its products carry a factor 256 that the epilogue
// shifts out exactly.  ci8 (re, im) pairs are de-interleaved with v_perm.
// MFMA: v_mfma_i32_32x32x32_i8, two waves per SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "bfx_internal.h"

namespace bfx {
namespace {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v2i lds_v2i;
typedef __attribute__((address_space(3))) v4s lds_v4s;

constexpr int kBlk = 64;          // inputs per block / LDS slot
constexpr int kSlots = 4;         // input blocks held per work item
constexpr int kWaves = 8;         // two block-pair halves per SIMD
constexpr int kDmaWaves = kWaves; // every wave issues part of each stage's DMA
constexpr int kThreads = 64 * kWaves;
constexpr int kStageBytes = 16384;
constexpr int kRing = 8;          // LDS stages in flight (128 KiB)
constexpr int kLdsBytes = kRing * kStageBytes;
constexpr int kDmaPerWave = kStageBytes / 1024 / kDmaWaves;  // 16-byte-per-lane DMA instructions

// Layout traits of one LDS stage: kT time rows of 256 inputs.
template <bool CI4>
struct Fmt {
    static constexpr int kBps = CI4 ? 1 : 2;            // bytes per sample
    static constexpr int kRow = kSlots * kBlk * kBps;   // bytes per time row
    static constexpr int kT = kStageBytes / kRow;       // time rows per stage (64 / 32)
    static constexpr int kKK = kT / 32;                 // 32-sample MFMA steps per stage
    static constexpr int kChunks = kRow / 16;           // 16-byte chunks per row
    static constexpr int kChunksPerSlot = kChunks / kSlots;
    static constexpr int kInputsPerChunk = 16 / kBps;
    static constexpr int kRowsPerDma = 1024 / kRow;     // rows covered by one wave DMA
    // XOR swizzle of the 16-byte chunks of row t.  A transposing read touches
    // rows t0..t0+7 (ci4) or t0..t0+3 (ci8) of two adjacent chunks per
    // 16-lane group; these swizzles map the chunks of a 32-lane half to
    // distinct bank groups.
    __device__ static inline int swz(int t) { return CI4 ? ((t & 7) << 1) : ((t & 3) << 2); }
};

struct Task {
    int blk[kSlots];  // input block held by each LDS slot, -1 = unused
    int rs[4];        // per block pair: LDS slot of its row block, -1 = unused
    int cs[4];        // per block pair: LDS slot of its column block
};

__host__ __device__ inline int tri_items(int nb) {
    int h = nb / 2;
    int s = h * (h + 1) / 2;
    if (nb & 1) s += (h == 0) ? 1 : (h + 2) / 3;
    return s;
}

// Closed-form packing of the lower-triangle block pairs of an nb x nb grid.
__device__ inline void decode_item(int nb, int item, Task &tk) {
    const int h = nb / 2;
    const int S = h * (h + 1) / 2;
    const bool odd = nb & 1;
    for (int k = 0; k < 4; ++k) { tk.blk[k] = -1; tk.rs[k] = -1; tk.cs[k] = -1; }
    if (item < S) {
        int a = (int)((sqrtf(8.0f * item + 1.0f) - 1.0f) * 0.5f);
        while ((a + 1) * (a + 2) / 2 <= item) ++a;
        while (a * (a + 1) / 2 > item) --a;
        const int b = item - a * (a + 1) / 2;
        if (b < a) {
            tk.blk[0] = 2 * a; tk.blk[1] = 2 * a + 1; tk.blk[2] = 2 * b; tk.blk[3] = 2 * b + 1;
            tk.rs[0] = 0; tk.cs[0] = 2;
            tk.rs[1] = 0; tk.cs[1] = 3;
            tk.rs[2] = 1; tk.cs[2] = 2;
            tk.rs[3] = 1; tk.cs[3] = 3;
        } else {
            tk.blk[0] = 2 * a; tk.blk[1] = 2 * a + 1;
            tk.rs[0] = 0; tk.cs[0] = 0;
            tk.rs[1] = 1; tk.cs[1] = 0;
            tk.rs[2] = 1; tk.cs[2] = 1;
            if (odd) { tk.blk[2] = nb - 1; tk.rs[3] = 2; tk.cs[3] = 0; }
        }
    } else {
        const int g = item - S;
        tk.blk[0] = nb - 1;
        for (int w = 0; w < 3; ++w) {
            const int k = 3 * g + w;
            if (k < h) { tk.blk[w + 1] = 2 * k + 1; tk.rs[w] = 0; tk.cs[w] = w + 1; }
        }
        if (g == 0) { tk.rs[3] = 0; tk.cs[3] = 0; }
    }
}

// Select element k of a 4-element task array without dynamic indexing (which
// would place the array in scratch or LDS).
__device__ inline int pick4(const int (&a)[4], int k) {
    return k == 0 ? a[0] : k == 1 ? a[1] : k == 2 ? a[2] : a[3];
}

// Flat work id -> (channel, item); false for the padding ids of a channel
// count that is not a multiple of 8.
__device__ inline bool flat_item(int B, int nitems, int nchan, int &f, int &item) {
    const int s = B >> 3;
    const int cl = s / nitems;
    item = s - cl * nitems;
    f = cl * 8 + (B & 7);
    return f < nchan;
}

__device__ inline uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// 16 bytes from global memory straight into LDS at m0 + 16 * lane.  Issued as
// inline assembly so that the compiler does not serialise the ring with its
// own conservative waits; completion is tracked by the explicit vmcnt waits.
__device__ inline void dma16(const void *src, uint32_t lds_wave_base) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_wave_base)), "v"(src)
                 : "memory", "m0");
}

// Wait until at most N vector-memory operations of this wave are in flight
// (gfx9 encoding: vmcnt split over bits 3:0 and 15:14; expcnt and lgkmcnt
// left at their maxima).
template <int N>
__device__ inline void wait_vm() {
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}


// Wait until every DMA issued for stages up to the awaited one has landed,
// given `ahead` stages issued after it (each kDmaPerWave instructions).
__device__ __forceinline__ void wait_stage(int ahead) {
    static_assert(kRing - 2 <= 6, "extend the cases below");
    switch (ahead) {
        case 6: wait_vm<6 * kDmaPerWave>(); break;
        case 5: wait_vm<5 * kDmaPerWave>(); break;
        case 4: wait_vm<4 * kDmaPerWave>(); break;
        case 3: wait_vm<3 * kDmaPerWave>(); break;
        case 2: wait_vm<2 * kDmaPerWave>(); break;
        case 1: wait_vm<1 * kDmaPerWave>(); break;
        default: wait_vm<0>(); break;
    }
}

__device__ inline void block_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ const uint4 kZeroChunk = {0u, 0u, 0u, 0u};

// A wave's 64x32 tile: two 32x32 sub-blocks (row halves r = 0, 1).
struct Acc {
    v16i re[2], p[2], q[2];
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

__device__ __forceinline__ void mfma8(const Frag &a0, const Frag &a1, const Frag &b, Acc &acc) {
    // the two MFMAs adding into acc.re are separated by the others
    acc.re[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.re, b.re, acc.re[0], 0, 0, 0);
    acc.re[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.re, b.re, acc.re[1], 0, 0, 0);
    acc.p[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.im, b.re, acc.p[0], 0, 0, 0);
    acc.p[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.im, b.re, acc.p[1], 0, 0, 0);
    acc.q[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.re, b.im, acc.q[0], 0, 0, 0);
    acc.q[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.re, b.im, acc.q[1], 0, 0, 0);
    acc.re[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0.im, b.im, acc.re[0], 0, 0, 0);
    acc.re[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1.im, b.im, acc.re[1], 0, 0, 0);
}

// Scheduling masks of __builtin_amdgcn_sched_group_barrier.
constexpr int kSchedValu = 0x2;
constexpr int kSchedMfma = 0x8;

// One stage of a wave's 64x32 tile.  All transposing reads of the stage are
// issued first (one LDS latency per stage instead of one per fragment); the
// split of the next 32-sample step is interleaved with the MFMAs of the
// current one.  Every MFMA is unconditional (a dead sub-block of a diagonal
// or ragged pair is computed and simply not stored): conditional MFMAs force
// accumulator copies at every merge point.
template <bool CI4>
__device__ __forceinline__ void mfma_stage(const uint8_t *stage, const int (&fb)[3], Acc &acc) {
    constexpr int KK = Fmt<CI4>::kKK;
    RawFrag<CI4> raw[KK][3];
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
        for (int f = 0; f < 3; ++f) raw[kk][f] = read_frag<CI4>(stage + fb[f], kk);
    __builtin_amdgcn_sched_barrier(0);  // keep every read ahead of the arithmetic
    Frag cur[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) cur[f] = split_frag<CI4>(raw[0][f]);
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
        Frag nxt[3];
        if (kk + 1 < KK) {
#pragma unroll
            for (int f = 0; f < 3; ++f) nxt[f] = split_frag<CI4>(raw[kk + 1][f]);
        }
        mfma8(cur[0], cur[1], cur[2], acc);
        if (kk + 1 < KK) {
            // 8 MFMAs, each followed by a slice of the next step's split
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                __builtin_amdgcn_sched_group_barrier(kSchedMfma, 1, 0);
                __builtin_amdgcn_sched_group_barrier(kSchedValu, 5, 0);
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) cur[f] = nxt[f];
        }
    }
}

// Per-wave view of the current compute item: wave w works on block pair
// w % 4 of the item, column half w / 4 (the two waves of a pair share a SIMD).
struct WaveJob {
    int f;
    int rblk, cblk, ch;
    int rrow, crow;  // LDS input offsets of the row block and of this wave's column half
    bool active, diag, full;
    unsigned live;   // bit r: sub-block (row half r, this column half) is needed
};

__device__ inline WaveJob make_job(const Task &tk, int f, int wave, int ninput) {
    WaveJob j;
    j.f = f;
    const int pw = wave & 3;
    j.ch = wave >> 2;
    const int rs = pick4(tk.rs, pw);
    const int cs = pick4(tk.cs, pw);
    j.active = rs >= 0;
    j.rblk = j.active ? pick4(tk.blk, rs) : 0;
    j.cblk = j.active ? pick4(tk.blk, cs) : 0;
    j.rrow = (rs < 0 ? 0 : rs) * kBlk;
    j.crow = (cs < 0 ? 0 : cs) * kBlk + 32 * j.ch;
    j.diag = j.active && rs == cs;
    j.live = 0;
    if (j.active) {
        for (int r = 0; r < 2; ++r) {
            const bool ok = j.rblk * kBlk + 32 * r < ninput && j.cblk * kBlk + 32 * j.ch < ninput &&
                            !(j.diag && r == 0 && j.ch == 1);
            if (ok) j.live |= 1u << r;
        }
    }
    j.active = j.live != 0;
    j.full = j.live == 3u;
    return j;
}

// Store a wave's finished 64x32 tile.  32x32 output layout of
// v_mfma_*_32x32: lane l, register v hold row 8*(v/4) + 4*(l/32) + v%4,
// column l%32.  Row i of the packed triangle starts at element i(i+1)/2, so
// with i = i0 + d the element offset is tri(i0) + d*i0 + tri(d) + j: one
// multiply-add per register from per-lane bases (32-bit: a channel holds
// fewer than 2^31 bytes of visibilities).  Interior tiles (every element
// inside the triangle and the array) skip the per-element test.
template <bool CI4>
__device__ __forceinline__ void epilogue(const WaveJob &j, const Acc &acc, int lane, int ninput,
                                         int32_t *__restrict__ out, int overwrite) {
    const int64_t P = (int64_t)ninput * (ninput + 1) / 2;
    uint8_t *obase = (uint8_t *)(out + (int64_t)j.f * P * 2);
    const int g = lane >> 5;
    const int jj = j.cblk * kBlk + 32 * j.ch + (lane & 31);
    const int jmax_tile = j.cblk * kBlk + 32 * j.ch + 31;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (!((j.live >> r) & 1u)) continue;
        const int irow0 = j.rblk * kBlk + 32 * r;  // first row of the sub-block
        const int i0 = irow0 + 4 * g;
        const uint32_t base = (uint32_t)((i0 * (i0 + 1) / 2 + jj) * 8);
        const uint32_t step = (uint32_t)(i0 * 8);
        // every row >= every column and inside the array?
        const bool interior = irow0 >= jmax_tile && irow0 + 31 < ninput;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int d = 8 * (v >> 2) + (v & 3);
            const uint32_t off = base + (uint32_t)d * step + (uint32_t)(d * (d + 1) / 2 * 8);
            int vr = acc.re[r][v];
            int vi = acc.p[r][v] - acc.q[r][v];
            if (CI4) { vr >>= 8; vi >>= 8; }
            const int i = i0 + d;
            if (interior || (i < ninput && jj <= i)) {
                int2 *dst = (int2 *)(obase + off);
                if (!overwrite) {
                    const int2 old = *dst;
                    vr += old.x;
                    vi += old.y;
                }
                *dst = int2{vr, vi};
            }
        }
    }
}

__device__ inline void zero_acc(Acc &acc) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        acc.re[r] = v16i{0};
        acc.p[r] = v16i{0};
        acc.q[r] = v16i{0};
    }
}

// Kernel-wide constants of one launch.
struct Launch {
    const uint8_t *in;
    int64_t t_stride;
    int64_t fstride;
    int nt, nchan, ninput, nitems, total_flat, nb, nst, grid;
};

// DMA producer: walks the same work sequence as the consumer, kRing-1 stages
// ahead.  Per item it holds, for each of this lane's DMA instructions, the
// byte offset of its chunk from the stage's time-row base and (bit ii of
// okmask) whether the chunk lies inside the array.
template <bool CI4>
struct Producer {
    int B, f, item, ps, issued;
    bool valid, straddle;
    int okmask;
    int64_t d_off[kDmaPerWave];
};

// Geometry of DMA instruction ii of DMA wave dw: the stage row this lane
// fetches, and the LDS slot and first input (within the slot) of its chunk.
template <bool CI4>
__device__ __forceinline__ void dma_geom(int dw, int ii, int lane, int &row, int &slot, int &inp) {
    using F = Fmt<CI4>;
    row = (dw * kDmaPerWave + ii) * F::kRowsPerDma + lane / F::kChunks;
    const int c = (lane % F::kChunks) ^ F::swz(row);
    slot = c / F::kChunksPerSlot;
    inp = (c % F::kChunksPerSlot) * F::kInputsPerChunk;
}

template <bool CI4>
__device__ __forceinline__ void prod_item(Producer<CI4> &P, const Launch &L, int dw, int lane) {
    using F = Fmt<CI4>;
    Task tk;
    decode_item(L.nb, P.item, tk);
    P.okmask = 0;
#pragma unroll
    for (int ii = 0; ii < kDmaPerWave; ++ii) {
        int row, slot, inp0;
        dma_geom<CI4>(dw, ii, lane, row, slot, inp0);
        const int blk = pick4(tk.blk, slot);
        const int inp = blk * kBlk + inp0;
        const bool ok = blk >= 0 && inp < L.ninput;
        P.okmask |= ok ? (1 << ii) : 0;
        P.d_off[ii] = (int64_t)P.f * L.fstride + (int64_t)row * L.t_stride + (int64_t)inp * F::kBps;
    }
    // A chunk can run past ninput only in the block holding the last input,
    // and only when ninput is not a multiple of the inputs per chunk.
    const int last = (L.ninput - 1) / kBlk;
    P.straddle = (L.ninput % F::kInputsPerChunk) != 0 &&
                 (tk.blk[0] == last || tk.blk[1] == last || tk.blk[2] == last || tk.blk[3] == last);
}

template <bool CI4>
__device__ __forceinline__ void prod_advance(Producer<CI4> &P, const Launch &L, int dw, int lane) {
    P.valid = false;
    while (P.B < L.total_flat && !(P.valid = flat_item(P.B, L.nitems, L.nchan, P.f, P.item)))
        P.B += L.grid;
    if (P.valid) prod_item(P, L, dw, lane);
}

template <bool CI4>
__device__ __forceinline__ void prod_issue(Producer<CI4> &P, const Launch &L, uint8_t *lds,
                                           uint32_t lds_base, int dw, int lane) {
    using F = Fmt<CI4>;
    const uint8_t *zero = (const uint8_t *)&kZeroChunk;
    const int slot = P.issued % kRing;
    const uint32_t sbase = lds_base + slot * kStageBytes + dw * kDmaPerWave * 1024;
    const int t0 = P.ps * F::kT;
    const uint8_t *rowbase = L.in + (int64_t)t0 * L.t_stride;
    if (!P.straddle && t0 + F::kT <= L.nt) {
        // fast path: every row of the stage exists and no chunk straddles
#pragma unroll
        for (int ii = 0; ii < kDmaPerWave; ++ii)
            dma16(((P.okmask >> ii) & 1) ? rowbase + P.d_off[ii] : zero, sbase + ii * 1024);
    } else {
#pragma unroll
        for (int ii = 0; ii < kDmaPerWave; ++ii) {
            int row, sl, inp0;
            dma_geom<CI4>(dw, ii, lane, row, sl, inp0);
            const int t = t0 + row;
            const int inp = (int)((P.d_off[ii] - (int64_t)P.f * L.fstride - (int64_t)row * L.t_stride) /
                                  F::kBps);
            const bool ok = ((P.okmask >> ii) & 1) && t < L.nt;
            const bool straddle = ok && inp + F::kInputsPerChunk > L.ninput;
            if (!straddle) dma16(ok ? rowbase + P.d_off[ii] : zero, sbase + ii * 1024);
            if (straddle) {
                // chunk runs past the last input: fetch whole 4-byte words
                // (ninput % 4 == 0) and zero-fill the rest.
                const uint8_t *p = rowbase + P.d_off[ii];
                const int nwords = ((L.ninput - inp) * F::kBps) / 4;
                uint32_t w[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) w[k] = k < nwords ? ((const uint32_t *)p)[k] : 0u;
                uint8_t *l = lds + slot * kStageBytes + (dw * kDmaPerWave + ii) * 1024 + lane * 16;
                *(uint4 *)l = uint4{w[0], w[1], w[2], w[3]};
            }
        }
    }
    ++P.issued;
    if (++P.ps == L.nst) {
        P.ps = 0;
        P.B += L.grid;
        prod_advance(P, L, dw, lane);
    }
}

// Advance the producer cursor without loading (waves 4..7): keeps the
// workgroup-wide synchronisation inside prod_item in step.
template <bool CI4>
__device__ __forceinline__ void prod_skip(Producer<CI4> &P, const Launch &L, int dw, int lane) {
    ++P.issued;
    if (++P.ps == L.nst) {
        P.ps = 0;
        P.B += L.grid;
        prod_advance(P, L, dw, lane);
    }
}

template <bool CI4>
__global__ __launch_bounds__(kThreads, 1) void xengine_int_kernel(
    const uint8_t *__restrict__ in, int64_t t_stride, int nt, int nchan, int ninput, int nitems,
    int total_flat, int32_t *__restrict__ out, int overwrite) {
    using F = Fmt<CI4>;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int lane = tid & 63;
    const int dw = wave;  // every wave issues kDmaPerWave of each stage's DMA
    Launch L;
    L.in = in;
    L.t_stride = t_stride;
    L.fstride = (int64_t)ninput * F::kBps;
    L.nt = nt;
    L.nchan = nchan;
    L.ninput = ninput;
    L.nitems = nitems;
    L.total_flat = total_flat;
    L.nb = (ninput + kBlk - 1) / kBlk;
    L.nst = (nt + F::kT - 1) / F::kT;
    L.grid = gridDim.x;

    // ---- consumer cursor (drives the loop of every wave)
    int cB = blockIdx.x, cf = 0, citem = 0;
    bool cvalid = false;
    while (cB < total_flat && !(cvalid = flat_item(cB, nitems, nchan, cf, citem))) cB += L.grid;
    if (!cvalid) return;  // no work for this workgroup

    // ---- producer cursor (every wave issues its share of each stage)
    Producer<CI4> P;
    P.B = blockIdx.x;
    P.ps = 0;
    P.issued = 0;
    prod_advance(P, L, dw, lane);

    WaveJob job;
    int fb[3];
    {
        Task tk;
        decode_item(L.nb, citem, tk);
        job = make_job(tk, cf, wave, ninput);
        fb[0] = frag_base<CI4>(job.rrow, lane);
        fb[1] = frag_base<CI4>(job.rrow + 32, lane);
        fb[2] = frag_base<CI4>(job.crow, lane);
    }

    Acc acc;
    zero_acc(acc);

    for (int k = 0; k < kRing - 1 && P.valid; ++k) prod_issue(P, L, lds, lds_base, dw, lane);

    int consumed = 0;
    int cs = 0;
    bool after_epilogue = false;
    while (true) {
        // Stage `consumed` must have landed in LDS: each wave waits for its
        // own loads, then the barrier publishes them to every wave.  The
        // counter is in order for loads, but the epilogue's stores share it
        // and may complete out of order with them, so the first wait after
        // an epilogue (and the tail of the sequence) waits for everything.
        if (after_epilogue) wait_vm<0>();
        else wait_stage(P.issued - consumed - 1);
        block_barrier();
        if (P.valid) prod_issue(P, L, lds, lds_base, dw, lane);  // refills the slot read last

        const uint8_t *stage = lds + (consumed % kRing) * kStageBytes;
        if (job.active) mfma_stage<CI4>(stage, fb, acc);
        ++consumed;
        after_epilogue = false;
        if (++cs == L.nst) {
            if (job.active) epilogue<CI4>(job, acc, lane, ninput, out, overwrite);
            zero_acc(acc);
            cs = 0;
            cvalid = false;
            cB += L.grid;
            while (cB < total_flat && !(cvalid = flat_item(cB, nitems, nchan, cf, citem))) cB += L.grid;
            if (!cvalid) break;
            Task tk;
            decode_item(L.nb, citem, tk);
            job = make_job(tk, cf, wave, ninput);
            fb[0] = frag_base<CI4>(job.rrow, lane);
            fb[1] = frag_base<CI4>(job.rrow + 32, lane);
            fb[2] = frag_base<CI4>(job.crow, lane);
            after_epilogue = true;
        }
    }
    wait_vm<0>();  // no DMA may still target LDS when the workgroup retires
}

int g_num_cus = 0;
std::once_flag g_init_once;
hipError_t g_init_err = hipSuccess;

void init_once() {
    int dev = 0;
    g_init_err = hipGetDevice(&dev);
    if (g_init_err != hipSuccess) return;
    hipDeviceProp_t prop;
    g_init_err = hipGetDeviceProperties(&prop, dev);
    if (g_init_err != hipSuccess) return;
    g_num_cus = prop.multiProcessorCount;
    g_init_err = hipFuncSetAttribute((const void *)xengine_int_kernel<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (g_init_err != hipSuccess) return;
    g_init_err = hipFuncSetAttribute((const void *)xengine_int_kernel<false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
}

}  // namespace

int xengine_tri_items(int32_t ninput) { return tri_items((ninput + kBlk - 1) / kBlk); }

hipError_t launch_xengine_int(bool ci4, const void *in, int64_t nt, int32_t nchan, int32_t ninput,
                              int32_t *out, bool overwrite, hipStream_t s) {
    std::call_once(g_init_once, init_once);
    if (g_init_err != hipSuccess) return g_init_err;
    const int nb = (ninput + kBlk - 1) / kBlk;
    const int nitems = tri_items(nb);
    const int64_t nchan8 = ((int64_t)nchan + 7) / 8 * 8;
    const int64_t total_flat = nchan8 * nitems;
    int64_t grid = (int64_t)(g_num_cus > 0 ? g_num_cus : 256) / 8 * 8;
    if (grid < 8) grid = 8;
    if (grid > total_flat) grid = total_flat;  // total_flat is a multiple of 8
    const int64_t t_stride = (int64_t)nchan * ninput * (ci4 ? 1 : 2);
    if (ci4)
        hipLaunchKernelGGL(xengine_int_kernel<true>, dim3((unsigned)grid), dim3(kThreads),
                           kLdsBytes, s, (const uint8_t *)in, t_stride, (int)nt, nchan, ninput,
                           nitems, (int)total_flat, out, (int)overwrite);
    else
        hipLaunchKernelGGL(xengine_int_kernel<false>, dim3((unsigned)grid), dim3(kThreads),
                           kLdsBytes, s, (const uint8_t *)in, t_stride, (int)nt, nchan, ninput,
                           nitems, (int)total_flat, out, (int)overwrite);
    return hipGetLastError();
}

}  // namespace bfx
