// Shared machinery of the X-engine kernels (integer and binary16): work
// decomposition of the lower triangle, the LDS stage ring fed by direct
// global->LDS DMA, and the persistent producer/consumer loop.  The element
// arithmetic (fragment reads, MFMA, epilogue) is supplied by a consumer
// policy per input format.
//
// Work decomposition.  Inputs are grouped in blocks of 64.  One workgroup
// (8 waves, two per SIMD) holds up to four input blocks of one channel in LDS
// and produces up to four 64x64 block pairs (I >= J) of the triangle, each
// split between two waves (64 rows x 32 columns each).  The block pairs of a
// channel are packed into work items in closed form (decode_item): 2x2
// super-tiles below the diagonal, diagonal super-tiles that borrow a pair from
// the odd last block row, and the rest of that row in groups of three.  The
// grid is persistent (one workgroup per CU); workgroup b walks the flat work
// ids b, b + grid, ...; a work source maps a flat id to (channel, item).
//
// Data path.  A ring of kRing LDS stages of 16 KiB receives raw time rows of
// the four blocks (256 inputs) straight from HBM with global_load_lds_dwordx4
// (no staging registers), kRing-1 stages ahead of the MFMA work and across
// work-item boundaries; one wave per SIMD issues four of each stage's 16 DMA
// instructions and waits on its own vector-memory counter before the stage
// barrier.  Each row's 16-byte chunks are XOR-swizzled by the row index so the
// consumers' transposing LDS reads are free of bank conflicts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfx {
namespace {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) v2i lds_v2i;
typedef __attribute__((address_space(3))) v4s lds_v4s;

constexpr int kBlk = 64;          // inputs per block / LDS slot
constexpr int kSlots = 4;         // input blocks held per work item
constexpr int kStageBytes = 16384;
constexpr int kRing = 8;          // LDS stages in flight (128 KiB)
constexpr int kRingBytes = kRing * kStageBytes;
// The ring plus 1 KiB that receives the dummy DMA of a chunk fetched by the
// synchronous path (keeps every stage at exactly its DMA operation count
// per wave, which the vmcnt waits count on).
// Then the task table of a single array's items (see SingleArray): 8 bytes
// per item, at most tri_items(128) items (8192 inputs).
constexpr int kTaskTabEntries = 2080;
constexpr int kTaskTabOff = kRingBytes + 1024;
constexpr int kLdsBytes = kTaskTabOff + kTaskTabEntries * 8;
// Each of NW DMA waves issues an equal share of each stage's DMA
// (16-byte-per-lane instructions, 1 KiB each).
template <int NW>
constexpr int dma_per_wave() { return kStageBytes / 1024 / NW; }

// Layout of one LDS stage: kT time rows of 256 inputs of BPS bytes each
// (1: ci4, 2: ci8, 4: cf16).
template <int BPS>
struct RowFmt {
    static constexpr int kBps = BPS;                    // bytes per sample
    static constexpr int kRow = kSlots * kBlk * kBps;   // bytes per time row
    static constexpr int kT = kStageBytes / kRow;       // time rows per stage (64 / 32 / 16)
    static constexpr int kChunks = kRow / 16;           // 16-byte chunks per row
    static constexpr int kChunksPerSlot = kChunks / kSlots;
    static constexpr int kInputsPerChunk = 16 / kBps;
    static constexpr int kRowsPerDma = 1024 / kRow;     // rows covered by one wave DMA
    static_assert(kRowsPerDma >= 1, "a wave DMA must cover whole rows");
    // XOR swizzle of the 16-byte chunks of row t.  A transposing read touches
    // rows t0..t0+7 (ds_read_b64_tr_b8) or t0..t0+3 (ds_read_b64_tr_b16) of
    // adjacent chunks per 16-lane group; these swizzles map the chunks read
    // by a 32-lane half to distinct bank groups.
    __device__ static inline int swz(int t) { return BPS == 1 ? ((t & 7) << 1) : ((t & 3) << 2); }
};

struct Task {
    int blk[kSlots];   // input block held by each LDS slot, -1 = unused
    int chan[kSlots];  // channel of each LDS slot, relative to the item's first
    int rs[4];         // per block pair: LDS slot of its row block, -1 = unused
    int cs[4];         // per block pair: LDS slot of its column block
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
    for (int k = 0; k < 4; ++k) { tk.blk[k] = -1; tk.chan[k] = 0; tk.rs[k] = -1; tk.cs[k] = -1; }
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

// Compact form of a triangle item's task (every slot in channel 0): the input
// block of each slot as a signed byte, and the row and column slot of each
// pair as 4-bit two's-complement fields (-1 = unused).
__device__ inline uint2 pack_task(const Task &tk) {
    uint32_t b = 0, s = 0;
    for (int k = 0; k < 4; ++k) {
        b |= (uint32_t)(tk.blk[k] & 0xFF) << (8 * k);
        s |= ((uint32_t)(tk.rs[k] & 15) << (4 * k)) | ((uint32_t)(tk.cs[k] & 15) << (16 + 4 * k));
    }
    return uint2{b, s};
}

__device__ __forceinline__ void unpack_task(uint32_t b, uint32_t s, Task &tk) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        tk.blk[k] = (int)(b << (24 - 8 * k)) >> 24;
        tk.rs[k] = (int)(s << (28 - 4 * k)) >> 28;
        tk.cs[k] = (int)(s << (12 - 4 * k)) >> 28;
        tk.chan[k] = 0;
    }
}

// A packed item: npack (1..4) channels of a one-block array (<= 64 inputs),
// channel k in LDS slot k, block pairs (k, k) -- so small arrays fill all four
// pair slots of a work item instead of one.
__device__ inline void decode_packed(int npack, Task &tk) {
    for (int k = 0; k < 4; ++k) {
        const bool on = k < npack;
        tk.blk[k] = on ? 0 : -1;
        tk.chan[k] = k;
        tk.rs[k] = on ? k : -1;
        tk.cs[k] = on ? k : -1;
    }
}

// Select element k of a 4-element task array without dynamic indexing (which
// would place the array in scratch or LDS).  For a wave-uniform k.
__device__ inline int pick4(const int (&a)[4], int k) {
    return k == 0 ? a[0] : k == 1 ? a[1] : k == 2 ? a[2] : a[3];
}

// The same for a per-lane k, in bit operations only: a chain of conditional
// selects here is turned into divergent branches by the compiler.
__device__ inline int lane_pick4(const int (&a)[4], int k) {
    const int m1 = -(k & 1), m2 = -((k >> 1) & 1);
    const int lo = a[0] ^ ((a[0] ^ a[1]) & m1);
    const int hi = a[2] ^ ((a[2] ^ a[3]) & m1);
    return lo ^ ((lo ^ hi) & m2);
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

__device__ inline void block_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ const uint4 kZeroChunk = {0u, 0u, 0u, 0u};

// Scheduling masks of __builtin_amdgcn_sched_group_barrier.
constexpr int kSchedValu = 0x2;
constexpr int kSchedMfma = 0x8;

// Per-wave view of the current compute item: one block pair of the item
// (row block rblk, column block cblk), or one 32-column half of it.
struct WaveJob {
    int rblk, cblk, ch;
    int ochan;       // channel of the pair, relative to the item's first
    int rrow, crow;  // LDS input offsets of the row block and of this wave's columns
    bool active, diag;
    unsigned live;   // bit 2*r + c: 32x32 sub-block (row half r, column half c) is needed
};

__device__ inline void job_common(const Task &tk, int pair, int ch, WaveJob &j) {
    const int rs = pick4(tk.rs, pair);
    const int cs = pick4(tk.cs, pair);
    j.ch = ch;
    j.active = rs >= 0;
    j.rblk = j.active ? pick4(tk.blk, rs) : 0;
    j.cblk = j.active ? pick4(tk.blk, cs) : 0;
    j.ochan = j.active ? pick4(tk.chan, rs) : 0;
    j.rrow = (rs < 0 ? 0 : rs) * kBlk;
    j.crow = (cs < 0 ? 0 : cs) * kBlk + 32 * ch;
    j.diag = j.active && rs == cs;
}

// Sub-block (r, c) of a pair holds a needed output: inside the array and not
// entirely above the diagonal of a diagonal pair.
__device__ inline bool sub_live(const WaveJob &j, int r, int c, int ninput) {
    return j.rblk * kBlk + 32 * r < ninput && j.cblk * kBlk + 32 * c < ninput &&
           !(j.diag && r < c);
}

// Eight waves: wave w works on block pair w % 4, column half w / 4 (the two
// waves of a pair share a SIMD).  live bits 2*r + ch.
__device__ inline WaveJob make_job_half(const Task &tk, int wave, int ninput) {
    WaveJob j;
    job_common(tk, wave & 3, wave >> 2, j);
    j.live = 0;
    if (j.active)
        for (int r = 0; r < 2; ++r)
            if (sub_live(j, r, j.ch, ninput)) j.live |= 1u << (2 * r + j.ch);
    j.active = j.live != 0;
    return j;
}

// Four waves: wave w works on the whole block pair w.
__device__ inline WaveJob make_job_pair(const Task &tk, int wave, int ninput) {
    WaveJob j;
    job_common(tk, wave, 0, j);
    j.live = 0;
    if (j.active)
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c)
                if (sub_live(j, r, c, ninput)) j.live |= 1u << (2 * r + c);
    j.active = j.live != 0;
    return j;
}

// One work item as the producer and the consumer see it.
struct Item {
    const uint8_t *base;     // time row 0, input 0 of the item's (first) channel
    int64_t t_stride;        // bytes between time rows
    int64_t chan_bytes;      // bytes of one channel in a time row (ninput * sample bytes)
    int64_t out_chan_bytes;  // bytes of one channel's packed visibilities
    void *out;               // the (first) channel's visibilities
    int ninput, nb, item;
    int npack;               // 0: triangle item `item` of one channel; 1..4: packed item
};

__device__ inline void decode_task(const Item &it, Task &tk) {
    if (it.npack) decode_packed(it.npack, tk);
    else decode_item(it.nb, it.item, tk);
}

// The task of an item, from the work source's table in LDS when it keeps one
// (a wave-uniform LDS read instead of the closed-form decode).
template <class W>
__device__ __forceinline__ void task_of(const Item &it, const uint2 *tab, Task &tk) {
    if constexpr (W::kTable) {
        if (it.npack) {
            decode_packed(it.npack, tk);
        } else {
            const uint2 e = tab[it.item];
            unpack_task(__builtin_amdgcn_readfirstlane(e.x), __builtin_amdgcn_readfirstlane(e.y), tk);
        }
    } else {
        decode_task(it, tk);
    }
}

// Work source of a single array.  Flat id B maps to channel group g with
// B % 8 == g % 8, so with round-robin dispatch over the 8 XCDs all items of a
// channel run on one XCD and share its L2.  A group is one channel, or four
// channels packed into one item when the array has a single input block.
// Padding ids of a group count that is not a multiple of 8 return false.
struct SingleArray {
    // The tasks of a channel's items are decoded once per workgroup into an
    // LDS table (a one-block array's packed items need none).
    static constexpr bool kTable = true;
    __device__ __forceinline__ void fill_table(uint2 *tab, int tid, int nthreads) const {
        if (npk > 1) return;
        for (int i = tid; i < nitems; i += nthreads) {
            Task tk;
            decode_item(nb, i, tk);
            tab[i] = pack_task(tk);
        }
    }
    const uint8_t *in;
    void *out;
    int64_t t_stride;
    int64_t out_chan_bytes;  // bytes of one channel's visibilities
    int nchan, ninput, nitems, nb, bps;
    int npk;      // channels per group: 4 when nb == 1, else 1
    int ngroups;  // ceil(nchan / npk)

    __device__ __forceinline__ bool get(int B, Item &it) const {
        const int s = B >> 3;
        const int cl = s / nitems;
        it.item = s - cl * nitems;
        const int g = cl * 8 + (B & 7);
        const int f0 = g * npk;
        it.npack = npk > 1 ? min(npk, nchan - f0) : 0;
        it.chan_bytes = (int64_t)ninput * bps;
        it.base = in + (int64_t)f0 * it.chan_bytes;
        it.t_stride = t_stride;
        it.out_chan_bytes = out_chan_bytes;
        it.out = (uint8_t *)out + (int64_t)f0 * out_chan_bytes;
        it.ninput = ninput;
        it.nb = nb;
        return g < ngroups;
    }
};

// DMA producer: walks the same work sequence as the consumer, kRing-1 stages
// ahead.  Per item it holds, for each of this lane's DMA instructions, the
// byte offset of its chunk from the item's time-row base and (bit ii of
// okmask) whether the chunk lies inside the array.
template <int DPW>
struct Producer {
    int B, ps;
    unsigned issued;       // stages issued so far (real or dummy)
    bool valid, straddle;
    int okmask;
    Item it;
    const uint8_t *row;    // time row of the next stage of the current item
    const uint8_t *zero;   // a 16-byte zero chunk
    int64_t d_off[DPW];
    int inp[DPW];          // first input of each chunk within its channel
};

// Geometry of DMA instruction ii of DMA wave dw: the stage row this lane
// fetches, and the LDS slot and first input (within the slot) of its chunk.
template <class F, int DPW>
__device__ __forceinline__ void dma_geom(int dw, int ii, int lane, int &row, int &slot, int &inp) {
    row = (dw * DPW + ii) * F::kRowsPerDma + lane / F::kChunks;
    const int c = (lane % F::kChunks) ^ F::swz(row);
    slot = c / F::kChunksPerSlot;
    inp = (c % F::kChunksPerSlot) * F::kInputsPerChunk;
}

template <class F, int DPW, class W>
__device__ __forceinline__ void prod_item(Producer<DPW> &P, const uint2 *tab, int dw, int lane) {
    Task tk;
    task_of<W>(P.it, tab, tk);
    P.okmask = 0;
#pragma unroll
    for (int ii = 0; ii < DPW; ++ii) {
        int row, slot, inp0;
        dma_geom<F, DPW>(dw, ii, lane, row, slot, inp0);
        const int blk = lane_pick4(tk.blk, slot);
        const int inp = blk * kBlk + inp0;
        const bool ok = blk >= 0 && inp < P.it.ninput;
        P.okmask |= ok ? (1 << ii) : 0;
        // A chunk outside the array (an unused slot, or inputs past ninput)
        // fetches input 0 of the same row instead: such LDS inputs only feed
        // outputs that are never stored (every output depends on its own two
        // inputs alone), so no zero fill is needed -- except past the last
        // time row, which the slow path zero-fills.  The offset is masked,
        // not selected, so that no lane takes a branch.
        const int64_t off = (int64_t)lane_pick4(tk.chan, slot) * P.it.chan_bytes + (int64_t)inp * F::kBps;
        P.d_off[ii] = (int64_t)row * P.it.t_stride + (off & -(int64_t)ok);
        P.inp[ii] = inp;
    }
    P.row = P.it.base;
    // A chunk can run past ninput only in the block holding the last input,
    // and only when ninput is not a multiple of the inputs per chunk.
    const int last = (P.it.ninput - 1) / kBlk;
    P.straddle = (P.it.ninput % F::kInputsPerChunk) != 0 &&
                 (tk.blk[0] == last || tk.blk[1] == last || tk.blk[2] == last || tk.blk[3] == last);
}

template <class F, int DPW, class W>
__device__ __forceinline__ void prod_advance(Producer<DPW> &P, const W &w, const uint2 *tab, int total_flat,
                                             int grid, int dw, int lane) {
    P.valid = false;
    while (P.B < total_flat && !(P.valid = w.get(P.B, P.it))) P.B += grid;
    if (P.valid) prod_item<F, DPW, W>(P, tab, dw, lane);
}

// Issue the next stage's DMA into ring slot issued % kRing.  Past the end of
// the work sequence the producer keeps issuing a dummy stage (zero chunks into
// the slot just consumed), so that exactly kRing - 2 stages are always in
// flight after the awaited one and every wait is the same constant.
template <class F, int DPW, class W>
__device__ __forceinline__ void prod_issue(Producer<DPW> &P, const W &w, const uint2 *tab, int nt, int nst,
                                           int total_flat, int grid, uint8_t *lds, uint32_t lds_base,
                                           int dw, int lane) {
    const unsigned slot = P.issued & (kRing - 1);
    const uint32_t sbase = lds_base + slot * kStageBytes + dw * DPW * 1024;
    ++P.issued;
    if (!P.valid) {
#pragma unroll
        for (int ii = 0; ii < DPW; ++ii) dma16(P.zero, sbase + ii * 1024);
        return;
    }
    const uint8_t *rowbase = P.row;
    const int t0 = P.ps * F::kT;
    if (!P.straddle && t0 + F::kT <= nt) {
        // fast path: every row of the stage exists and no chunk straddles
#pragma unroll
        for (int ii = 0; ii < DPW; ++ii) dma16(rowbase + P.d_off[ii], sbase + ii * 1024);
    } else {
#pragma unroll
        for (int ii = 0; ii < DPW; ++ii) {
            int row, sl, inp0;
            dma_geom<F, DPW>(dw, ii, lane, row, sl, inp0);
            const int t = t0 + row;
            const int inp = P.inp[ii];
            const bool ok = ((P.okmask >> ii) & 1) && t < nt;
            const bool straddle = ok && inp + F::kInputsPerChunk > P.it.ninput;
            if (!straddle) dma16(ok ? rowbase + P.d_off[ii] : P.zero, sbase + ii * 1024);
            if (straddle) {
                // chunk runs past the last input (possibly the end of the
                // buffer): fetch whole 4-byte words (ninput % 4 == 0) and
                // zero-fill the rest; a DMA of the zero chunk into the spare
                // kilobyte keeps the per-stage count.
                dma16(P.zero, lds_base + kRingBytes);
                const uint8_t *p = rowbase + P.d_off[ii];
                const int nwords = ((P.it.ninput - inp) * F::kBps) / 4;
                uint32_t wd[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) wd[k] = k < nwords ? ((const uint32_t *)p)[k] : 0u;
                uint8_t *l = lds + slot * kStageBytes + (dw * DPW + ii) * 1024 + lane * 16;
                *(uint4 *)l = uint4{wd[0], wd[1], wd[2], wd[3]};
            }
        }
    }
    P.row += (int64_t)F::kT * P.it.t_stride;
    if (++P.ps == nst) {
        P.ps = 0;
        P.B += grid;
        prod_advance<F, DPW>(P, w, tab, total_flat, grid, dw, lane);
    }
}

// Wait until this wave's LDS reads have returned (lgkmcnt = 0; vmcnt and
// expcnt left at their maxima).
__device__ inline void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// The persistent loop shared by every X-engine kernel, software-pipelined
// across stages.  F is the LDS row format, C the consumer policy:
//   C::kWaves (waves per workgroup), C::job(task, wave, ninput);
//   C::Acc, C::Raw (a stage's transposing-read results), C::Pre (operands of
//   a stage's first MFMA step, formed ahead), C::Bases;
//   C::zero(acc);  C::bind(job, lane, bases);
//   C::read(stage_ptr, bases, raw)  -- issue the stage's transposing LDS reads;
//   C::prep(raw, pre)               -- form pre from raw;
//   C::head(pre, raw, acc)          -- the stage's first MFMAs, from pre;
//   C::tail(pre, raw, nraw, npre, acc) -- the rest of the stage's MFMAs, and
//                                      npre from the next stage's nraw;
//   C::epilogue(job, it, acc, lane, overwrite).
// Iteration s: every DMA wave waits for its own DMA of stage s+1, the
// barrier publishes it, and the MFMAs of stage s start at once from operands
// already in registers.  Behind the first of them the ring slot of stage s
// (read completely by every wave before the barrier) is refilled and the
// reads of stage s+1 are issued; the remaining MFMAs of stage s then cover
// those reads and the forming of stage s+1's first operands.  Only the first
// kDmaWaves waves issue DMA.  With four (one per SIMD) the other wave of each
// SIMD goes straight on to its MFMAs while its partner does the producer's
// work; with eight every wave takes a smaller share.  Which is faster depends
// on the shape, so the plan picks (see the autotuner in the host API).  At an item's last stage the
// next item's job is decoded first, so its first stage is read under the same
// overlap.  The loop body runs twice per trip with the two register sets
// swapped, so no operand is copied.
// The vector-memory counter also counts the epilogue's stores, and it counts
// down in issue order (the compiler's own waits rely on that).  A wait for
// "at most N outstanding", N = the DMA loads issued after the awaited stage,
// is therefore safe whatever the stores do: while the awaited DMA is
// outstanding so is every later load, so at least N + 1 operations are.
// Stores issued after the awaited stage lengthen the wait; counting them in
// as well was timed and gained nothing, so the wait stays a constant.  Waves
// that issue no DMA do not wait on the counter at all.
template <class F, class C, int DMA_WAVES, class W>
__device__ __forceinline__ void xe_loop(const W &w, int nt, int total_flat, int overwrite) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int lane = tid & 63;
    constexpr int kDmaWaves = DMA_WAVES;
    static_assert(C::kWaves % kDmaWaves == 0, "DMA waves spread over the SIMDs");
    const bool dma_wave = wave < kDmaWaves;
    const int dw = wave;  // DMA waves issue DPW of each stage's DMA each
    constexpr int DPW = dma_per_wave<kDmaWaves>();
    const int grid = gridDim.x;
    const int nst = (nt + F::kT - 1) / F::kT;
    uint2 *tab = (uint2 *)(lds + kTaskTabOff);
    if constexpr (W::kTable) {
        w.fill_table(tab, tid, C::kThreads);
        wait_lds();  // the table's LDS writes have landed
        block_barrier();
    }

    // ---- consumer cursor (drives the loop of every wave)
    int cB = blockIdx.x;
    Item cit;
    bool cvalid = false;
    while (cB < total_flat && !(cvalid = w.get(cB, cit))) cB += grid;
    if (!cvalid) return;  // no work for this workgroup

    // ---- producer cursor (every wave issues its share of each stage)
    Producer<DPW> P;
    P.B = blockIdx.x;
    P.ps = 0;
    P.issued = 0;
    P.zero = (const uint8_t *)&kZeroChunk;
    if (dma_wave) prod_advance<F, DPW>(P, w, tab, total_flat, grid, dw, lane);

    WaveJob job;
    typename C::Bases fb;
    {
        Task tk;
        task_of<W>(cit, tab, tk);
        job = C::job(tk, wave, cit.ninput);
        C::bind(job, lane, fb);
    }

    typename C::Acc acc;
    C::zero(acc);
    // Both register sets are defined on every path (zeroed here, then read
    // unconditionally while work remains -- an inactive wave's bases still
    // point inside the stage).
    typename C::Raw ra = {}, rb = {};
    typename C::Pre pa = {}, pb = {};

    constexpr int kAhead = (kRing - 2) * DPW;  // DMA operations after the awaited stage
    static_assert(kAhead + DPW < 64, "vmcnt range");
    if (dma_wave)
        for (int k = 0; k < kRing - 1; ++k)
            prod_issue<F, DPW>(P, w, tab, nt, nst, total_flat, grid, lds, lds_base, dw, lane);
    if (dma_wave) wait_vm<kAhead>();
    wait_lds();  // and any LDS stores of the synchronous (zero-fill) path
    block_barrier();
    if (dma_wave) prod_issue<F, DPW>(P, w, tab, nt, nst, total_flat, grid, lds, lds_base, dw, lane);
    C::read(lds, fb, ra);
    wait_lds();
    C::prep(ra, pa);

    unsigned s = 0;  // stage whose MFMA work the next step does
    int cs = 0;      // its index within the current item
    // One stage: MFMAs of stage s from (cur, pcur); reads of stage s+1 into
    // nxt and its first operands into pnxt.  Returns whether work remains.
    auto step = [&](typename C::Raw &cur, typename C::Pre &pcur, typename C::Raw &nxt,
                    typename C::Pre &pnxt) __attribute__((always_inline)) {
        const bool last = cs + 1 == nst;
        WaveJob njob = job;
        typename C::Bases nfb = fb;
        Item nit = cit;
        bool more = true;
        if (last) {
            cB += grid;
            more = false;
            while (cB < total_flat && !(more = w.get(cB, nit))) cB += grid;
            if (more) {
                Task tk;
                task_of<W>(nit, tab, tk);
                njob = C::job(tk, wave, nit.ninput);
                C::bind(njob, lane, nfb);
            }
        }
        if (more) {
            // every read of stage s has returned: its slot may be refilled
            wait_lds();
            if (dma_wave) wait_vm<kAhead>();
            block_barrier();
        }
        C::head(pcur, cur, acc);
        __builtin_amdgcn_sched_barrier(0);
        if (more) {
            if (dma_wave) prod_issue<F, DPW>(P, w, tab, nt, nst, total_flat, grid, lds, lds_base, dw, lane);
            C::read(lds + ((s + 1) & (kRing - 1)) * kStageBytes, nfb, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);
        C::tail(pcur, cur, nxt, pnxt, acc);
        if (last) {
            if (job.active) C::epilogue(job, cit, acc, lane, overwrite);
            C::zero(acc);
            job = njob;
            fb = nfb;
            cit = nit;
        }
        cs = last ? 0 : cs + 1;
        ++s;
        return more;
    };
    while (step(ra, pa, rb, pb) && step(rb, pb, ra, pa)) {
    }
    wait_vm<0>();  // no DMA may still target LDS when the workgroup retires
}

// A work source that decodes every task in closed form (no LDS table).
template <class W>
struct ClosedForm : W {
    static constexpr bool kTable = false;
    __device__ explicit ClosedForm(const W &w) : W(w) {}
};

// Wait until at most N of this wave's LDS operations are in flight (vmcnt and
// expcnt left at their maxima).
template <int N>
__device__ inline void wait_lgkm() {
    static_assert(N >= 0 && N < 16, "lgkmcnt range");
    __builtin_amdgcn_s_waitcnt(0xC07F | (N << 8));
}

// The same persistent loop with each stage's transposing reads issued two
// stages ahead, for a consumer whose MFMA operands are the reads themselves
// (C::Pre empty; C::kLdsReads LDS instructions per stage).  Iteration s: the
// reads of stage s+1 are in flight; every wave waits for its reads of stage s
// only, the DMA waves for their DMA of stage s+2, and the barrier publishes
// stage s+2 and frees the slot of stage s.  The MFMAs of stage s then start,
// the slot is refilled, and the reads of stage s+2 go out behind them, so a
// stage's reads have two stages of MFMA work to return in.  Three register
// sets rotate.  A read cursor runs two stages ahead of the MFMA work and
// decodes each next item (in closed form: an LDS table read would wait for
// the reads in flight); the MFMA side takes the item over at its last stage.
// Items must have at least two stages (the host launches this loop only
// then), so the read cursor is at most one item ahead.
template <class F, class C, int DMA_WAVES, class W0>
__device__ __forceinline__ void xe_loop_ra2(const W0 &w0, int nt, int total_flat, int overwrite) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;
    typedef ClosedForm<W0> W;
    const W w(w0);

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int lane = tid & 63;
    constexpr int kDmaWaves = DMA_WAVES;
    static_assert(C::kWaves % kDmaWaves == 0, "DMA waves spread over the SIMDs");
    const bool dma_wave = wave < kDmaWaves;
    const int dw = wave;
    constexpr int DPW = dma_per_wave<kDmaWaves>();
    const int grid = gridDim.x;
    const int nst = (nt + F::kT - 1) / F::kT;
    const uint2 *tab = nullptr;  // (closed-form decode)

    // ---- the MFMA side's item
    int cB = blockIdx.x;
    Item cit;
    bool cvalid = false;
    while (cB < total_flat && !(cvalid = w.get(cB, cit))) cB += grid;
    if (!cvalid) return;  // no work for this workgroup

    // ---- producer cursor
    Producer<DPW> P;
    P.B = blockIdx.x;
    P.ps = 0;
    P.issued = 0;
    P.zero = (const uint8_t *)&kZeroChunk;
    if (dma_wave) prod_advance<F, DPW>(P, w, tab, total_flat, grid, dw, lane);

    WaveJob job;
    typename C::Bases rfb;  // bases of the stage the read cursor reads next
    {
        Task tk;
        decode_task(cit, tk);
        job = C::job(tk, wave, cit.ninput);
        C::bind(job, lane, rfb);
    }
    // ---- read cursor: flat id, stage within its item; the item it moved on
    // to last, for the MFMA side (pvalid: there is one)
    int rB = cB, rcs = 0;
    bool rvalid = true, pvalid = false;
    WaveJob pjob = job;
    Item pit = cit;
    auto radvance = [&]() __attribute__((always_inline)) {
        if (++rcs < nst) return;
        rcs = 0;
        rB += grid;
        Item nit = cit;
        bool v = false;
        while (rB < total_flat && !(v = w.get(rB, nit))) rB += grid;
        rvalid = v;
        pvalid = v;
        if (v) {
            Task tk;
            decode_task(nit, tk);
            pjob = C::job(tk, wave, nit.ninput);
            C::bind(pjob, lane, rfb);
            pit = nit;
        }
    };

    typename C::Acc acc;
    C::zero(acc);
    typename C::Raw ra = {}, rb = {}, rc = {};
    typename C::Pre pre = {};

    constexpr int kAhead2 = (kRing - 3) * DPW;  // DMA operations after the stage two ahead
    if (dma_wave)
        for (int k = 0; k < kRing - 1; ++k)
            prod_issue<F, DPW>(P, w, tab, nt, nst, total_flat, grid, lds, lds_base, dw, lane);
    if (dma_wave) wait_vm<kAhead2>();  // stages 0 and 1 have landed
    wait_lds();
    block_barrier();
    if (dma_wave) prod_issue<F, DPW>(P, w, tab, nt, nst, total_flat, grid, lds, lds_base, dw, lane);
    C::read(lds, rfb, ra);
    radvance();
    C::read(lds + kStageBytes, rfb, rb);
    radvance();

    unsigned s = 0;  // stage whose MFMA work the next step does
    int cs = 0;      // its index within the MFMA side's item
    // One stage: MFMAs of stage s from cur; reads of stage s+2 into nxt.
    // Returns whether a stage follows.
    auto step = [&](typename C::Raw &cur, typename C::Raw &nxt) __attribute__((always_inline)) {
        const bool last = cs + 1 == nst;
        const bool more = !last || pvalid;
        const bool rd = rvalid;  // stage s+2 exists
        if (rd) {
            // this wave's reads of stage s are back (those of stage s+1 may
            // not be): its slot may be refilled once every wave is here
            wait_lgkm<C::kLdsReads>();
            if (dma_wave) wait_vm<kAhead2>();
            block_barrier();
        }
        C::head(pre, cur, acc);
        __builtin_amdgcn_sched_barrier(0);
        if (rd) {
            if (dma_wave) prod_issue<F, DPW>(P, w, tab, nt, nst, total_flat, grid, lds, lds_base, dw, lane);
            C::read(lds + ((s + 2) & (kRing - 1)) * kStageBytes, rfb, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);
        C::tail(pre, cur, nxt, pre, acc);
        if (last) {
            if (job.active) C::epilogue(job, cit, acc, lane, overwrite);
            C::zero(acc);
            job = pjob;
            cit = pit;
        }
        cs = last ? 0 : cs + 1;
        if (rd) radvance();
        ++s;
        return more;
    };
    while (step(ra, rc) && step(rb, ra) && step(rc, rb)) {
    }
    wait_vm<0>();  // no DMA may still target LDS when the workgroup retires
}

// Persistent grid: one workgroup per CU, a multiple of 8 (the XCD count) and
// at most the number of flat ids.
inline int64_t persistent_grid(int num_cus, int64_t total_flat) {
    int64_t grid = (int64_t)(num_cus > 0 ? num_cus : 256) / 8 * 8;
    if (grid < 8) grid = 8;
    if (grid > total_flat) grid = total_flat;
    return grid;
}

}  // namespace
}  // namespace bfx
