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
// (4 waves) stages up to four input blocks of one channel through LDS and each
// wave produces one 64x64 block pair (I >= J) of the triangle.  The block
// pairs of a channel are packed into workgroups in closed form (decode_item):
// 2x2 super-tiles below the diagonal, diagonal super-tiles that borrow a pair
// from the odd last block row, and the rest of that row in groups of three.
//
// Data path per stage of KT = 64 samples:
//   HBM/L2 -> registers: each thread reads 16 consecutive time rows of 4
//            inputs (one dword per row for ci4, two for ci8), coalesced along
//            the input axis;
//   registers: 4x4 byte transposes (v_perm) turn rows into per-input runs of
//            time; ci4 is split into 16*re and 16*im bytes (the nibble kept in
//            the high half of the byte, which is that value times 16 as int8);
//   LDS:     planes [re|im][t16][slot*64 + input][16 bytes]; a lane's MFMA
//            fragment is one 16-byte ds_read;
//   MFMA:    v_mfma_i32_32x32x32_i8 on 32x32 sub-blocks.
// ci4 results carry a factor 256 in the registers and are shifted back
// (exactly) in the epilogue.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfx_internal.h"

namespace bfx {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kBlk = 64;                       // inputs per block / LDS slot
constexpr int kSlots = 4;                      // input blocks staged per workgroup
constexpr int kKT = 64;                        // time samples per stage
constexpr int kRows = kSlots * kBlk;           // 256 LDS rows per t16 group
constexpr int kPlane = (kKT / 16) * kRows * 16;  // 16 KiB
constexpr int kStage = 2 * kPlane;             // re + im planes
constexpr int kThreads = 256;

struct Task {
    int blk[kSlots];  // input block held by each LDS slot, -1 = unused
    int rs[4];        // per wave: LDS slot of its row block, -1 = idle wave
    int cs[4];        // per wave: LDS slot of its column block
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

__device__ inline uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// Transpose a 4x4 byte matrix held as rows r0..r3 (byte k of row r = element
// (r, k)) into columns c0..c3 (byte r of column k = element (r, k)).
__device__ inline void transpose4(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3,
                                  uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3) {
    const uint32_t t0 = perm(r1, r0, 0x05010400u);
    const uint32_t t1 = perm(r1, r0, 0x07030602u);
    const uint32_t t2 = perm(r3, r2, 0x05010400u);
    const uint32_t t3 = perm(r3, r2, 0x07030602u);
    c0 = perm(t2, t0, 0x05040100u);
    c1 = perm(t2, t0, 0x07060302u);
    c2 = perm(t3, t1, 0x05040100u);
    c3 = perm(t3, t1, 0x07060302u);
}

template <bool CI4>
struct Stage;

// ci4: one dword (4 packed samples of 4 consecutive inputs) per time row.
template <>
struct Stage<true> {
    uint32_t d[16];

    __device__ inline void load(const uint8_t *row0, int64_t t_stride, int nrows, bool ok) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            d[r] = 0;
            if (ok && r < nrows) d[r] = *(const uint32_t *)(row0 + (int64_t)r * t_stride);
        }
    }

    // Write the 4 inputs' re / im runs of 16 samples into both planes.
    __device__ inline void store(uint8_t *plane_re, uint8_t *plane_im, int row) const {
        uint32_t c[4][4];  // c[m][e]: samples 4m..4m+3 of input e
#pragma unroll
        for (int m = 0; m < 4; ++m)
            transpose4(d[4 * m], d[4 * m + 1], d[4 * m + 2], d[4 * m + 3],
                       c[m][0], c[m][1], c[m][2], c[m][3]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v4i re, im;
            re.x = (int)(c[0][e] & 0xF0F0F0F0u);
            re.y = (int)(c[1][e] & 0xF0F0F0F0u);
            re.z = (int)(c[2][e] & 0xF0F0F0F0u);
            re.w = (int)(c[3][e] & 0xF0F0F0F0u);
            im.x = (int)((c[0][e] << 4) & 0xF0F0F0F0u);
            im.y = (int)((c[1][e] << 4) & 0xF0F0F0F0u);
            im.z = (int)((c[2][e] << 4) & 0xF0F0F0F0u);
            im.w = (int)((c[3][e] << 4) & 0xF0F0F0F0u);
            *(v4i *)(plane_re + (row + e) * 16) = re;
            *(v4i *)(plane_im + (row + e) * 16) = im;
        }
    }
};

// ci8: two dwords (re, im of 4 consecutive inputs) per time row.
template <>
struct Stage<false> {
    uint32_t lo[16], hi[16];

    __device__ inline void load(const uint8_t *row0, int64_t t_stride, int nrows, bool ok) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            lo[r] = 0;
            hi[r] = 0;
            if (ok && r < nrows) {
                const uint2 v = *(const uint2 *)(row0 + (int64_t)r * t_stride);
                lo[r] = v.x;
                hi[r] = v.y;
            }
        }
    }

    __device__ inline void store(uint8_t *plane_re, uint8_t *plane_im, int row) const {
        // lo bytes: in0.re in0.im in1.re in1.im ; hi: in2.re in2.im in3.re in3.im
        uint32_t cl[4][4], ch[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            transpose4(lo[4 * m], lo[4 * m + 1], lo[4 * m + 2], lo[4 * m + 3],
                       cl[m][0], cl[m][1], cl[m][2], cl[m][3]);
            transpose4(hi[4 * m], hi[4 * m + 1], hi[4 * m + 2], hi[4 * m + 3],
                       ch[m][0], ch[m][1], ch[m][2], ch[m][3]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = (e & 1) * 2;
            v4i re, im;
            if (e < 2) {
                re = v4i{(int)cl[0][k], (int)cl[1][k], (int)cl[2][k], (int)cl[3][k]};
                im = v4i{(int)cl[0][k + 1], (int)cl[1][k + 1], (int)cl[2][k + 1], (int)cl[3][k + 1]};
            } else {
                re = v4i{(int)ch[0][k], (int)ch[1][k], (int)ch[2][k], (int)ch[3][k]};
                im = v4i{(int)ch[0][k + 1], (int)ch[1][k + 1], (int)ch[2][k + 1], (int)ch[3][k + 1]};
            }
            *(v4i *)(plane_re + (row + e) * 16) = re;
            *(v4i *)(plane_im + (row + e) * 16) = im;
        }
    }
};

struct Acc {
    v16i re[2][2], p[2][2], q[2][2];
};

// One 32-sample MFMA step of a wave's 64x64 block pair.  `full` is true when
// all four 32x32 sub-blocks are live; otherwise `live` masks them.
template <bool FULL>
__device__ inline void mfma_step(const uint8_t *stage, int kk, int lane, int rrow, int crow,
                                 unsigned live, Acc &acc) {
    const int g = lane >> 5;
    const int r32 = lane & 31;
    const uint8_t *pre = stage + ((2 * kk + g) * kRows) * 16;
    const uint8_t *pim = pre + kPlane;
    v4i ar[2], ai[2], br[2], bi[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        ar[r] = *(const v4i *)(pre + (rrow + 32 * r + r32) * 16);
        ai[r] = *(const v4i *)(pim + (rrow + 32 * r + r32) * 16);
        br[r] = *(const v4i *)(pre + (crow + 32 * r + r32) * 16);
        bi[r] = *(const v4i *)(pim + (crow + 32 * r + r32) * 16);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (FULL || (live >> (2 * r + c)) & 1u) {
                acc.re[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ar[r], br[c], acc.re[r][c], 0, 0, 0);
                acc.re[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ai[r], bi[c], acc.re[r][c], 0, 0, 0);
                acc.p[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ai[r], br[c], acc.p[r][c], 0, 0, 0);
                acc.q[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ar[r], bi[c], acc.q[r][c], 0, 0, 0);
            }
        }
    }
}

template <bool CI4>
__global__ __launch_bounds__(kThreads, 1) void xengine_int_kernel(
    const uint8_t *__restrict__ in, int64_t t_stride, int nt, int nchan, int ninput, int nitems,
    int32_t *__restrict__ out, int overwrite) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kStage];

    // XCD-aware order: consecutive block ids go to different XCDs (round
    // robin), so channel f is given to the blocks whose id is f mod 8; the
    // items of one channel then share one XCD's L2.
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int s = bid >> 3;
    const int cl = s / nitems;
    const int item = s - cl * nitems;
    const int f = cl * 8 + xcd;
    if (f >= nchan) return;

    const int nb = (ninput + kBlk - 1) / kBlk;
    Task tk;
    decode_item(nb, item, tk);

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;

    // ---- staging role: wave = t16 group, lane = (slot, input quad)
    const int slot = lane >> 4;
    const int quad = lane & 15;
    const int sblk = pick4(tk.blk, slot);
    const int in0 = sblk * kBlk + quad * 4;
    const bool sok = sblk >= 0 && in0 < ninput;
    constexpr int bps = CI4 ? 1 : 2;
    const uint8_t *src = in + (int64_t)f * ninput * bps + (int64_t)(sok ? in0 : 0) * bps;
    const int lrow = slot * kBlk + quad * 4;

    // ---- compute role
    const int rs = pick4(tk.rs, wave);
    const int cs = pick4(tk.cs, wave);
    const bool active = rs >= 0;
    const int rblk = active ? pick4(tk.blk, rs) : 0;
    const int cblk = active ? pick4(tk.blk, cs) : 0;
    unsigned live = 0;
    if (active) {
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                const bool ok = rblk * kBlk + 32 * r < ninput && cblk * kBlk + 32 * c < ninput &&
                                !(rblk == cblk && r == 0 && c == 1);
                if (ok) live |= 1u << (2 * r + c);
            }
    }
    const bool full = live == 0xFu;

    Acc acc;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            acc.re[r][c] = v16i{0};
            acc.p[r][c] = v16i{0};
            acc.q[r][c] = v16i{0};
        }

    const int nst = (nt + kKT - 1) / kKT;
    Stage<CI4> st;
    auto issue = [&](int stage_idx) {
        const int t0 = stage_idx * kKT + wave * 16;
        const int nrows = nt - t0;
        st.load(src + (int64_t)t0 * t_stride, t_stride, nrows, sok);
    };
    auto put = [&](int buf) {
        uint8_t *base = lds + buf * kStage + (wave * kRows) * 16;
        if (sblk >= 0) st.store(base, base + kPlane, lrow);
    };

    issue(0);
    put(0);
    if (nst > 1) issue(1);
    __syncthreads();

    for (int sidx = 0; sidx < nst; ++sidx) {
        const uint8_t *stage = lds + (sidx & 1) * kStage;
        if (active) {
            if (full) {
#pragma unroll
                for (int kk = 0; kk < 2; ++kk)
                    mfma_step<true>(stage, kk, lane, rs * kBlk, cs * kBlk, live, acc);
            } else {
#pragma unroll
                for (int kk = 0; kk < 2; ++kk)
                    mfma_step<false>(stage, kk, lane, rs * kBlk, cs * kBlk, live, acc);
            }
        }
        if (sidx + 1 < nst) {
            put((sidx + 1) & 1);
            if (sidx + 2 < nst) issue(sidx + 2);
        }
        __syncthreads();
    }

    if (!active) return;

    // ---- epilogue: 32x32 output layout of v_mfma_*_32x32: lane l, register v
    // hold row 8*(v/4) + 4*(l/32) + v%4, column l%32.
    const int64_t P = (int64_t)ninput * (ninput + 1) / 2;
    int32_t *obase = out + (int64_t)f * P * 2;
    const int g = lane >> 5;
    const int n = lane & 31;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (!((live >> (2 * r + c)) & 1u)) continue;
            const int j = cblk * kBlk + 32 * c + n;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = rblk * kBlk + 32 * r + 8 * (v >> 2) + 4 * g + (v & 3);
                if (i < ninput && j <= i) {
                    int vr = acc.re[r][c][v];
                    int vi = acc.p[r][c][v] - acc.q[r][c][v];
                    if (CI4) { vr >>= 8; vi >>= 8; }
                    int2 *dst = (int2 *)(obase + ((int64_t)i * (i + 1) / 2 + j) * 2);
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
}

}  // namespace

int xengine_tri_items(int32_t ninput) { return tri_items((ninput + kBlk - 1) / kBlk); }

hipError_t launch_xengine_int(bool ci4, const void *in, int64_t nt, int32_t nchan, int32_t ninput,
                              int32_t *out, bool overwrite, hipStream_t s) {
    const int nb = (ninput + kBlk - 1) / kBlk;
    const int nitems = tri_items(nb);
    const int64_t nchan8 = ((int64_t)nchan + 7) / 8 * 8;
    const int64_t grid = nchan8 * nitems;
    const int64_t t_stride = (int64_t)nchan * ninput * (ci4 ? 1 : 2);
    if (ci4)
        hipLaunchKernelGGL(xengine_int_kernel<true>, dim3((unsigned)grid), dim3(kThreads), 0, s,
                           (const uint8_t *)in, t_stride, (int)nt, nchan, ninput, nitems, out,
                           (int)overwrite);
    else
        hipLaunchKernelGGL(xengine_int_kernel<false>, dim3((unsigned)grid), dim3(kThreads), 0, s,
                           (const uint8_t *)in, t_stride, (int)nt, nchan, ninput, nitems, out,
                           (int)overwrite);
    return hipGetLastError();
}

}  // namespace bfx
