// F-engine for gfx950: real 8-bit samples -> FP32 spectra -> requantized ci8.
//
// The paper's F-engine (Sec. 6) turns 204.8 MS/s real samples into 4096
// channels; the library's FFT and quantize modules (Sec. 2.2) are the GPU
// building blocks.  Per frame s and input i:
//   X_s[k][i] = sum_{n<4096} x[4096 s + n][i] exp(-2 pi i k n / 4096),
//   k = 0 .. 2047 (bin 0 = DC, Nyquist dropped, no window, no normalisation),
// then, for ci8 output, q = clamp(round_half_even(scale_k * X), -127, 127)
// applied to the real and imaginary parts in binary32.
//
// Organisation.  The grid is persistent (two workgroups of 4 waves per CU,
// so that one's barriers and LDS exchanges overlap the other's arithmetic);
// a work item is one frame of 8 adjacent inputs, and consecutive items of a
// workgroup belong to frames on the same XCD, so the row segments of
// neighbouring input groups meet in one L2.  Two adjacent real inputs a, b
// form one complex sequence z = x_a + i x_b (two-for-one); the workgroup's
// 256 lanes transform its 4 pairs one at a time with a radix-16 Stockham FFT
// (4096 = 16^3, three passes, 16 points per lane in registers), and
//   X_a[k] = (Z[k] + conj Z[-k]) / 2,   X_b[k] = (Z[k] - conj Z[-k]) / (2i).
//
// Exchanges.  Passes 1 -> 2 and 2 -> 3 go through two LDS buffers (one
// barrier each; the buffers alternate so no other barrier is needed).  Every
// half-wave's accesses of each exchange fall on distinct banks: the first
// buffer is padded (an additive map, folded into the instructions' offsets),
// the second XOR-swizzled (no additive map serves its accesses).  The third
// pass gives each wave a set of butterflies closed under b -> 256 - b, with
// butterfly b in lane i < 32 and 256 - b in lane i + 32 (wave 0 keeps the
// self-paired 0 and 128 in lanes 0 and 32).  Butterfly b holds Z[b + 256 m],
// and Z[-k] for k = b + 256 m is register 15 - m of butterfly 256 - b, so the
// split needs one ds_bpermute per register component from the lane 32 away --
// a wavefront shuffle through the LDS crossbar, no LDS storage and no
// barrier.  The third pass reads butterflies above 128 in reversed
// order in a buffer laid out to match (index map piB), so both half-waves read
// ascending addresses.
//
// The samples a lane needs for the first pass (16 rows, the item's 8 inputs)
// come straight from global memory into registers; the next item's are
// fetched into the same registers once the last pair has taken them, so the
// loads overlap that pair's transform.  The twiddles of the
// lane's second- and third-pass butterflies (which depend only on the lane)
// are loaded once per workgroup into registers.  A lane's requantized bytes
// of its 8 channels stay in registers across the 4 pairs and leave as one
// 16-byte [k][8 inputs] segment per channel.  Twiddles come from a 4096-entry
// table computed once per device in FP64 on the host from the exact integer
// phase k n mod 4096, then rounded to binary32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "bfx_internal.h"
#include "fft16.h"

namespace bfx {
namespace {

constexpr int kN = 4096;           // transform length
constexpr int kChan = kN / 2;      // channels kept
constexpr int kGroup = 8;          // inputs per workgroup
constexpr int kPairs = kGroup / 2; // complex sequences per workgroup
constexpr int kThreads = 256;      // lanes of one FFT (4096 / 16 points each)
constexpr int kABytes = kPadAElems * 8;             // pass 1 -> 2, padded (pad_a)
constexpr int kBBytes = kN * 8;                     // pass 2 -> 3, swizzled (swz_b)
constexpr int kLdsBytes = kABytes + kBBytes;      // two workgroups per CU

// Buffer A (pass 1 -> 2) uses the additive pad_a (fft16.h).
// Buffer B (pass 2 -> 3): butterflies above 128 of each 256 block in reversed
// order (piB), then x ^ (((x >> 8) & 15) << 4): conflict-free for the pass-2
// writes (16-lane groups) and for both half-waves' pass-3 reads.
__device__ __forceinline__ int swz_b(int x) {
    const int b = x & 255;
    const int y = (x & ~255) | (b <= 128 ? b : 384 - b);
    return y ^ (((y >> 8) & 15) << 4);
}
// Third-pass butterfly of lane tid (see the header).
__device__ __forceinline__ int pass3_butterfly(int tid) {
    const int w = tid >> 6, i = tid & 63;
    if (i < 32) return 32 * w + i;
    const int i2 = i - 32;
    return (w == 0 && i2 == 0) ? 128 : 256 - 32 * w - i2;
}

__device__ float2 g_twiddle[kN];  // exp(-2 pi i m / 4096), m = 0..4095

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Requantize: round half to even of v s, saturated to +-127, returned as the
// low byte of a binary32 bit pattern.  fma(v, s, 1.5 2^23) rounds the exact
// product to an integer n once (|v s| < 2^22 keeps the sum in [2^23, 2^24),
// where the spacing is 1, and 1.5 2^23 is even, so ties go to even n) and
// leaves 1.5 2^23 + n, whose bit pattern is 0x4B400000 + n; clamping that
// float to 1.5 2^23 +- 127 saturates n, and every |v s| >= 2^22 lands
// outside the clamp range on the correct side.
__device__ __forceinline__ uint32_t requant_bits(float v, float s) {
    constexpr float kMagic = 12582912.0f;
    const float t = __builtin_fmaf(v, s, kMagic);
    return __float_as_uint(__builtin_amdgcn_fmed3f(t, kMagic - 127.0f, kMagic + 127.0f));
}

// Low bytes of four words as one word, r0 in byte 0.
__device__ __forceinline__ uint32_t pack_low_bytes(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3) {
    const uint32_t lo = __builtin_amdgcn_perm(r1, r0, 0x0c0c0400u);
    const uint32_t hi = __builtin_amdgcn_perm(r3, r2, 0x0c0c0400u);
    return lo | (hi << 16);
}

// Work item B -> (frame s, input group g); frames map to XCDs by s % 8.
__device__ __forceinline__ bool item_of(int B, int ngroup, int nspec, int &s, int &g) {
    const int sq = B >> 3;
    const int fl = sq / ngroup;
    g = sq - fl * ngroup;
    s = fl * 8 + (B & 7);
    return s < nspec;
}

// Sample loads: raw buffer access, a uniform base in a buffer descriptor
// (scalar registers) plus a lane's 32-bit offset and a uniform 32-bit offset.
// A frame spans fewer than 2^32 bytes, so per-lane addresses need no 64-bit
// vector arithmetic.  Descriptor word 3: 32-bit data format (required by gfx9
// for raw buffer access); no range is enforced below 2^32.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t frame_rsrc(const void *base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)0xFFFFFFFFu, 0x00020000);
}

// Output stores go through global (not buffer) stores: the same kind of
// uniform base, kept whole in scalar registers, plus the lane's 32-bit offset.
// (A 16-byte buffer store with a scalar offset register gets no wait state
// before its data registers are overwritten, and its first dword was seen to
// take the overwriting value.)
#define BFX_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ BFX_GLOBAL T *uniform_ptr(T *p) {
    uint64_t u = (uint64_t)p;
    asm volatile("" : "+s"(u));
    return (BFX_GLOBAL T *)u;
}

// The 16 first-pass rows (j + 256 r) of this lane for the item's 8 inputs,
// joff = j ninput.
__device__ __forceinline__ void load_samples(uint64_t (&x)[16], const int8_t *in, int ninput, int s,
                                             int g, uint32_t joff) {
    const __amdgpu_buffer_rsrc_t rs = frame_rsrc(in + (int64_t)s * kN * ninput + g * kGroup);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, joff, 256 * r * ninput, 0);
        x[r] = (uint64_t)(uint32_t)w[0] | ((uint64_t)(uint32_t)w[1] << 32);
    }
}

template <bool CI8>
__global__ __launch_bounds__(kThreads, 2) void fengine_kernel(
    const int8_t *__restrict__ in, int ninput, int nspec, int ngroup, int total_flat,
    const float *__restrict__ scale, void *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int j = tid;                     // lane of the FFT
    float2 *buf0 = (float2 *)lds;          // pass 1 -> 2, pass 3 -> split
    float2 *buf1 = (float2 *)(lds + kABytes);  // pass 2 -> 3

    int B = blockIdx.x, s = 0, g = 0;
    bool valid = false;
    while (B < total_flat && !(valid = item_of(B, ngroup, nspec, s, g))) B += gridDim.x;
    if (!valid) return;

    // twiddles of this lane's pass-2 (Ns = 16) and pass-3 (Ns = 256) butterflies
    const int b3 = pass3_butterfly(j);
    const bool self0 = b3 == 0;  // butterflies 0 and 128 pair with themselves
    // Z[-k] of butterfly b3 lives in the lane holding 256 - b3: lane j ^ 32,
    // except for the self-paired butterflies (lanes 0 and 32 of wave 0), which
    // read their own registers (ds_bpermute byte address of the source lane)
    const int partner = (b3 == 0 || b3 == 128) ? (j & 63) : ((j & 63) ^ 32);
    const int paddr = 4 * partner;
    // pass-2 (W^(16 r (j % 16))) and pass-3 (W^(r b3)) twiddles in registers
    // (holding the pass-2 ones in an LDS table instead was 2.5% slower)
    float2 tw2[16], tw3[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        tw2[r] = g_twiddle[(r * (j & 15) * (kN / 256)) & (kN - 1)];
        tw3[r] = g_twiddle[(r * b3) & (kN - 1)];
    }
    // scale of channel b3 + 256 c, halved (the split's 1/2 rides on it:
    // fl(s fl(x / 2)) = fl((s / 2) x))
    float hs[kChan / kThreads];
    if (CI8) {
#pragma unroll
        for (int c = 0; c < kChan / kThreads; ++c) hs[c] = 0.5f * scale[b3 + kThreads * c];
    }
    // 32-bit per-lane offsets within a frame (a frame spans < 2^32 bytes)
    const uint32_t joff = (uint32_t)(j * ninput);
    const uint32_t koff = (uint32_t)(b3 * ninput) * (CI8 ? 2u : 8u);  // channel b3's row
    const uint32_t cstride = (uint32_t)(kThreads * ninput) * (CI8 ? 2u : 8u);  // 256 channels
    // a row's 8 bytes (the item's 8 inputs); pair p takes bytes 2 p, 2 p + 1
    // with one v_perm whose selector is uniform, so the pair loop never
    // selects registers by its index
    uint64_t xs[16];
    load_samples(xs, in, ninput, s, g, joff);

    while (true) {
        // next item: its samples are fetched into the registers of this
        // item's samples once the last pair has taken them (the loads then
        // overlap that pair's transform)
        int Bn = B + gridDim.x, sn = 0, gn = 0;
        bool nvalid = false;
        while (Bn < total_flat && !(nvalid = item_of(Bn, ngroup, nspec, sn, gn))) Bn += gridDim.x;
        const int i0 = g * kGroup;
        // frame s, input i0 of the output (uniform); channel rows add koff
        uint8_t *orow = (uint8_t *)out + ((int64_t)s * kChan * ninput + i0) * (CI8 ? 2 : 8);

        // ci8 bytes (a_re, a_im, b_re, b_im) of each pair, rotated in pair by
        // pair so that after the last pair q[c] holds pairs 0..3 in order
        uint4 q[kChan / kThreads];
        // Buffers: pass 1 -> A, pass 2 A -> B, pass 3 reads B.  The next
        // pair's pass-1 writes to A follow this pair's barrier after pass 2
        // (all reads of A done) and its pass-2 writes to B follow the next
        // pair's first barrier (all pass-3 reads of B done): two barriers per
        // pair.
        float2 *A = buf0;
        float2 *Bf = buf1;
        // One pair's transform.  Pairs 0..2 run in a loop (not unrolled: one
        // pair's registers at a time); the last pair, peeled, also fetches the
        // next item's samples once its own are taken, so within the loop the
        // sample registers never change.
        auto pair = [&](const int p, const bool prefetch) {
            // pass 1 (Ns = 1): z[n] = x_a[n] + i x_b[n], n = j + 256 r
            float2 v[16];
            // bytes 2 p, 2 p + 1 of a row word to bytes 0, 1 (v_perm selector)
            const uint32_t sel = 0x0c0c0000u | (uint32_t)(2 * p) | ((uint32_t)(2 * p + 1) << 8);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t two = __builtin_amdgcn_perm((uint32_t)(xs[r] >> 32), (uint32_t)xs[r], sel);
                v[r] = float2{(float)(int8_t)(two & 0xFF), (float)(int8_t)((two >> 8) & 0xFF)};
            }
            if (prefetch) load_samples(xs, in, ninput, sn, gn, joff);
            dft16(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) A[pad_a(16 * j + r)] = v[r];
            block_barrier();
            // pass 2 (Ns = 16): A -> B
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = A[pad_a(j + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw2[r]);
            }
            dft16(v);
            {
                const int base = (j / 16) * 256 + (j & 15);
#pragma unroll
                for (int r = 0; r < 16; ++r) Bf[swz_b(base + r * 16)] = v[r];
            }
            block_barrier();
            // pass 3 (Ns = 256): butterfly b3, outputs Z[b3 + 256 m] in v[m]
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = Bf[swz_b(b3 + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw3[r]);
            }
            dft16(v);
            // two-for-one split for k = b3 + 256 m, m = 0..7:
            // Z[-k] = register 15 - m of butterfly 256 - b3, 32 lanes away
            // (a ds_bpermute per component: a wavefront shuffle through the
            // LDS crossbar, no LDS storage and no barrier); butterfly 128
            // reads its own register 15 - m, butterfly 0 its own register
            // (16 - m) % 16
            float2 wv[kChan / kThreads];
#pragma unroll
            for (int c = 0; c < kChan / kThreads; ++c) {
                wv[c].x = __int_as_float(__builtin_amdgcn_ds_bpermute(paddr, __float_as_int(v[15 - c].x)));
                wv[c].y = __int_as_float(__builtin_amdgcn_ds_bpermute(paddr, __float_as_int(v[15 - c].y)));
            }
            if (self0) {
#pragma unroll
                for (int c = 0; c < kChan / kThreads; ++c) wv[c] = v[(16 - c) & 15];
            }
#pragma unroll
            for (int c = 0; c < kChan / kThreads; ++c) {
                const float2 z = v[c];
                const float2 w = wv[c];
                // X_a = (z + conj w)/2, X_b = (z - conj w)/(2i) = -i (z - conj w)/2
                if (CI8) {
                    const uint32_t word = pack_low_bytes(requant_bits(z.x + w.x, hs[c]),
                                                         requant_bits(z.y - w.y, hs[c]),
                                                         requant_bits(z.y + w.y, hs[c]),
                                                         requant_bits(w.x - z.x, hs[c]));
                    q[c] = uint4{q[c].y, q[c].z, q[c].w, word};
                } else {
                    const float2 xa{0.5f * (z.x + w.x), 0.5f * (z.y - w.y)};
                    const float2 xb{0.5f * (z.y + w.y), -0.5f * (z.x - w.x)};
                    *(BFX_GLOBAL v4u *)(uniform_ptr(orow + 16 * p + c * cstride) + koff) =
                        v4u{__float_as_uint(xa.x), __float_as_uint(xa.y), __float_as_uint(xb.x),
                            __float_as_uint(xb.y)};
                }
            }
        };
#pragma unroll 1
        for (int p = 0; p < kPairs - 1; ++p) pair(p, false);
        pair(kPairs - 1, nvalid);
        if (CI8) {
            // [k][8 inputs][re, im] = the 4 pairs' bytes in order: 16 bytes
#pragma unroll
            for (int c = 0; c < kChan / kThreads; ++c)
                *(BFX_GLOBAL v4u *)(uniform_ptr(orow + c * cstride) + koff) = v4u{q[c].x, q[c].y, q[c].z, q[c].w};
        }
        if (!nvalid) break;
        B = Bn;
        s = sn;
        g = gn;
    }
}

DeviceInit g_init;

// The twiddle table (per device) and the kernels' LDS attribute.
hipError_t init_device() {
    static float2 host[kN];
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < kN; ++m) {
        host[m].x = (float)cos(two_pi * m / kN);
        host[m].y = (float)-sin(two_pi * m / kN);
    }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle), host, sizeof host, 0, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)fengine_kernel<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)fengine_kernel<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    return e;
}

}  // namespace

bool fengine_supported(int32_t ninput, int32_t nfft) { return nfft == kN && ninput % kGroup == 0; }

hipError_t launch_fengine(const int8_t *in, int32_t ninput, int32_t nfft, int64_t nspec,
                          const float *scale, void *out, bool ci8, hipStream_t s) {
    if (!fengine_supported(ninput, nfft)) return hipErrorNotSupported;
    int num_cus = 0;
    const hipError_t e = g_init.ensure(init_device, &num_cus);
    if (e != hipSuccess) return e;
    const int ngroup = ninput / kGroup;
    const int64_t nspec8 = (nspec + 7) / 8 * 8;
    const int64_t total = nspec8 * ngroup;
    if (total > INT32_MAX) return hipErrorInvalidValue;
    // persistent grid: two workgroups per CU, a multiple of 8 (the XCD count)
    int64_t grid = (int64_t)num_cus * 2 / 8 * 8;
    if (grid < 8) grid = 8;
    if (grid > total) grid = total;
    if (ci8)
        hipLaunchKernelGGL(fengine_kernel<true>, dim3((unsigned)grid), dim3(kThreads), kLdsBytes,
                           s, in, ninput, (int)nspec, ngroup, (int)total, scale, out);
    else
        hipLaunchKernelGGL(fengine_kernel<false>, dim3((unsigned)grid), dim3(kThreads), kLdsBytes,
                           s, in, ninput, (int)nspec, ngroup, (int)total, scale, out);
    return hipGetLastError();
}

}  // namespace bfx
