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
// split needs one v_permlane32_swap per register -- a wavefront shuffle, no
// LDS and no barrier.  The third pass reads butterflies above 128 in reversed
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
constexpr int kTw2Bytes = 256 * 8;                  // pass-2 twiddles W^(16 r c), r, c < 16
constexpr int kLdsBytes = kABytes + kBBytes + kTw2Bytes;  // two workgroups per CU

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

__device__ __forceinline__ int8_t requant(float v, float s) {
    float r = rintf(s * v);  // round half to even
    r = fminf(fmaxf(r, -127.0f), 127.0f);
    return (int8_t)r;
}

// Work item B -> (frame s, input group g); frames map to XCDs by s % 8.
__device__ __forceinline__ bool item_of(int B, int ngroup, int nspec, int &s, int &g) {
    const int sq = B >> 3;
    const int fl = sq / ngroup;
    g = sq - fl * ngroup;
    s = fl * 8 + (B & 7);
    return s < nspec;
}

// The 16 first-pass rows (j + 256 r) of this lane for the item's 8 inputs.
__device__ __forceinline__ void load_samples(uint64_t (&x)[16], const int8_t *in, int ninput, int s,
                                             int g, int j) {
    const int8_t *src = in + ((int64_t)s * kN + j) * ninput + g * kGroup;
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = *(const uint64_t *)(src + (int64_t)(256 * r) * ninput);
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
    const bool self0 = b3 == 0, self128 = b3 == 128;  // self-paired butterflies
    const bool lower = (j & 63) < 32;
    // pass-3 twiddles in registers; the pass-2 ones (16 distinct sets, by
    // j % 16) in a small LDS table, published by the first barrier
    float2 tw3[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) tw3[r] = g_twiddle[(r * b3) & (kN - 1)];
    float2 *tw2 = (float2 *)(lds + kABytes + kBBytes);
    tw2[j] = g_twiddle[((j >> 4) * (j & 15) * (kN / 256)) & (kN - 1)];  // entry 16 r + c
    // a row's 8 bytes (the item's 8 inputs); each pair takes the low 16 bits
    // and shifts them out, so the pair loop never selects by its index
    uint64_t xs[16];
    load_samples(xs, in, ninput, s, g, j);

    while (true) {
        // next item: its samples are fetched into the registers of this
        // item's samples once the last pair has taken them (the loads then
        // overlap that pair's transform)
        int Bn = B + gridDim.x, sn = 0, gn = 0;
        bool nvalid = false;
        while (Bn < total_flat && !(nvalid = item_of(Bn, ngroup, nspec, sn, gn))) Bn += gridDim.x;
        const int i0 = g * kGroup;

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
        // (not unrolled: one pair's registers at a time)
#pragma unroll 1
        for (int p = 0; p < kPairs; ++p) {
            // pass 1 (Ns = 1): z[n] = x_a[n] + i x_b[n], n = j + 256 r
            float2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t two = (uint32_t)xs[r];  // bytes 2 p, 2 p + 1 of the row
                xs[r] >>= 16;
                v[r] = float2{(float)(int8_t)(two & 0xFF), (float)(int8_t)((two >> 8) & 0xFF)};
            }
            if (p == kPairs - 1 && nvalid) load_samples(xs, in, ninput, sn, gn, j);
            dft16(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) A[pad_a(16 * j + r)] = v[r];
            block_barrier();
            // pass 2 (Ns = 16): A -> B
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = A[pad_a(j + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw2[16 * r + (j & 15)]);
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
            // (one v_permlane32_swap per component); butterfly 0 uses its own
            // register (16 - m) % 16, butterfly 128 its own register 15 - m
#pragma unroll
            for (int c = 0; c < kChan / kThreads; ++c) {
                const int k = b3 + kThreads * c;
                const float2 z = v[c];
                const auto sx = __builtin_amdgcn_permlane32_swap(__float_as_int(v[15 - c].x),
                                                                  __float_as_int(v[15 - c].x), false, false);
                const auto sy = __builtin_amdgcn_permlane32_swap(__float_as_int(v[15 - c].y),
                                                                  __float_as_int(v[15 - c].y), false, false);
                float2 w{__int_as_float(lower ? sx[1] : sx[0]), __int_as_float(lower ? sy[1] : sy[0])};
                if (self128) w = v[15 - c];
                if (self0) w = v[(16 - c) & 15];
                // X_a = (z + conj w)/2, X_b = (z - conj w)/(2i) = -i (z - conj w)/2
                if (CI8) {
                    // the halving rides on the scale: fl(s fl(x / 2)) = fl((s / 2) x)
                    const float hs = 0.5f * scale[k];
                    const uint32_t word = (uint32_t)(uint8_t)requant(z.x + w.x, hs) |
                                          ((uint32_t)(uint8_t)requant(z.y - w.y, hs) << 8) |
                                          ((uint32_t)(uint8_t)requant(z.y + w.y, hs) << 16) |
                                          ((uint32_t)(uint8_t)requant(w.x - z.x, hs) << 24);
                    q[c] = uint4{q[c].y, q[c].z, q[c].w, word};
                } else {
                    const float2 xa{0.5f * (z.x + w.x), 0.5f * (z.y - w.y)};
                    const float2 xb{0.5f * (z.y + w.y), -0.5f * (z.x - w.x)};
                    float4 *o = (float4 *)((float *)out +
                                           (((int64_t)s * kChan + k) * ninput + i0 + 2 * p) * 2);
                    *o = float4{xa.x, xa.y, xb.x, xb.y};
                }
            }
        }
        if (CI8) {
            // [k][8 inputs][re, im] = the 4 pairs' bytes in order: 16 bytes
            int8_t *o = (int8_t *)out;
#pragma unroll
            for (int c = 0; c < kChan / kThreads; ++c) {
                const int k = b3 + kThreads * c;
                *(uint4 *)(o + (((int64_t)s * kChan + k) * ninput + i0) * 2) = q[c];
            }
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
