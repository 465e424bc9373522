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
// Organisation.  One workgroup (8 waves) handles one frame of 16 adjacent
// inputs.  Their 4096 x 16-byte block of samples arrives in LDS through
// global_load_lds_dwordx4 (a 16-byte row segment per lane).  Two adjacent
// real inputs a, b form one complex sequence z = x_a + i x_b (two-for-one);
// each team of 4 waves (256 lanes) transforms one such pair at a time with a
// radix-16 Stockham FFT (4096 = 16^3, three passes, 16 points per lane in
// registers, the passes exchanging through a padded LDS buffer), and
//   X_a[k] = (Z[k] + conj Z[-k]) / 2,   X_b[k] = (Z[k] - conj Z[-k]) / (2i).
// The requantized bytes of a pair are parked in the LDS bytes its samples
// occupied (consumed by then); when all 8 pairs are done the workgroup writes
// the [k][16 inputs] ci8 block as 32-byte row segments.  Twiddles come from a
// 4096-entry table computed once per device in FP64 on the host from the
// exact integer phase k n mod 4096, then rounded to binary32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "bfx_internal.h"

namespace bfx {
namespace {

constexpr int kN = 4096;           // transform length
constexpr int kChan = kN / 2;      // channels kept
constexpr int kGroup = 16;         // inputs per workgroup
constexpr int kPairs = kGroup / 2; // complex sequences per workgroup
constexpr int kTeamLanes = 256;    // lanes per FFT team (4096 / 16)
constexpr int kTeams = 2;
constexpr int kThreads = kTeamLanes * kTeams;
constexpr int kInBytes = kN * kGroup;               // 64 KiB of samples
constexpr int kFftElems = kN + kN / 16;             // one pad float2 per 16
constexpr int kFftBytes = kFftElems * 8;            // 34 KiB per team
constexpr int kLdsBytes = kInBytes + kTeams * kFftBytes;

__device__ float2 g_twiddle[kN];  // exp(-2 pi i m / 4096), m = 0..4095

__device__ __forceinline__ int pad(int idx) { return idx + (idx >> 4); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return float2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// forward radix-4 DFT in place on (a0, a1, a2, a3)
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    const float2 b0{a0.x + a2.x, a0.y + a2.y}, b1{a0.x - a2.x, a0.y - a2.y};
    const float2 b2{a1.x + a3.x, a1.y + a3.y}, b3{a1.x - a3.x, a1.y - a3.y};
    a0 = float2{b0.x + b2.x, b0.y + b2.y};
    a2 = float2{b0.x - b2.x, b0.y - b2.y};
    a1 = float2{b1.x + b3.y, b1.y - b3.x};  // b1 - i b3
    a3 = float2{b1.x - b3.y, b1.y + b3.x};  // b1 + i b3
}

// forward 16-point DFT in registers, natural order in and out:
// n = 4 n1 + n2, k = k1 + 4 k2,
// X[k1 + 4 k2] = sum_n2 W4^(n2 k2) W16^(n2 k1) sum_n1 v[4 n1 + n2] W4^(n1 k1).
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
    // W16^m = exp(-2 pi i m / 16), m = 0..9 (the products n2 * k1 needed)
    constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    constexpr float c2 = 0.70710678118654752440f;
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    // v[n2 + 4 k1] now holds T[n2][k1]; apply W16^(n2 k1)
    const float2 w1{c1, -s1}, w2{c2, -c2}, w3{s1, -c1}, w4{0.0f, -1.0f}, w6{-c2, -c2},
        w9{-c1, s1};
    v[1 + 4] = cmul(v[1 + 4], w1);
    v[1 + 8] = cmul(v[1 + 8], w2);
    v[1 + 12] = cmul(v[1 + 12], w3);
    v[2 + 4] = cmul(v[2 + 4], w2);
    v[2 + 8] = cmul(v[2 + 8], w4);
    v[2 + 12] = cmul(v[2 + 12], w6);
    v[3 + 4] = cmul(v[3 + 4], w3);
    v[3 + 8] = cmul(v[3 + 8], w6);
    v[3 + 12] = cmul(v[3 + 12], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4x4 index to natural order
    float2 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = t[k];
}

__device__ __forceinline__ void block_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ void dma16(const void *src, uint32_t lds_wave_base) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_wave_base)), "v"(src)
                 : "memory", "m0");
}

__device__ __forceinline__ int8_t requant(float v, float s) {
    float r = rintf(s * v);  // round half to even
    r = fminf(fmaxf(r, -127.0f), 127.0f);
    return (int8_t)r;
}

template <bool CI8>
__global__ __launch_bounds__(kThreads, 1) void fengine_kernel(
    const int8_t *__restrict__ in, int ninput, int nspec, int ngroup, int total_flat,
    const float *__restrict__ scale, void *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    // XCD-aware order: the groups of one frame share its rows in L2
    const int B = blockIdx.x;
    if (B >= total_flat) return;
    const int sq = B >> 3;
    const int fl = sq / ngroup;
    const int g = sq - fl * ngroup;
    const int s = fl * 8 + (B & 7);
    if (s >= nspec) return;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int team = wave >> 2;
    const int j = tid & (kTeamLanes - 1);  // lane within the team
    uint8_t *smp = lds;                    // [4096 rows][16 bytes]
    float2 *fft = (float2 *)(lds + kInBytes + team * kFftBytes);
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;

    // ---- samples of the 16 inputs of this frame: rows 4096 s + t
    const int i0 = g * kGroup;
    const int8_t *src = in + ((int64_t)s * kN) * ninput + i0;
#pragma unroll
    for (int c = 0; c < kN / 64 / 8; ++c) {  // 8 DMA instructions per wave
        const int row0 = (wave * (kN / 64 / 8) + c) * 64;
        dma16(src + (int64_t)(row0 + lane) * ninput, lds_base + row0 * kGroup);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    block_barrier();

    const float2 *tw = g_twiddle;
#pragma unroll 1
    for (int pr = 0; pr < kPairs / kTeams; ++pr) {
        const int p = team * (kPairs / kTeams) + pr;  // pair handled by this team
        // pass 1 (Ns = 1): z[n] = x_a[n] + i x_b[n], n = j + 256 r
        float2 v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint16_t two = *(const uint16_t *)(smp + (j + 256 * r) * kGroup + 2 * p);
            v[r] = float2{(float)(int8_t)(two & 0xFF), (float)(int8_t)(two >> 8)};
        }
        dft16(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) fft[pad(16 * j + r)] = v[r];
        block_barrier();
        // pass 2 (Ns = 16) and pass 3 (Ns = 256)
#pragma unroll
        for (int ps = 0; ps < 2; ++ps) {
            const int Ns = ps == 0 ? 16 : 256;
            const int k = j & (Ns - 1);
            const int mstep = k * (kN / (16 * Ns));  // twiddle index step
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = fft[pad(j + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw[(r * mstep) & (kN - 1)]);
            }
            block_barrier();  // every read of this pass is done
            dft16(v);
            const int base = (j / Ns) * 16 * Ns + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) fft[pad(base + r * Ns)] = v[r];
            block_barrier();
        }
        // two-for-one split for k = j + 256 c, c = 0..7
#pragma unroll
        for (int c = 0; c < kChan / kTeamLanes; ++c) {
            const int k = j + kTeamLanes * c;
            const float2 z = fft[pad(k)];
            const float2 w = fft[pad((kN - k) & (kN - 1))];
            // X_a = (z + conj w)/2, X_b = (z - conj w)/(2i) = -i (z - conj w)/2
            const float2 xa{0.5f * (z.x + w.x), 0.5f * (z.y - w.y)};
            const float2 xb{0.5f * (z.y + w.y), -0.5f * (z.x - w.x)};
            if (CI8) {
                const float sc = scale[k];
                const int8_t ar = requant(xa.x, sc), ai = requant(xa.y, sc);
                const int8_t br = requant(xb.x, sc), bi = requant(xb.y, sc);
                // park in this pair's consumed sample bytes: rows 2k (a), 2k+1 (b)
                *(uint16_t *)(smp + (2 * k) * kGroup + 2 * p) =
                    (uint16_t)((uint8_t)ar | ((uint16_t)(uint8_t)ai << 8));
                *(uint16_t *)(smp + (2 * k + 1) * kGroup + 2 * p) =
                    (uint16_t)((uint8_t)br | ((uint16_t)(uint8_t)bi << 8));
            } else {
                float4 *o = (float4 *)((float *)out + (((int64_t)s * kChan + k) * ninput + i0 + 2 * p) * 2);
                *o = float4{xa.x, xa.y, xb.x, xb.y};
            }
        }
        block_barrier();  // the team's buffer is reused by the next pair
    }

    if (CI8) {
        // ci8 block [k][16 inputs][re, im]: interleave rows 2k (inputs 2p) and
        // 2k+1 (inputs 2p+1) into 32-byte output segments
        int8_t *o = (int8_t *)out;
#pragma unroll
        for (int c = 0; c < kChan / kThreads; ++c) {
            const int k = tid + kThreads * c;
            const uint4 a = *(const uint4 *)(smp + (2 * k) * kGroup);
            const uint4 b = *(const uint4 *)(smp + (2 * k + 1) * kGroup);
            uint4 lo, hi;
            lo.x = __builtin_amdgcn_perm(b.x, a.x, 0x05040100u);
            lo.y = __builtin_amdgcn_perm(b.x, a.x, 0x07060302u);
            lo.z = __builtin_amdgcn_perm(b.y, a.y, 0x05040100u);
            lo.w = __builtin_amdgcn_perm(b.y, a.y, 0x07060302u);
            hi.x = __builtin_amdgcn_perm(b.z, a.z, 0x05040100u);
            hi.y = __builtin_amdgcn_perm(b.z, a.z, 0x07060302u);
            hi.z = __builtin_amdgcn_perm(b.w, a.w, 0x05040100u);
            hi.w = __builtin_amdgcn_perm(b.w, a.w, 0x07060302u);
            uint4 *dst = (uint4 *)(o + (((int64_t)s * kChan + k) * ninput + i0) * 2);
            dst[0] = lo;
            dst[1] = hi;
        }
    }
}

std::mutex g_mu;
bool g_ready[64];

hipError_t init_device() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ready[dev]) return hipSuccess;
    static float2 host[kN];
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < kN; ++m) {
        host[m].x = (float)cos(two_pi * m / kN);
        host[m].y = (float)-sin(two_pi * m / kN);
    }
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle), host, sizeof host, 0, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)fengine_kernel<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)fengine_kernel<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    g_ready[dev] = true;
    return hipSuccess;
}

}  // namespace

bool fengine_supported(int32_t ninput, int32_t nfft) { return nfft == kN && ninput % kGroup == 0; }

hipError_t launch_fengine(const int8_t *in, int32_t ninput, int32_t nfft, int64_t nspec,
                          const float *scale, void *out, bool ci8, hipStream_t s) {
    if (!fengine_supported(ninput, nfft)) return hipErrorNotSupported;
    hipError_t e = init_device();
    if (e != hipSuccess) return e;
    const int ngroup = ninput / kGroup;
    const int64_t nspec8 = (nspec + 7) / 8 * 8;
    const int64_t total = nspec8 * ngroup;
    if (total > INT32_MAX) return hipErrorInvalidValue;
    if (ci8)
        hipLaunchKernelGGL(fengine_kernel<true>, dim3((unsigned)total), dim3(kThreads), kLdsBytes,
                           s, in, ninput, (int)nspec, ngroup, (int)total, scale, out);
    else
        hipLaunchKernelGGL(fengine_kernel<false>, dim3((unsigned)total), dim3(kThreads), kLdsBytes,
                           s, in, ninput, (int)nspec, ngroup, (int)total, scale, out);
    return hipGetLastError();
}

}  // namespace bfx
