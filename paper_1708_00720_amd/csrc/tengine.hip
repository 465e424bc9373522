// T-engine for gfx950: channelized ci8 spectra back to a complex time series
// (Sec. 6: the TBN pipeline's T-engine and the DRX T-engine, which carries
// out its inverse transform on the GPU).  Per frame s and input i:
//   X_k   = x[s][chan0 + k][i],  k = 0 .. nfft-1            (band selection)
//   z[n]  = (1/nfft) sum_k X_k exp(+2 pi i (k - nfft/2) n / nfft)
//                                       (channel shift: band centre at DC)
//   z'[n] = z[n] exp(+2 pi i ((mix_num t) mod mix_den) / mix_den),
//           t = s nfft + n                     (complex mixer, phase runs on)
//   q     = clamp(round_half_even(scale z'), -L, L) per component,
//           L = 127 (8+8 output) or 7 (4+4 output)
// computed in binary32.
//
// The shift multiplies the inverse transform by exp(-i pi n) = (-1)^n.  The
// inverse transform is taken as conj(FFT(conj X)) with the forward radix-16
// Stockham machinery of the F-engine: 4096 = 16^3, 256 lanes with 16 points
// each, three passes.  The third pass leaves output n = j + 256 r in lane j's
// register r, so the shift, the mixer and the quantization run in registers
// and each transform exchanges through LDS twice (two barriers).
//
// Organisation.  Persistent grid, two workgroups per CU; a work item is one
// frame of 8 adjacent inputs (frames on an XCD by s % 8, so neighbouring
// input groups meet in one L2).  A lane loads its 16 rows of the band for the
// item's 8 inputs (16 bytes per row), transforms the 8 inputs in turn, and
// keeps its output codes of all 8 inputs in registers, so each output row
// segment [t][8 inputs] leaves as one store.  The mixer phase index
// (mix_num t) mod mix_den is exact integer arithmetic: a lane's phasor of its
// first output comes from it, and the phasors of its later outputs (256
// samples apart) are that one times lane-independent factors.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bfx_internal.h"
#include "fft16.h"

namespace bfx {
namespace {

constexpr int kN = 4096;
constexpr int kGroup = 8;
constexpr int kThreads = 256;
constexpr int kABytes = kPadAElems * 8;  // pass 1 -> 2 (pad_a)
constexpr int kBBytes = kPadBElems * 8;  // pass 2 -> 3 (pad_b)
constexpr int kLdsBytes = kABytes + kBBytes;

__device__ float2 g_tw[kN];  // exp(-2 pi i m / 4096), m = 0..4095

__device__ __forceinline__ bool item_of(int B, int ngroup, int nspec, int &s, int &g) {
    const int sq = B >> 3;
    const int fl = sq / ngroup;
    g = sq - fl * ngroup;
    s = fl * 8 + (B & 7);
    return s < nspec;
}

__device__ __forceinline__ int quant(float v, float lim) {
    return (int)fminf(fmaxf(rintf(v), -lim), lim);  // round half to even
}

// Mixer factors shared by every lane: output n = j + 256 r of a frame has
// phase index m(j) + r * ((256 mix_num) mod mix_den), so its phasor is the
// lane's phasor of r = 0 times E[r] = exp(2 pi i (r * step mod D) / D),
// computed on the host in double.
struct MixerSteps {
    float2 e[16];
};

template <bool CI4>
__global__ __launch_bounds__(kThreads, 2) void tengine_kernel(
    const int8_t *__restrict__ in, int nchan, int ninput, int nspec, int chan0, int ngroup, int total_flat,
    uint32_t mix_n, uint32_t mix_d, float inv_d, MixerSteps E, float scale, uint8_t *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int j = threadIdx.x;
    float2 *A = (float2 *)lds;
    float2 *Bf = (float2 *)(lds + kABytes);
    constexpr float lim = CI4 ? 7.0f : 127.0f;
    constexpr float inv_n = 1.0f / kN;

    float2 tw2[16], tw3[16];
    {
        const int m2 = (j & 15) * (kN / 256), m3 = j;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            tw2[r] = g_tw[(r * m2) & (kN - 1)];
            tw3[r] = g_tw[(r * m3) & (kN - 1)];
        }
    }
    // output n = j + 256 r has the shift sign (-1)^j; the sign, 1/nfft and the
    // scale ride on the lane's mixer phasor
    const float sgn_scale = ((j & 1) ? -inv_n : inv_n) * scale;

    for (int B = blockIdx.x; B < total_flat; B += gridDim.x) {
        int s, g;
        if (!item_of(B, ngroup, nspec, s, g)) continue;
        const int i0 = g * kGroup;
        uint4 xs[16];
        {
            const int8_t *src = in + (((int64_t)s * nchan + chan0 + j) * ninput + i0) * 2;
#pragma unroll
            for (int r = 0; r < 16; ++r) xs[r] = *(const uint4 *)(src + (int64_t)(256 * r) * ninput * 2);
        }
        // mixer phasor of this lane's output t = s N + j (exact phase index),
        // times the shift sign, 1/nfft and the scale
        float2 ph0;
        {
            const uint64_t t0 = (uint64_t)s * kN + j;
            const uint32_t m = (uint32_t)(((uint64_t)mix_n * (t0 % mix_d)) % mix_d);
            sincospif(2.0f * ((float)m * inv_d), &ph0.y, &ph0.x);
            ph0.x *= sgn_scale;
            ph0.y *= sgn_scale;
        }
        // codes of the 8 inputs at each of the lane's 16 outputs
        uint32_t code[16][CI4 ? 2 : 4];
#pragma unroll
        for (int ii = 0; ii < kGroup; ++ii) {
            float2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t w = ii < 2 ? xs[r].x : ii < 4 ? xs[r].y : ii < 6 ? xs[r].z : xs[r].w;
                const uint32_t two = w >> (16 * (ii & 1));
                // conj(X): the inverse transform as conj(FFT(conj X))
                v[r] = float2{(float)(int8_t)(two & 0xFF), -(float)(int8_t)((two >> 8) & 0xFF)};
            }
            dft16(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) A[pad_a(16 * j + r)] = v[r];
            block_barrier();
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = A[pad_a(j + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw2[r]);
            }
            dft16(v);
            {
                const int base = (j / 16) * 256 + (j & 15);
#pragma unroll
                for (int r = 0; r < 16; ++r) Bf[pad_b(base + r * 16)] = v[r];
            }
            block_barrier();
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = Bf[pad_b(j + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw3[r]);
            }
            dft16(v);
            // v[r] = FFT(conj X)[n], n = j + 256 r:  z = conj(v) (-1)^n / N, and
            // scale z e^{i phase} = conj(v) w with w = E_r ph0 (sign, 1/N, scale in
            // ph0).  w is formed anew for each input: hoisted out of the input
            // loop, its 16 values would take 32 more registers than there are.
            asm volatile("" : "+v"(ph0.x), "+v"(ph0.y));
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 w = cmul(E.e[r], ph0);
                const float2 zm{v[r].x * w.x + v[r].y * w.y, v[r].x * w.y - v[r].y * w.x};
                const int qr = quant(zm.x, lim), qi = quant(zm.y, lim);
                if (CI4) {
                    const uint32_t b = (((uint32_t)qr & 15u) << 4) | ((uint32_t)qi & 15u);
                    const int w = ii >> 2, sh = 8 * (ii & 3);
                    code[r][w] = (ii & 3) == 0 ? b : (code[r][w] | (b << sh));
                } else {
                    const uint32_t h = ((uint32_t)qr & 0xFFu) | (((uint32_t)qi & 0xFFu) << 8);
                    const int w = ii >> 1, sh = 16 * (ii & 1);
                    code[r][w] = (ii & 1) == 0 ? h : (code[r][w] | (h << sh));
                }
            }
        }
        // rows t = s N + j + 256 r, the item's 8 inputs
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t t = (int64_t)s * kN + j + 256 * r;
            if (CI4) {
                *(uint2 *)(out + t * ninput + i0) = uint2{code[r][0], code[r][1]};
            } else {
                *(uint4 *)(out + (t * ninput + i0) * 2) = uint4{code[r][0], code[r][1], code[r][2], code[r][3]};
            }
        }
    }
}

DeviceInit g_init;

hipError_t init_device() {
    static float2 host[kN];
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < kN; ++m) {
        host[m].x = (float)cos(two_pi * m / kN);
        host[m].y = (float)-sin(two_pi * m / kN);
    }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host, sizeof host, 0, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)tengine_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kLdsBytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)tengine_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kLdsBytes);
}

}  // namespace

bool tengine_supported(int32_t ninput, int32_t nfft) { return nfft == kN && ninput % kGroup == 0; }

hipError_t launch_tengine(const int8_t *in, int32_t nchan, int32_t ninput, int64_t nspec, int32_t chan0,
                          int32_t nfft, int64_t mix_num, int64_t mix_den, float scale, void *out, bool ci4,
                          hipStream_t s) {
    if (!tengine_supported(ninput, nfft)) return hipErrorNotSupported;
    int num_cus = 0;
    const hipError_t e = g_init.ensure(init_device, &num_cus);
    if (e != hipSuccess) return e;
    const int ngroup = ninput / kGroup;
    const int64_t total = (nspec + 7) / 8 * 8 * ngroup;
    if (total > INT32_MAX) return hipErrorInvalidValue;
    int64_t grid = (int64_t)num_cus * 2 / 8 * 8;
    if (grid < 8) grid = 8;
    if (grid > total) grid = total;
    const uint32_t d = (uint32_t)mix_den;
    const uint32_t mn = (uint32_t)(mix_num % mix_den);
    const uint64_t step = ((uint64_t)mn * 256u) % d;
    const float inv_d = (float)(1.0 / (double)d);
    MixerSteps E;
    const double two_pi = 6.283185307179586476925286766559;
    for (int r = 0; r < 16; ++r) {
        const double ph = two_pi * (double)((r * step) % d) / (double)d;
        E.e[r] = float2{(float)cos(ph), (float)sin(ph)};
    }
    if (ci4)
        hipLaunchKernelGGL(tengine_kernel<true>, dim3((unsigned)grid), dim3(kThreads), kLdsBytes, s, in, nchan,
                           ninput, (int)nspec, chan0, ngroup, (int)total, mn, d, inv_d, E, scale, (uint8_t *)out);
    else
        hipLaunchKernelGGL(tengine_kernel<false>, dim3((unsigned)grid), dim3(kThreads), kLdsBytes, s, in, nchan,
                           ninput, (int)nspec, chan0, ngroup, (int)total, mn, d, inv_d, E, scale, (uint8_t *)out);
    return hipGetLastError();
}

}  // namespace bfx
