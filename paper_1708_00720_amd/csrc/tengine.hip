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
// inverse transform is taken as swap(FFT(swap X)), swap(a + ib) = b + ia
// (= i conj(a + ib), so swap(FFT(swap X)) = conj(FFT(conj X)) = N IFFT(X);
// the swaps are register renamings, no arithmetic), with the forward radix-16
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

// Quantize: round half to even, saturated to +-lim, returned as the low bits
// of a binary32 bit pattern.  v + 1.5 2^23 rounds v to an integer n once
// (|v| < 2^22 keeps the sum in [2^23, 2^24), where the spacing is 1, and
// 1.5 2^23 is even, so ties go to even n) and leaves 1.5 2^23 + n, whose bit
// pattern is 0x4B400000 + n; clamping that float to 1.5 2^23 +- lim
// saturates n, and every |v| >= 2^22 lands outside the clamp range on the
// correct side.  The low byte is n as int8, the low nibble n as int4.
__device__ __forceinline__ uint32_t quant_bits(float v, float lim) {
    constexpr float kMagic = 12582912.0f;
    return __float_as_uint(__builtin_amdgcn_fmed3f(v + kMagic, kMagic - lim, kMagic + lim));
}

// Sample loads: raw buffer access, a uniform base in a buffer descriptor
// (scalar registers) plus a lane's 32-bit offset and a uniform 32-bit offset.
// Descriptor word 3: 32-bit data format (required by gfx9 for raw buffer
// access); no range is enforced below 2^32.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t frame_rsrc(const void *base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)0xFFFFFFFFu, 0x00020000);
}

// Output stores go through global (not buffer) stores: a uniform base kept
// whole in scalar registers plus the lane's 32-bit offset.  (A 16-byte buffer
// store with a scalar offset register gets no wait state before its data
// registers are overwritten.)
#define BFX_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ BFX_GLOBAL T *uniform_ptr(T *p) {
    uint64_t u = (uint64_t)p;
    asm volatile("" : "+s"(u));
    return (BFX_GLOBAL T *)u;
}
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

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
    // 32-bit per-lane offsets within a frame (a frame spans < 2^32 bytes of
    // input and of output): input row j of the band, output row j
    const uint32_t joff = (uint32_t)(j * ninput) * 2u;
    const uint32_t ooff = (uint32_t)(j * ninput) * (CI4 ? 1u : 2u);

    for (int B = blockIdx.x; B < total_flat; B += gridDim.x) {
        int s, g;
        if (!item_of(B, ngroup, nspec, s, g)) continue;
        const int i0 = g * kGroup;
        uint4 xs[16];
        {
            // frame s, channel chan0, input i0 (uniform); rows j + 256 r
            const __amdgpu_buffer_rsrc_t rs = frame_rsrc(in + (((int64_t)s * nchan + chan0) * ninput + i0) * 2);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, joff, 256 * r * ninput * 2, 0);
                xs[r] = uint4{(uint32_t)w[0], (uint32_t)w[1], (uint32_t)w[2], (uint32_t)w[3]};
            }
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
                // swap(X): the inverse transform as swap(FFT(swap X))
                v[r] = float2{(float)(int8_t)((two >> 8) & 0xFF), (float)(int8_t)(two & 0xFF)};
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
            // v[r] = FFT(swap X)[n], n = j + 256 r:  z = swap(v) (-1)^n / N, and
            // scale z e^{i phase} = swap(v) w with w = E_r ph0 (sign, 1/N, scale in
            // ph0).  w is formed anew for each input: hoisted out of the input
            // loop, its 16 values would take 32 more registers than there are.
            asm volatile("" : "+v"(ph0.x), "+v"(ph0.y));
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 w = cmul(E.e[r], ph0);
                const float2 zm{v[r].y * w.x - v[r].x * w.y, v[r].y * w.y + v[r].x * w.x};
                const uint32_t qr = quant_bits(zm.x, lim), qi = quant_bits(zm.y, lim);
                if (CI4) {
                    // byte (re << 4) | im of input ii into byte ii % 4 of word
                    // ii / 4 (v_perm: bytes below from the word, the new byte
                    // from b, bytes above cleared)
                    const uint32_t b = (qr << 4) | (qi & 15u);
                    constexpr uint32_t kIns[4] = {0x0c0c0c04u, 0x0c0c0400u, 0x0c040100u, 0x04020100u};
                    const int w = ii >> 2;
                    code[r][w] = __builtin_amdgcn_perm(b, (ii & 3) == 0 ? 0u : code[r][w], kIns[ii & 3]);
                } else {
                    // (re, im) bytes of input ii into half ii % 2 of word ii / 2
                    const uint32_t h = __builtin_amdgcn_perm(qi, qr, 0x0c0c0400u);
                    const int w = ii >> 1;
                    code[r][w] = (ii & 1) == 0 ? h : __builtin_amdgcn_perm(h, code[r][w], 0x05040100u);
                }
            }
        }
        // rows t = s N + j + 256 r, the item's 8 inputs
        uint8_t *orow = out + ((int64_t)s * kN * ninput + i0) * (CI4 ? 1 : 2);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t roff = (uint32_t)(256 * r * ninput) * (CI4 ? 1u : 2u);
            if (CI4) {
                *(BFX_GLOBAL v2u *)(uniform_ptr(orow + roff) + ooff) = v2u{code[r][0], code[r][1]};
            } else {
                *(BFX_GLOBAL v4u *)(uniform_ptr(orow + roff) + ooff) =
                    v4u{code[r][0], code[r][1], code[r][2], code[r][3]};
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
