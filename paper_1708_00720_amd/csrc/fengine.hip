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
// (4096 = 16^3, three passes, 16 points per lane in registers, the passes
// exchanging through two padded LDS buffers in turn, so each exchange needs
// one barrier), and
//   X_a[k] = (Z[k] + conj Z[-k]) / 2,   X_b[k] = (Z[k] - conj Z[-k]) / (2i).
// The samples a lane needs for the first pass (16 rows, the item's 8 inputs)
// come straight from global memory into registers, fetched one item ahead so
// that the loads overlap the current item's transforms; the twiddles of the
// lane's second- and third-pass butterflies (which depend only on the lane)
// are loaded once per workgroup into registers.  A lane's requantized bytes
// of its 8 channels stay in registers across the 4 pairs and leave as one
// 16-byte [k][8 inputs] segment per channel.  Twiddles come from a 4096-entry table
// computed once per device in FP64 on the host from the exact integer phase
// k n mod 4096, then rounded to binary32.
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
constexpr int kFftElems = kN + kN / 16;             // one pad float2 per 16
constexpr int kFftBytes = kFftElems * 8;            // 34 KiB
constexpr int kLdsBytes = 2 * kFftBytes;            // ping-pong; two workgroups per CU

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
__device__ __forceinline__ void load_samples(uint2 (&x)[16], const int8_t *in, int ninput, int s,
                                             int g, int j) {
    const int8_t *src = in + ((int64_t)s * kN + j) * ninput + g * kGroup;
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = *(const uint2 *)(src + (int64_t)(256 * r) * ninput);
}

template <bool CI8>
__global__ __launch_bounds__(kThreads, 2) void fengine_kernel(
    const int8_t *__restrict__ in, int ninput, int nspec, int ngroup, int total_flat,
    const float *__restrict__ scale, void *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int j = tid;                     // lane of the FFT
    float2 *buf0 = (float2 *)lds;          // pass 1 -> 2, pass 3 -> split
    float2 *buf1 = (float2 *)(lds + kFftBytes);  // pass 2 -> 3

    int B = blockIdx.x, s = 0, g = 0;
    bool valid = false;
    while (B < total_flat && !(valid = item_of(B, ngroup, nspec, s, g))) B += gridDim.x;
    if (!valid) return;

    // twiddles of this lane's pass-2 (Ns = 16) and pass-3 (Ns = 256) butterflies
    float2 tw2[16], tw3[16];
    {
        const int m2 = (j & 15) * (kN / 256), m3 = j;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            tw2[r] = g_twiddle[(r * m2) & (kN - 1)];
            tw3[r] = g_twiddle[(r * m3) & (kN - 1)];
        }
    }
    uint2 xs[16];
    load_samples(xs, in, ninput, s, g, j);

    while (true) {
        // next item: its samples are fetched while this one is transformed
        int Bn = B + gridDim.x, sn = 0, gn = 0;
        bool nvalid = false;
        while (Bn < total_flat && !(nvalid = item_of(Bn, ngroup, nspec, sn, gn))) Bn += gridDim.x;
        uint2 xn[16];
        if (nvalid) load_samples(xn, in, ninput, sn, gn, j);
        const int i0 = g * kGroup;

        uint32_t q[kChan / kThreads][kPairs];  // ci8 bytes (a_re, a_im, b_re, b_im)
        // Buffers: pass 1 -> A, pass 2 A -> B, pass 3 B -> A, split reads A,
        // with A and B swapping from pair to pair.  Every write then targets
        // a buffer whose last reads precede a barrier already passed, so one
        // barrier per exchange suffices (three per pair).
#pragma unroll
        for (int p = 0; p < kPairs; ++p) {
            float2 *A = (p & 1) ? buf1 : buf0;
            float2 *Bf = (p & 1) ? buf0 : buf1;
            // pass 1 (Ns = 1): z[n] = x_a[n] + i x_b[n], n = j + 256 r
            float2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t w = p < 2 ? xs[r].x : xs[r].y;  // bytes 2 p, 2 p + 1
                const uint32_t two = w >> (16 * (p & 1));
                v[r] = float2{(float)(int8_t)(two & 0xFF), (float)(int8_t)((two >> 8) & 0xFF)};
            }
            dft16(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) A[pad(16 * j + r)] = v[r];
            block_barrier();
            // pass 2 (Ns = 16): A -> B
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = A[pad(j + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw2[r]);
            }
            dft16(v);
            {
                const int base = (j / 16) * 256 + (j & 15);
#pragma unroll
                for (int r = 0; r < 16; ++r) Bf[pad(base + r * 16)] = v[r];
            }
            block_barrier();
            // pass 3 (Ns = 256): B -> A
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float2 x = Bf[pad(j + 256 * r)];
                v[r] = r == 0 ? x : cmul(x, tw3[r]);
            }
            dft16(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) A[pad(j + r * 256)] = v[r];
            block_barrier();
            // two-for-one split for k = j + 256 c, c = 0..7
#pragma unroll
            for (int c = 0; c < kChan / kThreads; ++c) {
                const int k = j + kThreads * c;
                const float2 z = A[pad(k)];
                const float2 w = A[pad((kN - k) & (kN - 1))];
                // X_a = (z + conj w)/2, X_b = (z - conj w)/(2i) = -i (z - conj w)/2
                const float2 xa{0.5f * (z.x + w.x), 0.5f * (z.y - w.y)};
                const float2 xb{0.5f * (z.y + w.y), -0.5f * (z.x - w.x)};
                if (CI8) {
                    const float sc = scale[k];
                    q[c][p] = (uint32_t)(uint8_t)requant(xa.x, sc) |
                              ((uint32_t)(uint8_t)requant(xa.y, sc) << 8) |
                              ((uint32_t)(uint8_t)requant(xb.x, sc) << 16) |
                              ((uint32_t)(uint8_t)requant(xb.y, sc) << 24);
                } else {
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
                const int k = j + kThreads * c;
                *(uint4 *)(o + (((int64_t)s * kChan + k) * ninput + i0) * 2) =
                    uint4{q[c][0], q[c][1], q[c][2], q[c][3]};
            }
        }
        if (!nvalid) break;
        B = Bn;
        s = sn;
        g = gn;
#pragma unroll
        for (int r = 0; r < 16; ++r) xs[r] = xn[r];
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
