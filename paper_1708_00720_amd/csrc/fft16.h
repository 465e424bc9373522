// Radix-16 building blocks of the FFT kernels (F-engine and T-engine):
// complex multiply, forward 4- and 16-point DFTs in registers, the padded
// LDS indices of the Stockham exchanges and the exchanges' workgroup barrier.
#pragma once
#include <hip/hip_runtime.h>

namespace bfx {
namespace {

// Padded float2 index of the 4096-point exchange buffers.  For 32 consecutive
// lanes j and a fixed r, 8-byte accesses at these indices fall on 64
// distinct banks; both paddings are additive, so a lane's 16 accesses of an
// exchange differ by constants and fold into the instructions' offsets.
//   pad_a: pass-1 writes 16 j + r and the reads j + 256 r that follow;
//   pad_b: writes (j / 16) 256 + j % 16 + 16 r and the reads j + 256 r.
// The LDS serves 8-byte writes 16 lanes at a time over 32 banks; there the
// pad_a writes put two lanes on each bank pair (a two-way conflict on the
// pass-1 writes only).  The XOR swizzle x ^ ((x >> 4) & 15) avoids it at two
// vector operations per write; both kernels time the same either way.
constexpr int kPadAElems = 4096 + 4096 / 32;
constexpr int kPadBElems = 4096 + 3 * (4096 / 64) + 2 * (4096 / 128);
__device__ __forceinline__ int pad_a(int x) { return x + (x >> 5); }
__device__ __forceinline__ int pad_b(int x) { return x + 3 * (x >> 6) + 2 * (x >> 7); }

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

// Workgroup barrier of an LDS exchange: the wave's LDS writes are complete
// (lgkmcnt = 0; vmcnt and expcnt left at their maxima) before it arrives, so
// every wave past the barrier reads them.  gfx950 does not wait for
// outstanding memory operations at s_barrier by itself, and no release fence
// is needed beyond that (the exchange is LDS only).
__device__ __forceinline__ void block_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

}  // namespace
}  // namespace bfx
