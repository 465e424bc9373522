// Peak probes: how fast this device sustains the resources the hot-path
// kernels are priced against.  They compute nothing of the method; they exist
// so that the roofline fractions can be quoted against a measured rate beside
// the published peak.
//
//   mfma probe: every wave keeps 8 independent accumulators and issues
//               back-to-back MFMAs (int8 32x32x32 or binary16 32x32x16) with
//               no memory traffic: the sustainable dense MFMA rate.
//   read probe: a grid covering the buffer streams it once with 16-byte loads
//               and folds it to one word per workgroup: the sustainable HBM
//               read rate.
//   lds probe:  every wave issues back-to-back LDS reads of one kind
//               (transposing 8-byte reads as the X-engines issue them, or
//               plain 16-byte reads) from a 16 KiB buffer: the LDS read
//               bandwidth per CU that those kernels' stages are bound by.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bfx_probe.h"
#include "bfx_internal.h"

namespace bfx {
namespace {

typedef int pv4i __attribute__((ext_vector_type(4)));
typedef int pv16i __attribute__((ext_vector_type(16)));
typedef _Float16 pv8h __attribute__((ext_vector_type(8)));
typedef float pv16f __attribute__((ext_vector_type(16)));

constexpr int kProbeThreads = 512;  // 8 waves, two per SIMD

__global__ __launch_bounds__(kProbeThreads) void mfma_i8_probe(int iters, int seed, int *sink) {
    const pv4i a = {seed + (int)threadIdx.x, seed * 3, seed ^ 5, 7};
    const pv4i b = {seed * 7, (int)threadIdx.x, 11, seed + 1};
    pv16i acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = pv16i{0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[k], 0, 0, 0);
    }
    int r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) r ^= acc[k][v];
    if (r == 0x7fffffff) sink[blockIdx.x] = r;  // keeps the loop live; practically never taken
}

__global__ __launch_bounds__(kProbeThreads) void mfma_f16_probe(int iters, int seed, int *sink) {
    pv8h a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (_Float16)((seed + k + (int)threadIdx.x) & 7);
        b[k] = (_Float16)((seed * k) & 3);
    }
    pv16f acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = pv16f{0.0f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[k], 0, 0, 0);
    }
    float r = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) r += acc[k][v];
    if (r == -1.0f) sink[blockIdx.x] = 1;  // never taken for non-negative data
}

__global__ __launch_bounds__(256) void read_probe(const uint4 *__restrict__ buf, int64_t n16, int *sink) {
    uint32_t x = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride) {
        const uint4 v = buf[k];
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // one word per workgroup (written only when the fold is non-zero, so a
    // zero buffer writes nothing)
    __shared__ uint32_t red[256];
    red[threadIdx.x] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] ^= red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) sink[blockIdx.x] = (int)red[0];
}

typedef short pv4s __attribute__((ext_vector_type(4)));
typedef int pv2i __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) pv4s lds_pv4s;
typedef __attribute__((address_space(3))) pv2i lds_pv2i;

constexpr int kLdsProbeBytes = 16384;
constexpr int kLdsProbeReads = 12;  // reads per iteration and wave

template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void lds_probe(int iters, int *sink) {
    __shared__ __attribute__((aligned(16))) uint8_t buf[kLdsProbeBytes];
    const int lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kLdsProbeBytes / 4; i += blockDim.x) ((uint32_t *)buf)[i] = i * 2654435761u;
    __syncthreads();
    // The FP16 X-engine's fragment read: 16-lane group G reads 4 rows of
    // 1 KiB (rows 8 (G >> 1) + k / 4), 8 bytes per lane, chunks XOR-swizzled
    // by the row -- conflict-free.  Every iteration shifts all lanes by a
    // multiple of 64 bytes, which keeps it so.
    const int G = (lane >> 4) & 3, k = lane & 15;
    const int t = 8 * (G >> 1) + (k >> 2);
    const int byte = 32 * (G & 1) + 8 * (k & 3);
    const int tr_base = t * 1024 + 16 * ((byte >> 4) ^ ((t & 3) << 2)) + (byte & 15);
    int acc = 0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < kLdsProbeReads; ++r) {
            if constexpr (KIND == BFX_PROBE_LDS_B128) {
                const int off = (lane * 16 + r * 1024 + (it & 7) * 16) & (kLdsProbeBytes - 16);
                const pv4i v = *(const pv4i *)(buf + off);
                acc ^= v.x ^ v.y ^ v.z ^ v.w;
            } else {
                // tr_base <= 11512, so off + 8 <= 13120: inside the buffer
                const int off = tr_base + r * 64 + (it & 7) * 128;
                if constexpr (KIND == BFX_PROBE_LDS_TR16) {
                    const pv4s v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_pv4s *)(buf + off));
                    const pv2i w = __builtin_bit_cast(pv2i, v);
                    acc ^= w.x ^ w.y;
                } else {
                    const pv2i w = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_pv2i *)(buf + off));
                    acc ^= w.x ^ w.y;
                }
            }
        }
    }
    if (acc == 0x7fffffff) sink[blockIdx.x] = acc;  // keeps the reads live; practically never taken
}

DeviceInit g_init;

hipError_t no_init() { return hipSuccess; }

}  // namespace
}  // namespace bfx

using namespace bfx;

extern "C" {

int64_t bfx_probe_mfma_ops(int32_t kind, int32_t iters, int32_t nblocks) {
    if ((kind != BFX_PROBE_MFMA_I8 && kind != BFX_PROBE_MFMA_F16) || iters <= 0 || nblocks <= 0) return -1;
    // per MFMA: 32 x 32 x K multiply-adds, 2 ops each (K = 32 int8, 16 binary16)
    const int64_t per = 2LL * 32 * 32 * (kind == BFX_PROBE_MFMA_I8 ? 32 : 16);
    return per * 8 * (kProbeThreads / 64) * (int64_t)iters * nblocks;
}

bfx_status bfx_probe_mfma(int32_t kind, int32_t iters, int32_t nblocks, int32_t *d_sink, bfx_stream stream) {
    if (kind != BFX_PROBE_MFMA_I8 && kind != BFX_PROBE_MFMA_F16)
        return fail(BFX_EINVAL, "probe kind %d is not BFX_PROBE_MFMA_I8 or BFX_PROBE_MFMA_F16", kind);
    if (iters <= 0 || nblocks <= 0 || nblocks > (1 << 20) || !d_sink)
        return fail(BFX_EINVAL, "iters and nblocks (<= 2^20) must be positive, d_sink non-NULL");
    hipError_t e = g_init.ensure(no_init, nullptr);
    if (e != hipSuccess) return hip_fail(e, "probe set-up");
    if (kind == BFX_PROBE_MFMA_I8)
        hipLaunchKernelGGL(mfma_i8_probe, dim3(nblocks), dim3(kProbeThreads), 0, (hipStream_t)stream, iters,
                           nblocks, d_sink);
    else
        hipLaunchKernelGGL(mfma_f16_probe, dim3(nblocks), dim3(kProbeThreads), 0, (hipStream_t)stream, iters,
                           nblocks, d_sink);
    e = hipGetLastError();
    return e == hipSuccess ? BFX_OK : hip_fail(e, "MFMA probe launch");
}

int64_t bfx_probe_lds_bytes(int32_t kind, int32_t iters, int32_t nblocks) {
    if (kind < BFX_PROBE_LDS_TR16 || kind > BFX_PROBE_LDS_B128 || iters <= 0 || nblocks <= 0) return -1;
    const int64_t per_lane = kind == BFX_PROBE_LDS_B128 ? 16 : 8;
    return per_lane * kProbeThreads * kLdsProbeReads * (int64_t)iters * nblocks;
}

bfx_status bfx_probe_lds(int32_t kind, int32_t iters, int32_t nblocks, int32_t *d_sink, bfx_stream stream) {
    if (kind < BFX_PROBE_LDS_TR16 || kind > BFX_PROBE_LDS_B128)
        return fail(BFX_EINVAL, "probe kind %d is not an LDS read kind", kind);
    if (iters <= 0 || nblocks <= 0 || nblocks > (1 << 20) || !d_sink)
        return fail(BFX_EINVAL, "iters and nblocks (<= 2^20) must be positive, d_sink non-NULL");
    const hipStream_t s = (hipStream_t)stream;
    if (kind == BFX_PROBE_LDS_TR16)
        hipLaunchKernelGGL(lds_probe<BFX_PROBE_LDS_TR16>, dim3(nblocks), dim3(kProbeThreads), 0, s, iters, d_sink);
    else if (kind == BFX_PROBE_LDS_TR8)
        hipLaunchKernelGGL(lds_probe<BFX_PROBE_LDS_TR8>, dim3(nblocks), dim3(kProbeThreads), 0, s, iters, d_sink);
    else
        hipLaunchKernelGGL(lds_probe<BFX_PROBE_LDS_B128>, dim3(nblocks), dim3(kProbeThreads), 0, s, iters, d_sink);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BFX_OK : hip_fail(e, "LDS probe launch");
}

bfx_status bfx_probe_read(const void *d_buf, int64_t nbytes, int32_t nblocks, int32_t *d_sink,
                          bfx_stream stream) {
    if (!d_buf || !d_sink || ((uintptr_t)d_buf & 15u) || nbytes <= 0 || (nbytes & 15))
        return fail(BFX_EINVAL, "d_buf must be 16-byte aligned with nbytes a positive multiple of 16");
    if (nblocks <= 0 || nblocks > (1 << 23))
        return fail(BFX_EINVAL, "nblocks=%d must be in [1, 2^23]", nblocks);
    hipLaunchKernelGGL(read_probe, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, (const uint4 *)d_buf,
                       nbytes / 16, d_sink);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BFX_OK : hip_fail(e, "read probe launch");
}

}  // extern "C"
