// Dump of an integration (the paper's accumulate block, Sec. 4.1): copy the
// visibility buffer out and/or fold it into a binary64 running sum,
// run64[k] += (double)acc[k].  Memory-bound elementwise pass: 16-byte
// non-temporal loads of the accumulator, 2 x 16-byte read-modify-write of the
// running sum per thread.  One group of four elements per thread: a grid that covers the
// buffer keeps more loads in flight than a capped grid-stride loop (5.4 vs
// 5.0 TB/s on 2048 x 131,328 cf32); the loop only strides beyond 2^23
// workgroups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfx_internal.h"

namespace bfx {
namespace {

typedef int v4i32 __attribute__((ext_vector_type(4)));

template <bool IS_INT>
__global__ __launch_bounds__(256) void dump_kernel(const void *__restrict__ acc,
                                                   void *__restrict__ out,
                                                   double *__restrict__ run64, int64_t n) {
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n4; k += stride) {
        // the accumulator is read once: a non-temporal load keeps it from
        // displacing the running sum's lines, which are read and written back
        const v4i32 rv = __builtin_nontemporal_load((const v4i32 *)acc + k);
        const int4 raw = make_int4(rv.x, rv.y, rv.z, rv.w);
        if (out) ((int4 *)out)[k] = raw;
        if (run64) {
            double v0, v1, v2, v3;
            if (IS_INT) {
                v0 = raw.x; v1 = raw.y; v2 = raw.z; v3 = raw.w;
            } else {
                v0 = __int_as_float(raw.x); v1 = __int_as_float(raw.y);
                v2 = __int_as_float(raw.z); v3 = __int_as_float(raw.w);
            }
            double2 *r = (double2 *)(run64 + 4 * k);
            double2 a = r[0], b = r[1];
            a.x += v0; a.y += v1; b.x += v2; b.y += v3;
            r[0] = a;
            r[1] = b;
        }
    }
    // tail (n not a multiple of 4)
    const int64_t k = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        const int32_t raw = ((const int32_t *)acc)[k];
        if (out) ((int32_t *)out)[k] = raw;
        if (run64) run64[k] += IS_INT ? (double)raw : (double)__int_as_float(raw);
    }
}

}  // namespace

hipError_t launch_dump(bool is_int, const void *acc, void *out, double *run64, int64_t n,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n / 4 + 255) / 256;
    // grid-stride beyond 2^23 workgroups (2^31 lanes, inside a launch's limit)
    if (blocks > ((int64_t)1 << 23)) blocks = (int64_t)1 << 23;
    if (blocks < 1) blocks = 1;
    if (is_int)
        hipLaunchKernelGGL(dump_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, acc, out,
                           run64, n);
    else
        hipLaunchKernelGGL(dump_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, acc, out,
                           run64, n);
    return hipGetLastError();
}

}  // namespace bfx
