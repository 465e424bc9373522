// Batched X-engine without any allocation, for callers that cannot allocate
// device memory (code under graph capture, tight serving loops).  The batched
// plan keeps its subarray table and work list in device memory it allocates
// at creation; this entry point builds both per call, on the device, in a
// file-scope scratch array of fixed size, and then runs the same batched
// kernel.  Every call on one device shares that device's array: calls that
// overlap on one device (different streams, or host threads) race.
//
// Work list.  Subarrays are ordered by items per group, largest first (a
// group is one channel with all its triangle items, or up to four channels
// of a one-block subarray packed into one item), and group g of that order
// goes to XCD queue g % 8.  The host passes, per subarray and queue, the
// number of queue entries that earlier subarrays put there; a build kernel
// then places every item in closed form and pads the shorter queues.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "bfx_internal.h"

namespace bfx {
namespace {

constexpr int kStaticMaxSub = 16;
constexpr int64_t kStaticMaxWork = (int64_t)1 << 16;  // work-list entries
constexpr size_t kUnitsBytes = ((kStaticMaxSub * sizeof(BatchUnit)) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kUnitsBytes + kStaticMaxWork * sizeof(int2);

// The scratch array (subarray table, then the work list).  Host code uses the
// per-device address from hipGetSymbolAddress, never this name.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

// Per-subarray record of the build, in sorted order j.
struct BuildSub {
    int32_t k;        // subarray index (its record in the table)
    int32_t ngroups;  // groups of this subarray
    int32_t size;     // items per group (1 for packed groups)
    int32_t packed;   // one-block subarray: groups of up to four channels
    int32_t nchan;
    int32_t g0;       // first global group index
    int32_t item0;    // first item index (prefix of ngroups * size)
    int32_t base[8];  // queue entries placed by subarrays 0 .. j-1, per queue
};

struct BuildArgs {
    BatchUnit units[kStaticMaxSub];  // in subarray order k
    BuildSub sub[kStaticMaxSub];     // in sorted order j
    int32_t nsub;
    int32_t qlen[8];                 // final queue lengths
    int32_t len;                     // entries per queue after padding
    int32_t nitems;                  // real items
};

// One thread per work-list slot: first the padding slots, then the items.
__global__ __launch_bounds__(256) void build_work_kernel(BuildArgs a, BatchUnit *units, int2 *work) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < a.nsub) units[tid] = a.units[tid];
    const int64_t npad = 8LL * a.len;
    for (int64_t e = tid; e < npad; e += stride) {
        const int x = (int)(e & 7);
        const int p = (int)(e >> 3);
        if (p >= a.qlen[x]) work[e] = int2{-1, 0};
    }
    for (int64_t t = tid; t < a.nitems; t += stride) {
        int j = 0;
        while (j + 1 < a.nsub && a.sub[j + 1].item0 <= t) ++j;
        const BuildSub &s = a.sub[j];
        const int idx = (int)(t - s.item0);
        const int c = idx / s.size;
        const int it = idx - c * s.size;
        const int g = s.g0 + c;
        const int x = g & 7;
        const int p = s.base[x] + (c >> 3) * s.size + it;
        int2 e;
        if (s.packed) {
            const int f0 = 4 * c;
            const int n = min(4, s.nchan - f0);
            e = int2{s.k | (n << kBatchSubBits) | kBatchPacked, f0};
        } else {
            e = int2{s.k | (it << kBatchSubBits), c};
        }
        work[8LL * p + x] = e;
    }
}

// Device address of `scratch` on each device, from hipGetSymbolAddress taken
// once with that device current (retried on a later call if it failed).
std::mutex g_mu;
void *g_scratch[kMaxDevices];

hipError_t scratch_of(int dev, uint8_t **p) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = q;
    }
    *p = (uint8_t *)g_scratch[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace bfx

using namespace bfx;

extern "C" {

bfx_status bfx_xengine_accumulate_batched_noalloc(int32_t nsub, const int32_t *ninput, const int32_t *nchan,
                                                  bfx_dtype in, const void *d_in, int64_t ntime, void *d_acc,
                                                  uint32_t flags, bfx_stream stream) {
    if (nsub <= 0 || nsub > kStaticMaxSub || !ninput || !nchan)
        return fail(BFX_EINVAL, "nsub=%d must be in [1, %d] with non-NULL size arrays", nsub, kStaticMaxSub);
    if (in != BFX_CI4 && in != BFX_CI8) return fail(BFX_ENOTSUP, "the batched X-engine takes ci4 or ci8 input");
    if (!d_in || !d_acc || ((uintptr_t)d_in & 15u) || ((uintptr_t)d_acc & 15u))
        return fail(BFX_EINVAL, "d_in / d_acc must be non-NULL and 16-byte aligned");
    if (flags != BFX_ACC_OVERWRITE)
        return fail(BFX_ENOTSUP, "this entry point keeps no integration state: every call overwrites "
                                 "(flags must be BFX_ACC_OVERWRITE)");
    const int64_t tmax = bfx_xengine_max_ntime(in);
    if (ntime <= 0 || ntime > tmax)
        return fail(ntime <= 0 ? BFX_EINVAL : BFX_ERANGE, "ntime=%lld must be in [1, %lld]",
                    (long long)ntime, (long long)tmax);
    const int64_t sb = in == BFX_CI4 ? 1 : 2;
    BuildArgs a;
    memset(&a, 0, sizeof a);
    a.nsub = nsub;
    int64_t io = 0, oo = 0;
    for (int32_t k = 0; k < nsub; ++k) {
        if (ninput[k] <= 0 || ninput[k] > 8192 || ninput[k] % 4 || nchan[k] <= 0 || nchan[k] > 65536)
            return fail(BFX_EINVAL, "subarray %d: ninput=%d must be a positive multiple of 4 <= 8192 and "
                                    "nchan=%d in [1, 65536]", k, ninput[k], nchan[k]);
        BatchUnit &u = a.units[k];
        u.in_row_off = io;
        u.t_stride = (int64_t)nchan[k] * ninput[k] * sb;
        u.out_off = oo;
        u.nchan = nchan[k];
        u.ninput = ninput[k];
        u.nb = (ninput[k] + 63) / 64;
        u.nitems = (int32_t)xengine_items(ninput[k], 1);
        io += (u.t_stride + 255) / 256 * 256;
        oo += ((int64_t)nchan[k] * ninput[k] * (ninput[k] + 1) / 2 * 8 + 255) / 256 * 256;
    }
    // sorted order: items per group, largest first (packed groups count one)
    int32_t order[kStaticMaxSub];
    for (int32_t k = 0; k < nsub; ++k) order[k] = k;
    std::stable_sort(order, order + nsub, [&](int32_t x, int32_t y) {
        const int32_t sx = a.units[x].nb == 1 ? 1 : a.units[x].nitems;
        const int32_t sy = a.units[y].nb == 1 ? 1 : a.units[y].nitems;
        return sx > sy;
    });
    int64_t g0 = 0, item0 = 0, qlen[8] = {};
    for (int32_t j = 0; j < nsub; ++j) {
        const BatchUnit &u = a.units[order[j]];
        BuildSub &s = a.sub[j];
        s.k = order[j];
        s.packed = u.nb == 1;
        s.size = s.packed ? 1 : u.nitems;
        s.ngroups = s.packed ? (u.nchan + 3) / 4 : u.nchan;
        s.nchan = u.nchan;
        s.g0 = (int32_t)g0;
        s.item0 = (int32_t)item0;
        for (int x = 0; x < 8; ++x) {
            s.base[x] = (int32_t)qlen[x];
            // groups c of this subarray with (g0 + c) % 8 == x
            const int r = (int)(((x - g0) % 8 + 8) % 8);
            const int64_t cnt = s.ngroups > r ? (s.ngroups - r + 7) / 8 : 0;
            qlen[x] += cnt * s.size;
        }
        g0 += s.ngroups;
        item0 += (int64_t)s.ngroups * s.size;
        if (item0 > kStaticMaxWork)
            return fail(BFX_ENOTSUP, "more than %lld work items: use a batched plan", (long long)kStaticMaxWork);
    }
    int64_t len = 0;
    for (int x = 0; x < 8; ++x) {
        a.qlen[x] = (int32_t)qlen[x];
        len = std::max(len, qlen[x]);
    }
    if (8 * len > kStaticMaxWork)
        return fail(BFX_ENOTSUP, "the work list needs %lld entries, more than the %lld this entry point "
                                 "holds: use a batched plan", (long long)(8 * len), (long long)kStaticMaxWork);
    a.len = (int32_t)len;
    a.nitems = (int32_t)item0;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(BFX_EHIP, "device %d beyond this build's %d", dev, kMaxDevices);
    uint8_t *base = nullptr;
    e = scratch_of(dev, &base);
    if (e != hipSuccess) return hip_fail(e, "locating the scratch array");
    BatchUnit *d_units = (BatchUnit *)base;
    int2 *d_work = (int2 *)(base + kUnitsBytes);
    hipStream_t s = (hipStream_t)stream;
    const int64_t nslots = std::max<int64_t>(8 * len, nsub);
    const unsigned blocks = (unsigned)std::min<int64_t>((nslots + 255) / 256, 1024);
    hipLaunchKernelGGL(build_work_kernel, dim3(blocks), dim3(256), 0, s, a, d_units, d_work);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "work-list build launch");
    const bool ci4 = in == BFX_CI4;
    for (int64_t t0 = 0; t0 < ntime && e == hipSuccess; t0 += kLaunchMaxTime) {
        const int64_t nt = ntime - t0 < kLaunchMaxTime ? ntime - t0 : kLaunchMaxTime;
        e = launch_xengine_batched(ci4, d_in, ntime, t0, nt, d_units, d_work, 8 * len, d_acc, t0 == 0, 0, s);
    }
    if (e != hipSuccess) return hip_fail(e, "X-engine launch");
    return BFX_OK;
}

}  // extern "C"
