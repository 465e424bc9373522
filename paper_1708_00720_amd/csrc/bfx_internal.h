// Internal declarations shared by the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/bfx.h"

namespace bfx {

// One-time set-up of a kernel family, per device: `init` (kernel attributes,
// device tables) runs under the lock the first time a launch finds device d
// current, and is retried on a later call if it failed.  ensure() also
// returns the current device's compute-unit count.
constexpr int kMaxDevices = 64;
struct DeviceInit {
    std::mutex mu;
    bool ready[kMaxDevices] = {};
    int cus[kMaxDevices] = {};
    template <class Fn>
    hipError_t ensure(Fn &&init, int *num_cus) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
        std::lock_guard<std::mutex> lk(mu);
        if (!ready[dev]) {
            hipDeviceProp_t prop;
            e = hipGetDeviceProperties(&prop, dev);
            if (e != hipSuccess) return e;
            e = init();
            if (e != hipSuccess) return e;
            cus[dev] = prop.multiProcessorCount;
            ready[dev] = true;
        }
        if (num_cus) *num_cus = cus[dev];
        return hipSuccess;
    }
};

// Largest grid of 256-lane workgroups one launch can take: the total lane
// count of a grid dimension must stay below 2^32.
constexpr int64_t kMaxWorkgroups256 = (((int64_t)1 << 32) - 1) / 256;

// Thread-local error detail; returns `s` for convenient `return fail(...)`.
bfx_status fail(bfx_status s, const char *fmt, ...);
bfx_status hip_fail(hipError_t e, const char *what);

// Largest number of samples one integer X-engine launch may sum: the int32
// registers hold sums of products bounded by 2*128^2 per sample (ci8, and ci4
// in its 16x-scaled form), so floor((2^31-1) / 32768) = 65535.
constexpr int64_t kLaunchMaxTime = 65535;

// Integer X-engine (ci4 / ci8 -> int32 packed lower triangle) over one
// contiguous array.  `in` points at time row t0 of a [t][nchan][ninput] gulp,
// `nt` <= kLaunchMaxTime rows follow.  `overwrite` stores V, else adds.
// Kernel variants of the X-engines: 0 and 1 run the plan's own MFMA type
// with four or eight DMA waves; ci4 plans also have 2 and 3, the same with
// FP8 MFMA.  Batched plans have variants 0 and 1.
constexpr int kXengineVariants = 4;
constexpr int kBatchedVariants = 2;
int xengine_num_variants(bfx_dtype in, bool batched);

hipError_t launch_xengine_int(bool ci4, const void *in, int64_t nt, int32_t nchan,
                              int32_t ninput, int32_t *out, bool overwrite, int variant, hipStream_t s);

// Binary16 X-engine over one contiguous cf16 array (`nt` <= kLaunchMaxTime
// rows from `in`).  Its output: add V to the binary32 buffer `out`, store it
// there, or add (double)V to the binary64 running sum `out` (16-byte
// elements, the same packed lower triangle).
enum class F16Out { kAdd, kStore, kAddRun64 };
hipError_t launch_xengine_f16(const void *in, int64_t nt, int32_t nchan, int32_t ninput, void *out,
                              F16Out mode, int variant, hipStream_t s);

// Per-subarray record of a batched plan (device table, built at plan
// creation).  Subarray k's gulp of ntime samples starts at byte
// ntime * in_row_off of the input arena and is [ntime][nchan][ninput]
// contiguous (t_stride bytes per time row); its visibilities start at byte
// out_off of the output arena.
struct BatchUnit {
    int64_t in_row_off;  // sum over earlier subarrays of their 256-byte-padded row bytes
    int64_t t_stride;    // nchan * ninput * bytes per sample
    int64_t out_off;     // byte offset in the output arena
    int32_t nchan;
    int32_t ninput;
    int32_t nitems;      // work items per channel (triangle tiles)
    int32_t nb;          // input blocks of 64
};

// Work-list entry of a batched launch: x = subarray | field << 12, y = first
// channel; field = triangle item of channel y, or, with kBatchPacked set, the
// number (1..4) of channels y, y+1, ... of a one-block subarray packed into
// one item.  x < 0: a padding entry.
constexpr int kBatchSubBits = 12;
constexpr int kBatchPacked = 1 << 30;

// Work items of one array: channels x triangle items, or groups of four
// channels when the array has a single 64-input block.
int64_t xengine_items(int32_t ninput, int32_t nchan);

// Integer X-engine over a batched plan: `nwork` work-list entries (a multiple
// of 8; entry B runs on XCD B % 8), time rows [t0, t0 + nt) of every
// subarray's gulp of ntime samples.
hipError_t launch_xengine_batched(bool ci4, const void *arena, int64_t ntime, int64_t t0,
                                  int64_t nt, const BatchUnit *d_units, const int2 *d_work,
                                  int64_t nwork, void *out, bool overwrite, int variant, hipStream_t s);

}  // namespace bfx
