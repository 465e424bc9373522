// Internal declarations shared by the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bfx.h"

namespace bfx {

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
hipError_t launch_xengine_int(bool ci4, const void *in, int64_t nt, int32_t nchan,
                              int32_t ninput, int32_t *out, bool overwrite, hipStream_t s);

// One work unit of a batched (multi-array) integer launch.
struct BatchUnit {
    int64_t in_off;   // byte offset of the subarray's gulp in the input arena
    int64_t out_off;  // int32 offset of its visibilities in the output arena
    int32_t nchan;
    int32_t ninput;
    int32_t nitems;   // work items per channel (triangle tiles)
    int32_t first;    // index of this subarray's first work item in the flat list
};

}  // namespace bfx
