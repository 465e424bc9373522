// Host side of the C ABI: argument checking, plan bookkeeping, launches.
//
// Every check runs before anything is enqueued, so a rejected call leaves the
// stream untouched.  No call here allocates device memory except
// bfx_xengine_create_batched (its work list).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "bfx_internal.h"

namespace bfx {

static thread_local char g_detail[512];

bfx_status fail(bfx_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_detail, sizeof g_detail, fmt, ap);
    va_end(ap);
    return s;
}

bfx_status hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorNotSupported) return fail(BFX_ENOTSUP, "%s: not built in this library", what);
    return fail(BFX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Defined with the kernels.
hipError_t launch_dump(bool is_int, const void *acc, void *out, double *run64, int64_t n,
                       hipStream_t s);
hipError_t launch_fengine(const int8_t *in, int32_t ninput, int32_t nfft, int64_t nspec,
                          const float *scale, void *out, bool ci8, hipStream_t s);
bool fengine_supported(int32_t ninput, int32_t nfft);
hipError_t launch_beamform(const void *x, const void *w, int32_t ninput, int32_t nchan,
                           int32_t nbeam, int64_t ntime, int32_t navg, float *out, hipStream_t s);
bool beamform_supported(int32_t navg);
int64_t beamform_units(int32_t nchan, int32_t nbeam, int64_t ntime);
hipError_t launch_beamform_ci4(const void *x, const int8_t *w, const float *scale, int32_t ninput,
                               int32_t nchan, int32_t nbeam, int64_t ntime, int32_t navg, float *out,
                               hipStream_t s);
bool beamform_ci4_supported(int32_t navg);
hipError_t launch_tengine(const int8_t *in, int32_t nchan, int32_t ninput, int64_t nspec, int32_t chan0,
                          int32_t nfft, int64_t mix_num, int64_t mix_den, float scale, void *out, bool ci4,
                          hipStream_t s);
bool tengine_supported(int32_t ninput, int32_t nfft);
int64_t beamform_ci4_units(int32_t nchan, int32_t nbeam, int64_t ntime);

}  // namespace bfx

using namespace bfx;

struct Sub {
    int32_t ninput;
    int32_t nchan;
};

struct bfx_xengine {
    bfx_dtype in;
    bool batched;
    std::vector<Sub> subs;
    int64_t nacc;
    int variant;  // kernel variant (bfx_xengine_autotune)
    // graph capture: id of the capture sequence in which an overwrite call
    // was last recorded (valid when cap_set)
    bool cap_set;
    unsigned long long cap_id;
    // batched plans only: device unit table and work list
    BatchUnit *d_units;
    int2 *d_work;
    int64_t nwork;
};

namespace {

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

inline int64_t in_sample_bytes(bfx_dtype d) {
    switch (d) {
        case BFX_CI4: return 1;
        case BFX_CI8: return 2;
        case BFX_CF16: return 4;
        default: return 0;
    }
}

inline int64_t out_pair_bytes(bfx_dtype d) { return 8; /* int32 pair or float pair */ }

inline int64_t round256(int64_t x) { return (x + 255) / 256 * 256; }

inline int64_t tri(int64_t n) { return n * (n + 1) / 2; }

bfx_status check_dims(int32_t ninput, int32_t nchan) {
    if (ninput <= 0 || ninput > 8192 || (ninput % 4) != 0)
        return fail(BFX_EINVAL, "ninput=%d must be a positive multiple of 4 <= 8192", ninput);
    if (nchan <= 0 || nchan > 65536)
        return fail(BFX_EINVAL, "nchan=%d must be in [1, 65536]", nchan);
    return BFX_OK;
}

// Offsets for subarray k of a plan, for a gulp of ntime samples.  Each
// subarray's time row is padded to 256 bytes in the arena layout, so its
// input offset is ntime times a per-plan constant.
void offsets(const bfx_xengine *p, int32_t k, int64_t ntime, int64_t *in_off, int64_t *out_off) {
    int64_t io = 0, oo = 0;
    const int64_t sb = in_sample_bytes(p->in);
    for (int32_t s = 0; s < k; ++s) {
        io += round256((int64_t)p->subs[s].nchan * p->subs[s].ninput * sb);
        oo += round256(p->subs[s].nchan * tri(p->subs[s].ninput) * out_pair_bytes(p->in));
    }
    *in_off = io * ntime;
    *out_off = oo;
}

// Work list of a batched plan.  Every work item costs the same (a fixed
// number of LDS stages, whatever its tile count), so balance is by item
// count.  A work group is one channel (all its triangle items) or, for a
// one-block subarray, up to four channels packed into one item.  Groups,
// largest first, go whole to the least loaded of 8 queues (one per XCD, so a
// channel's items share an L2 and run side by side); the queues are padded to
// equal length and interleaved (entry 8q + x = item q of queue x).
std::vector<int2> build_work(const std::vector<BatchUnit> &units) {
    struct Group { int32_t k, f0, n; bool packed; };
    std::vector<Group> groups;
    for (int32_t k = 0; k < (int32_t)units.size(); ++k) {
        const BatchUnit &u = units[k];
        if (u.nb == 1) {
            for (int32_t f = 0; f < u.nchan; f += 4)
                groups.push_back(Group{k, f, u.nchan - f < 4 ? u.nchan - f : 4, true});
        } else {
            for (int32_t f = 0; f < u.nchan; ++f) groups.push_back(Group{k, f, u.nitems, false});
        }
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group &a, const Group &b) {
        return (a.packed ? 1 : a.n) > (b.packed ? 1 : b.n);
    });
    std::vector<int2> q[8];
    for (const Group &g : groups) {
        int best = 0;
        for (int x = 1; x < 8; ++x)
            if (q[x].size() < q[best].size()) best = x;
        if (g.packed) {
            q[best].push_back(int2{g.k | (g.n << kBatchSubBits) | kBatchPacked, g.f0});
        } else {
            for (int32_t it = 0; it < g.n; ++it)
                q[best].push_back(int2{g.k | (it << kBatchSubBits), g.f0});
        }
    }
    size_t len = 0;
    for (int x = 0; x < 8; ++x) len = q[x].size() > len ? q[x].size() : len;
    std::vector<int2> work(8 * len, int2{-1, 0});
    for (int x = 0; x < 8; ++x)
        for (size_t i = 0; i < q[x].size(); ++i) work[8 * i + x] = q[x][i];
    return work;
}

}  // namespace

extern "C" {

const char *bfx_strerror(bfx_status s) {
    switch (s) {
        case BFX_OK: return "BFX_OK: success";
        case BFX_EINVAL: return "BFX_EINVAL: invalid argument";
        case BFX_ERANGE: return "BFX_ERANGE: integration exceeds the int32 bound";
        case BFX_EHIP: return "BFX_EHIP: HIP runtime error";
        case BFX_ENOTSUP: return "BFX_ENOTSUP: not supported";
        case BFX_ENOMEM: return "BFX_ENOMEM: allocation failed";
    }
    return "unknown bfx_status";
}

const char *bfx_last_error_detail(void) { return g_detail; }

int64_t bfx_xengine_max_ntime(bfx_dtype in) {
    switch (in) {
        case BFX_CI8: return (int64_t)2147483647 / (2 * 128 * 128);  // 65535
        case BFX_CI4: return (int64_t)2147483647 / (2 * 8 * 8);      // 16777215
        case BFX_CF16: return INT64_MAX;
        default: return -1;
    }
}

}  // extern "C"

namespace {

// ---- autotuning: the kernel variant of a plan, chosen by timing, optionally
// remembered in a cache file of JSON lines
//   {"arch": "gfx950", "dtype": "ci4", "shape": "704x192", "variant": 0, "us": [233.1, 241.7]}
// keyed by (arch, dtype, shape); the last matching line wins.

const char *dtype_name(bfx_dtype d) {
    switch (d) {
        case BFX_CI4: return "ci4";
        case BFX_CI8: return "ci8";
        case BFX_CF16: return "cf16";
        default: return "?";
    }
}

// "ninput x nchan" of every subarray, "," separated ("b:" prefix when batched).
std::string shape_key(const bfx_xengine *p) {
    std::string k = p->batched ? "b:" : "";
    for (size_t i = 0; i < p->subs.size(); ++i) {
        if (i) k += ",";
        k += std::to_string(p->subs[i].ninput) + "x" + std::to_string(p->subs[i].nchan);
    }
    return k;
}

// The string value of "key": "..." in a cache line, or "" if absent.
std::string json_str(const std::string &line, const char *key) {
    const std::string pat = std::string("\"") + key + "\": \"";
    const size_t a = line.find(pat);
    if (a == std::string::npos) return "";
    const size_t b = line.find('"', a + pat.size());
    if (b == std::string::npos) return "";
    return line.substr(a + pat.size(), b - a - pat.size());
}

int lookup_variant(const char *path, const std::string &arch, const std::string &dtype,
                   const std::string &shape) {
    FILE *f = path ? fopen(path, "r") : nullptr;
    if (!f) return -1;
    int found = -1;
    char buf[8192];
    while (fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        if (json_str(line, "arch") != arch || json_str(line, "dtype") != dtype ||
            json_str(line, "shape") != shape)
            continue;
        const size_t a = line.find("\"variant\": ");
        if (a == std::string::npos) continue;
        const int v = atoi(line.c_str() + a + 11);
        if (v >= 0 && v < kXengineVariants) found = v;
    }
    fclose(f);
    return found;
}

// Input of the tuning runs: seeded pseudo-random samples spread like the
// workloads' rounded Gaussians (so the MFMA operands toggle as they do on real
// data; a constant fill runs measurably faster): ci4 components uniform in
// [-3, 3], ci8 in [-14, 14], cf16 in [-1.67, 1.67].  A hash of the byte index
// (splitmix64 finaliser) gives the values.
__global__ void tune_fill_kernel(uint8_t *buf, int64_t n, int dtype) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        uint8_t b;
        if (dtype == BFX_CI4) {
            const int re = (int)(z % 7) - 3, im = (int)((z >> 20) % 7) - 3;
            b = (uint8_t)(((re & 15) << 4) | (im & 15));
        } else if (dtype == BFX_CI8) {
            b = (uint8_t)(int8_t)((int)(z % 29) - 14);
        } else {
            // byte pair of one binary16 value; the high byte alone decides the
            // magnitude, so pairs are filled from the pair index
            const uint64_t pair = (uint64_t)(i >> 1);
            uint64_t y = pair * 0xD1342543DE82EF95ull + 0x632BE59BD9B4E019ull;
            y ^= y >> 29;
            const _Float16 v = (_Float16)(((float)(int)(y % 2001) - 1000.0f) / 600.0f);
            const uint16_t u = __builtin_bit_cast(uint16_t, v);
            b = (uint8_t)((i & 1) ? (u >> 8) : (u & 0xFF));
        }
        buf[i] = b;
    }
}

// Name of the current device's architecture ("" when there is no device).
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int num_variants(const bfx_xengine *p) { return xengine_num_variants(p->in, p->batched); }

// Variant for a new plan: the cache's entry for it (if the plan has that
// variant), else 0.
int cached_variant(const bfx_xengine *p) {
    const char *path = getenv("BFX_TUNE_CACHE");
    if (!path || !*path) return 0;
    const std::string arch = device_arch();
    if (arch.empty()) return 0;
    const int v = lookup_variant(path, arch, dtype_name(p->in), shape_key(p));
    return v < 0 || v >= num_variants(p) ? 0 : v;
}

}  // namespace

extern "C" {

bfx_status bfx_xengine_create(bfx_xengine **plan, int32_t ninput, int32_t nchan, bfx_dtype in) {
    g_detail[0] = 0;
    if (!plan) return fail(BFX_EINVAL, "plan pointer is NULL");
    *plan = nullptr;
    if (in != BFX_CI4 && in != BFX_CI8 && in != BFX_CF16)
        return fail(BFX_EINVAL, "input dtype %d is not ci4, ci8 or cf16", (int)in);
    bfx_status st = check_dims(ninput, nchan);
    if (st != BFX_OK) return st;
    bfx_xengine *p = new (std::nothrow) bfx_xengine();
    if (!p) return fail(BFX_ENOMEM, "host allocation of the plan failed");
    p->in = in;
    p->batched = false;
    p->subs.push_back(Sub{ninput, nchan});
    p->nacc = 0;
    p->cap_set = false;
    p->cap_id = 0;
    p->d_units = nullptr;
    p->d_work = nullptr;
    p->nwork = 0;
    p->variant = cached_variant(p);
    *plan = p;
    return BFX_OK;
}

bfx_status bfx_xengine_create_batched(bfx_xengine **plan, int32_t nsub, const int32_t *ninput,
                                      const int32_t *nchan, bfx_dtype in) {
    g_detail[0] = 0;
    if (!plan) return fail(BFX_EINVAL, "plan pointer is NULL");
    *plan = nullptr;
    if (nsub <= 0 || nsub > 4096 || !ninput || !nchan)
        return fail(BFX_EINVAL, "nsub=%d must be in [1, 4096] with non-NULL size arrays", nsub);
    if (in != BFX_CI4 && in != BFX_CI8)
        return fail(BFX_ENOTSUP, "batched plans take ci4 or ci8 input");
    int64_t nwork = 0;
    for (int32_t k = 0; k < nsub; ++k) {
        bfx_status st = check_dims(ninput[k], nchan[k]);
        if (st != BFX_OK) return st;
        nwork += xengine_items(ninput[k], nchan[k]);
    }
    if (nwork > (int64_t)1 << 24)
        return fail(BFX_EINVAL, "batched plan has %lld work items (limit 2^24)", (long long)nwork);
    bfx_xengine *p = new (std::nothrow) bfx_xengine();
    if (!p) return fail(BFX_ENOMEM, "host allocation of the plan failed");
    p->in = in;
    p->batched = true;
    p->nacc = 0;
    p->cap_set = false;
    p->cap_id = 0;
    p->d_units = nullptr;
    p->d_work = nullptr;
    for (int32_t k = 0; k < nsub; ++k) p->subs.push_back(Sub{ninput[k], nchan[k]});
    std::vector<BatchUnit> units(nsub);
    for (int32_t k = 0; k < nsub; ++k) {
        int64_t row_off, out_off;
        offsets(p, k, 1, &row_off, &out_off);
        BatchUnit &u = units[k];
        u.in_row_off = row_off;
        u.t_stride = (int64_t)nchan[k] * ninput[k] * in_sample_bytes(in);
        u.out_off = out_off;
        u.nchan = nchan[k];
        u.ninput = ninput[k];
        u.nb = (ninput[k] + 63) / 64;
        u.nitems = (int32_t)(xengine_items(ninput[k], 1));  // per channel (1 when packed)
    }
    const std::vector<int2> work = build_work(units);
    p->nwork = (int64_t)work.size();
    hipError_t e = hipMalloc((void **)&p->d_units, units.size() * sizeof(BatchUnit));
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_work, work.size() * sizeof(int2));
    if (e != hipSuccess) {
        (void)hipFree(p->d_units);
        delete p;
        return fail(BFX_ENOMEM, "device allocation of the work list failed: %s",
                    hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_units, units.data(), units.size() * sizeof(BatchUnit),
                  hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_work, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->d_units);
        (void)hipFree(p->d_work);
        delete p;
        return hip_fail(e, "copying the work list");
    }
    p->variant = cached_variant(p);
    *plan = p;
    return BFX_OK;
}

bfx_status bfx_xengine_destroy(bfx_xengine *plan) {
    g_detail[0] = 0;
    if (!plan) return BFX_OK;
    hipError_t e = hipSuccess;
    if (plan->d_units) e = hipFree(plan->d_units);
    if (plan->d_work) {
        hipError_t e2 = hipFree(plan->d_work);
        if (e == hipSuccess) e = e2;
    }
    delete plan;
    if (e != hipSuccess) return hip_fail(e, "freeing the work list");
    return BFX_OK;
}

size_t bfx_xengine_in_bytes(const bfx_xengine *plan, int64_t ntime) {
    if (!plan || ntime < 0) return 0;
    int64_t io, oo;
    offsets(plan, (int32_t)plan->subs.size(), ntime, &io, &oo);
    if (!plan->batched) {
        const Sub &s = plan->subs[0];
        return (size_t)(ntime * s.nchan * s.ninput * in_sample_bytes(plan->in));
    }
    return (size_t)io;
}

size_t bfx_xengine_out_bytes(const bfx_xengine *plan) {
    if (!plan) return 0;
    if (!plan->batched) {
        const Sub &s = plan->subs[0];
        return (size_t)(s.nchan * tri(s.ninput) * out_pair_bytes(plan->in));
    }
    int64_t io, oo;
    offsets(plan, (int32_t)plan->subs.size(), 0, &io, &oo);
    return (size_t)oo;
}

bfx_status bfx_xengine_sub_offsets(const bfx_xengine *plan, int32_t k, int64_t ntime,
                                   int64_t *in_offset, int64_t *out_offset) {
    g_detail[0] = 0;
    if (!plan || !in_offset || !out_offset) return fail(BFX_EINVAL, "NULL argument");
    if (k < 0 || k >= (int32_t)plan->subs.size())
        return fail(BFX_EINVAL, "subarray %d out of range [0, %d)", k, (int)plan->subs.size());
    if (ntime < 0) return fail(BFX_EINVAL, "ntime=%lld is negative", (long long)ntime);
    offsets(plan, k, ntime, in_offset, out_offset);
    return BFX_OK;
}

int64_t bfx_xengine_nacc(const bfx_xengine *plan) { return plan ? plan->nacc : -1; }

int32_t bfx_xengine_variant(const bfx_xengine *plan) { return plan ? plan->variant : -1; }

int32_t bfx_xengine_num_variants(const bfx_xengine *plan) { return plan ? num_variants(plan) : -1; }

bfx_status bfx_xengine_set_variant(bfx_xengine *plan, int32_t variant) {
    g_detail[0] = 0;
    if (!plan) return fail(BFX_EINVAL, "plan is NULL");
    if (variant < 0 || variant >= num_variants(plan))
        return fail(BFX_EINVAL, "variant %d out of range [0, %d) for this plan", variant, num_variants(plan));
    plan->variant = variant;
    return BFX_OK;
}

int32_t bfx_tune_cache_lookup(const char *path, const char *arch, const char *dtype, const char *shape) {
    if (!path || !arch || !dtype || !shape) return -1;
    return lookup_variant(path, arch, dtype, shape);
}

bfx_status bfx_xengine_autotune(bfx_xengine *plan, int64_t ntime, float *times_us, bfx_stream stream) {
    g_detail[0] = 0;
    if (!plan) return fail(BFX_EINVAL, "plan is NULL");
    const int64_t tmax = bfx_xengine_max_ntime(plan->in);
    if (ntime <= 0 || ntime > tmax || ntime > ((int64_t)1 << 20))
        return fail(BFX_EINVAL, "ntime=%lld must be in [1, min(%lld, 2^20)]", (long long)ntime,
                    (long long)tmax);
    hipStream_t s = (hipStream_t)stream;
    const size_t in_bytes = bfx_xengine_in_bytes(plan, ntime);
    const size_t out_bytes = bfx_xengine_out_bytes(plan);
    void *d_in = nullptr, *d_acc = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc(&d_in, in_bytes);
    if (e == hipSuccess) e = hipMalloc(&d_acc, out_bytes);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) {
        const int64_t blocks = std::min<int64_t>(((int64_t)in_bytes + 255) / 256, 65536);
        hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint8_t *)d_in,
                           (int64_t)in_bytes, (int)plan->in);
        e = hipGetLastError();
    }
    const int saved = plan->variant;
    const int64_t saved_nacc = plan->nacc;
    float us[kXengineVariants] = {};
    if (times_us)
        for (int v = 0; v < kXengineVariants; ++v) times_us[v] = 0.0f;
    float best_ms = 0.0f;
    int best = 0;
    bfx_status st = BFX_OK;
    const int nv = num_variants(plan);
    for (int v = 0; v < nv && e == hipSuccess && st == BFX_OK; ++v) {
        plan->variant = v;
        float ms = 0.0f;
        for (int rep = 0; rep < 4 && e == hipSuccess && st == BFX_OK; ++rep) {
            // the first run warms up; the fastest of the other three counts
            if (rep > 0) e = hipEventRecord(ev[0], s);
            if (e != hipSuccess) break;
            st = bfx_xengine_accumulate(plan, d_in, ntime, d_acc, BFX_ACC_OVERWRITE, stream);
            if (st != BFX_OK || rep == 0) continue;
            e = hipEventRecord(ev[1], s);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
            if (e == hipSuccess && (rep == 1 || t < ms)) ms = t;
        }
        if (e == hipSuccess && st == BFX_OK) {
            us[v] = ms * 1000.0f;
            if (times_us) times_us[v] = us[v];
            if (v == 0 || ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_in);
    (void)hipFree(d_acc);
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    plan->nacc = saved_nacc;
    if (st != BFX_OK) {
        plan->variant = saved;
        return st;
    }
    if (e != hipSuccess) {
        plan->variant = saved;
        return hip_fail(e, "autotuning");
    }
    plan->variant = best;
    const char *path = getenv("BFX_TUNE_CACHE");
    if (path && *path) {
        FILE *f = fopen(path, "a");
        if (!f) return fail(BFX_EINVAL, "cannot append to the tune cache %s", path);
        fprintf(f, "{\"arch\": \"%s\", \"dtype\": \"%s\", \"shape\": \"%s\", \"variant\": %d, \"us\": [",
                device_arch().c_str(), dtype_name(plan->in), shape_key(plan).c_str(), best);
        for (int v = 0; v < nv; ++v)
            fprintf(f, "%s%.1f", v ? ", " : "", us[v]);
        fprintf(f, "]}\n");
        fclose(f);
    }
    return BFX_OK;
}

bfx_status bfx_xengine_accumulate(bfx_xengine *plan, const void *d_in, int64_t ntime, void *d_acc,
                                  uint32_t flags, bfx_stream stream) {
    g_detail[0] = 0;
    if (!plan) return fail(BFX_EINVAL, "plan is NULL");
    if (!d_in || !d_acc) return fail(BFX_EINVAL, "d_in / d_acc must be device pointers, got NULL");
    if (!aligned16(d_in) || !aligned16(d_acc))
        return fail(BFX_EINVAL, "d_in / d_acc must be 16-byte aligned");
    if (ntime <= 0) return fail(BFX_EINVAL, "ntime=%lld must be positive", (long long)ntime);
    if (flags & ~BFX_ACC_OVERWRITE) return fail(BFX_EINVAL, "unknown flag bits 0x%x", flags);
    const bool overwrite = flags & BFX_ACC_OVERWRITE;
    const int64_t base = overwrite ? 0 : plan->nacc;
    const int64_t tmax = bfx_xengine_max_ntime(plan->in);
    if (ntime > tmax - base)
        return fail(BFX_ERANGE,
                    "%lld samples already accumulated + %lld new exceed the int32-exact bound "
                    "%lld for this dtype; dump and start a new integration",
                    (long long)base, (long long)ntime, (long long)tmax);
    hipStream_t s = (hipStream_t)stream;
    // Under stream capture the host-side bound is checked once, at capture,
    // while every replay adds to d_acc again.  A captured call that adds is
    // therefore accepted only after an overwrite call captured into the same
    // graph: each replay then restarts the integration, and the samples of one
    // replay are the nacc checked here.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    unsigned long long cap_id = 0;
    hipError_t e = hipStreamGetCaptureInfo(s, &cap, &cap_id);
    if (e != hipSuccess) return hip_fail(e, "querying the stream's capture state");
    const bool capturing = cap == hipStreamCaptureStatusActive;
    if (capturing && !overwrite && !(plan->cap_set && plan->cap_id == cap_id))
        return fail(BFX_ENOTSUP,
                    "an accumulate that adds (no BFX_ACC_OVERWRITE) may be captured into a graph "
                    "only after an overwrite call captured into the same graph: replays would "
                    "otherwise grow the integration past the checked bound");
    if (plan->in == BFX_CF16) {
        // binary32 accumulation has no integer bound; launches are still cut
        // at kLaunchMaxTime rows so the kernel's row counter stays 32-bit.
        const Sub &sb = plan->subs[0];
        for (int64_t t0 = 0; t0 < ntime && e == hipSuccess; t0 += kLaunchMaxTime) {
            const int64_t nt = ntime - t0 < kLaunchMaxTime ? ntime - t0 : kLaunchMaxTime;
            const uint8_t *src = (const uint8_t *)d_in + t0 * sb.nchan * sb.ninput * 4;
            e = launch_xengine_f16(src, nt, sb.nchan, sb.ninput, d_acc,
                                   overwrite && t0 == 0 ? F16Out::kStore : F16Out::kAdd, plan->variant, s);
        }
    } else {
        const bool ci4 = plan->in == BFX_CI4;
        const int64_t row_bytes_per_input = ci4 ? 1 : 2;
        // Integer launches are split so no launch sums more than
        // kLaunchMaxTime samples in its int32 registers.
        for (int64_t t0 = 0; t0 < ntime && e == hipSuccess; t0 += kLaunchMaxTime) {
            const int64_t nt = ntime - t0 < kLaunchMaxTime ? ntime - t0 : kLaunchMaxTime;
            const bool ow = overwrite && t0 == 0;
            if (!plan->batched) {
                const Sub &sb = plan->subs[0];
                const uint8_t *src =
                    (const uint8_t *)d_in + t0 * sb.nchan * sb.ninput * row_bytes_per_input;
                e = launch_xengine_int(ci4, src, nt, sb.nchan, sb.ninput, (int32_t *)d_acc, ow,
                                       plan->variant, s);
            } else {
                e = launch_xengine_batched(ci4, d_in, ntime, t0, nt, plan->d_units, plan->d_work,
                                           plan->nwork, d_acc, ow, plan->variant, s);
            }
        }
    }
    if (e != hipSuccess) return hip_fail(e, "X-engine launch");
    plan->nacc = base + ntime;
    if (capturing && overwrite) {
        plan->cap_set = true;
        plan->cap_id = cap_id;
    }
    return BFX_OK;
}

bfx_status bfx_xengine_dump(bfx_xengine *plan, const void *d_acc, void *d_out, double *d_run64,
                            bfx_stream stream) {
    g_detail[0] = 0;
    if (!plan) return fail(BFX_EINVAL, "plan is NULL");
    if (!d_acc) return fail(BFX_EINVAL, "d_acc is NULL");
    if (!aligned16(d_acc) || (d_out && !aligned16(d_out)) || (d_run64 && !aligned16(d_run64)))
        return fail(BFX_EINVAL, "buffers must be 16-byte aligned");
    const int64_t nbytes = (int64_t)bfx_xengine_out_bytes(plan);
    const int64_t n = nbytes / 4;  // scalar elements (int32 or float)
    const bool is_int = plan->in != BFX_CF16;
    hipStream_t s = (hipStream_t)stream;
    const bool copy = d_out && d_out != d_acc;
    if (!copy && !d_run64) return BFX_OK;
    if (plan->batched && d_run64)
        return fail(BFX_ENOTSUP, "running sums of batched arenas are not supported");
    hipError_t e = launch_dump(is_int, d_acc, copy ? d_out : nullptr, d_run64, n, s);
    if (e != hipSuccess) return hip_fail(e, "dump launch");
    return BFX_OK;
}

bfx_status bfx_xengine_accumulate_run64(bfx_xengine *plan, const void *d_in, int64_t ntime, double *d_run64,
                                        bfx_stream stream) {
    g_detail[0] = 0;
    if (!plan) return fail(BFX_EINVAL, "plan is NULL");
    if (!d_in || !d_run64) return fail(BFX_EINVAL, "d_in / d_run64 is NULL");
    if (!aligned16(d_in) || !aligned16(d_run64))
        return fail(BFX_EINVAL, "d_in and d_run64 must be 16-byte aligned");
    if (plan->in != BFX_CF16 || plan->batched)
        return fail(BFX_ENOTSUP, "the fused running sum is built for single-array cf16 plans");
    if (ntime <= 0) return fail(BFX_EINVAL, "ntime=%lld must be positive", (long long)ntime);
    if (ntime > kLaunchMaxTime)
        return fail(BFX_ERANGE, "ntime=%lld: the fused running sum takes at most %lld samples per call "
                                "(one launch); accumulate longer integrations into a binary32 buffer "
                                "and dump it", (long long)ntime, (long long)kLaunchMaxTime);
    const Sub &sb = plan->subs[0];
    hipError_t e = launch_xengine_f16(d_in, ntime, sb.nchan, sb.ninput, d_run64, F16Out::kAddRun64,
                                      plan->variant, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "X-engine launch");
    return BFX_OK;
}

bfx_status bfx_fengine(const int8_t *d_in, int32_t ninput, int32_t nfft, int64_t nspec,
                       const float *d_scale, void *d_out, bfx_dtype out, bfx_stream stream) {
    g_detail[0] = 0;
    if (!d_in || !d_out) return fail(BFX_EINVAL, "d_in / d_out is NULL");
    if (!aligned16(d_in) || !aligned16(d_out))
        return fail(BFX_EINVAL, "d_in / d_out must be 16-byte aligned");
    if (out != BFX_CI8 && out != BFX_CF32)
        return fail(BFX_EINVAL, "output dtype must be BFX_CI8 or BFX_CF32");
    if (out == BFX_CI8 && !d_scale) return fail(BFX_EINVAL, "ci8 output needs d_scale");
    if (nfft < 64 || nfft > 8192 || (nfft & (nfft - 1)))
        return fail(BFX_EINVAL, "nfft=%d must be a power of two in [64, 8192]", nfft);
    if (ninput <= 0 || (ninput & 1) || ninput > 65536)
        return fail(BFX_EINVAL, "ninput=%d must be positive and even", ninput);
    if (nspec <= 0 || nspec > ((int64_t)1 << 28))
        return fail(BFX_EINVAL, "nspec=%lld out of range", (long long)nspec);
    if (!fengine_supported(ninput, nfft))
        return fail(BFX_ENOTSUP, "this build transforms nfft=4096 with ninput a multiple of 8 "
                                 "(got nfft=%d, ninput=%d)", nfft, ninput);
    hipError_t e = launch_fengine(d_in, ninput, nfft, nspec, d_scale, d_out, out == BFX_CI8,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "F-engine launch");
    return BFX_OK;
}

bfx_status bfx_beamform_detect(const void *d_x, const void *d_w, int32_t ninput, int32_t nchan,
                               int32_t nbeam, int64_t ntime, int32_t navg, float *d_out,
                               bfx_stream stream) {
    g_detail[0] = 0;
    if (!d_x || !d_w || !d_out) return fail(BFX_EINVAL, "NULL buffer");
    if (!aligned16(d_x) || !aligned16(d_w) || !aligned16(d_out))
        return fail(BFX_EINVAL, "buffers must be 16-byte aligned");
    if (ninput <= 0 || ninput % 32 || ninput > 8192)
        return fail(BFX_EINVAL, "ninput=%d must be a positive multiple of 32", ninput);
    if (nchan <= 0 || nchan > 65536) return fail(BFX_EINVAL, "nchan=%d out of range", nchan);
    if (nbeam <= 0 || nbeam > 256) return fail(BFX_EINVAL, "nbeam=%d must be in [1, 256]", nbeam);
    if (navg <= 0 || ntime <= 0 || ntime % navg || ntime > ((int64_t)1 << 30))
        return fail(BFX_EINVAL, "ntime=%lld must be a positive multiple of navg=%d, <= 2^30",
                    (long long)ntime, navg);
    if (beamform_units(nchan, nbeam, ntime) > kMaxWorkgroups256)
        return fail(BFX_ENOTSUP, "nchan=%d x nbeam=%d x ntime=%lld needs more workgroups than one "
                                 "launch can hold; split the gulp in time",
                    nchan, nbeam, (long long)ntime);
    if (!beamform_supported(navg))
        return fail(BFX_ENOTSUP, "this build integrates navg = 1, 2, 4, 8, 16 or 32 samples "
                                 "(got %d)", navg);
    hipError_t e = launch_beamform(d_x, d_w, ninput, nchan, nbeam, ntime, navg, d_out,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "beamformer launch");
    return BFX_OK;
}

bfx_status bfx_tengine(const int8_t *d_in, int32_t nchan, int32_t ninput, int64_t nspec, int32_t chan0,
                       int32_t nfft, int64_t mix_num, int64_t mix_den, float scale, void *d_out, bfx_dtype out,
                       bfx_stream stream) {
    g_detail[0] = 0;
    if (!d_in || !d_out) return fail(BFX_EINVAL, "d_in / d_out is NULL");
    if (!aligned16(d_in) || !aligned16(d_out))
        return fail(BFX_EINVAL, "d_in / d_out must be 16-byte aligned");
    if (out != BFX_CI8 && out != BFX_CI4) return fail(BFX_EINVAL, "output dtype must be BFX_CI8 or BFX_CI4");
    if (nfft < 64 || nfft > 8192 || (nfft & (nfft - 1)))
        return fail(BFX_EINVAL, "nfft=%d must be a power of two in [64, 8192]", nfft);
    if (ninput <= 0 || (ninput & 1) || ninput > 65536)
        return fail(BFX_EINVAL, "ninput=%d must be positive and even", ninput);
    if (nchan <= 0 || nchan > 65536 || chan0 < 0 || (int64_t)chan0 + nfft > nchan)
        return fail(BFX_EINVAL, "channels chan0=%d .. chan0+nfft-1 must lie inside nchan=%d", chan0, nchan);
    if (nspec <= 0 || nspec > ((int64_t)1 << 28))
        return fail(BFX_EINVAL, "nspec=%lld out of range", (long long)nspec);
    if (mix_den <= 0 || mix_den > 2147483647LL || mix_num < 0)
        return fail(BFX_EINVAL, "mix_den=%lld must be in [1, 2^31-1] and mix_num=%lld non-negative",
                    (long long)mix_den, (long long)mix_num);
    if (!(scale == scale) || scale > 3.4e38f || scale < -3.4e38f)
        return fail(BFX_EINVAL, "scale must be finite");
    if (!tengine_supported(ninput, nfft))
        return fail(BFX_ENOTSUP, "this build transforms nfft=4096 with ninput a multiple of 8 "
                                 "(got nfft=%d, ninput=%d)", nfft, ninput);
    hipError_t e = launch_tengine(d_in, nchan, ninput, nspec, chan0, nfft, mix_num, mix_den, scale, d_out,
                                  out == BFX_CI4, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "T-engine launch");
    return BFX_OK;
}

bfx_status bfx_beamform_ci4(const void *d_x, const int8_t *d_w, const float *d_scale, int32_t ninput,
                            int32_t nchan, int32_t nbeam, int64_t ntime, int32_t navg, float *d_out,
                            bfx_stream stream) {
    g_detail[0] = 0;
    if (!d_x || !d_w || !d_scale || !d_out) return fail(BFX_EINVAL, "NULL buffer");
    if (!aligned16(d_x) || !aligned16(d_w) || ((uintptr_t)d_scale & 3u) || ((uintptr_t)d_out & 3u))
        return fail(BFX_EINVAL, "d_x and d_w must be 16-byte aligned, d_scale and d_out 4-byte aligned");
    if (ninput <= 0 || ninput % 64 || ninput > 8192)
        return fail(BFX_EINVAL, "ninput=%d must be a positive multiple of 64 <= 8192", ninput);
    if (nchan <= 0 || nchan > 65536) return fail(BFX_EINVAL, "nchan=%d out of range", nchan);
    if (nbeam <= 0 || nbeam > 256) return fail(BFX_EINVAL, "nbeam=%d must be in [1, 256]", nbeam);
    if (navg <= 0 || ntime <= 0 || ntime % navg || ntime > ((int64_t)1 << 30))
        return fail(BFX_EINVAL, "ntime=%lld must be a positive multiple of navg=%d, <= 2^30",
                    (long long)ntime, navg);
    if (!beamform_ci4_supported(navg))
        return fail(BFX_ENOTSUP, "this build integrates navg = 1, 2, 4, ..., 64 samples (got %d)", navg);
    if (beamform_ci4_units(nchan, nbeam, ntime) > kMaxWorkgroups256)
        return fail(BFX_ENOTSUP, "nchan=%d x nbeam=%d x ntime=%lld needs more workgroups than one "
                                 "launch can hold; split the gulp in time",
                    nchan, nbeam, (long long)ntime);
    hipError_t e = launch_beamform_ci4(d_x, d_w, d_scale, ninput, nchan, nbeam, ntime, navg, d_out,
                                       (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ci4 beamformer launch");
    return BFX_OK;
}

}  // extern "C"
