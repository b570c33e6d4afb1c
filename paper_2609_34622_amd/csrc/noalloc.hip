// bmnd_denoise_noalloc: the two-stage denoise of bmnd_denoise with every
// piece of device scratch (match lists, counts, FP64 numerator and
// denominator, pilot, reference-origin lists, transform tables) taken from
// one file-scope device array instead of a caller workspace or a library
// allocation.  For callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "bmnd_internal.h"
#include "denoise_plan.h"

namespace {

constexpr size_t kScratchBytes = size_t(BMND_NOALLOC_SCRATCH_BYTES);

// One copy per device, held until the process ends.  In host code this name
// is only a handle for hipGetSymbolAddress, never a device address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, unsigned char*> g_scratch_ptr;  // device -> address of `scratch`

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bmnd_status fail(bmnd_status st, const std::string& msg)
{
    bmnd::set_error(msg);
    return st;
}

// Address of the current device's copy of `scratch` (looked up once per
// device, with that device current).
hipError_t scratch_for_current_device(unsigned char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    *out = static_cast<unsigned char*>(p);
    return hipSuccess;
}

}  // namespace

extern "C" bmnd_status bmnd_denoise_noalloc(const float* d_y, const bmnd_geometry* geom,
                                            const bmnd_noise* noise, const bmnd_params* params,
                                            float* d_out, float* d_pilot, void* stream)
{
    using namespace bmnd;
    set_error("");
    DenoisePlan pl;
    bmnd_status st = plan_denoise_host(geom, noise, params, &pl);
    if (st != BMND_OK) return st;
    if (!d_y || !d_out) return fail(BMND_E_ARG, "NULL device pointer");
    if (pl.c1.metric != BMND_METRIC_SSD)
        return fail(BMND_E_UNSUPPORTED,
                    "bmnd_denoise_noalloc: Poisson-likelihood matching needs library moment "
                    "tables; use bmnd_denoise");

    // host copies of what the kernels read besides the arrays
    bmnd_geometry one = *geom;
    one.batch = 1;
    // N-D filter stages take their origins in block order, with block offsets
    // (held until the copies below have read them: a copy from pageable
    // host memory has taken its data when hipMemcpyAsync returns)
    const auto hb1 = pl.nd1 ? host_blocks_cached(one, params->ht, pl.c1.g) : nullptr;
    const auto hb2 = pl.nd2 ? host_blocks_cached(one, params->wiener, pl.c2.g) : nullptr;
    const auto ho1 = hb1 ? nullptr : host_origins_cached(one, params->ht);
    const auto ho2 = hb2 ? nullptr : host_origins_cached(one, params->wiener);
    const std::vector<int64_t>& o1 = hb1 ? hb1->refs : *ho1;
    const std::vector<int64_t>& o2 = hb2 ? hb2->refs : *ho2;
    const HostTables& h1 = host_tables_cached(pl.c1);
    const HostTables& h2 = host_tables_cached(pl.c2);

    // scratch layout: tables, origin lists, then the denoise workspace
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const size_t o_t1f = take(h1.f.size() * sizeof(float));
    const size_t o_t1d = take(h1.f64.size() * sizeof(double));
    const size_t o_t2f = take(h2.f.size() * sizeof(float));
    const size_t o_t2d = take(h2.f64.size() * sizeof(double));
    const size_t o_r1 = take(std::max<size_t>(1, o1.size()) * sizeof(int64_t));
    const size_t o_r2 = take(std::max<size_t>(1, o2.size()) * sizeof(int64_t));
    const size_t o_b1 = hb1 ? take(hb1->start.size() * sizeof(int)) : 0;
    const size_t o_b2 = hb2 ? take(hb2->start.size() * sizeof(int)) : 0;
    const size_t o_ws = take(pl.total);
    if (off > kScratchBytes)
        return fail(BMND_E_WORKSPACE,
                    "bmnd_denoise_noalloc: this denoise needs " + std::to_string(off) +
                        " bytes of scratch, more than the static " +
                        std::to_string(kScratchBytes) + " bytes; use bmnd_denoise");

    unsigned char* base = nullptr;
    hipError_t e = scratch_for_current_device(&base);
    if (e != hipSuccess)
        return fail(BMND_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto up = [&](size_t at, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes > 0)
            e = hipMemcpyAsync(base + at, src, bytes, hipMemcpyHostToDevice, s);
    };
    up(o_t1f, h1.f.data(), h1.f.size() * sizeof(float));
    up(o_t1d, h1.f64.data(), h1.f64.size() * sizeof(double));
    up(o_t2f, h2.f.data(), h2.f.size() * sizeof(float));
    up(o_t2d, h2.f64.data(), h2.f64.size() * sizeof(double));
    up(o_r1, o1.data(), o1.size() * sizeof(int64_t));
    up(o_r2, o2.data(), o2.size() * sizeof(int64_t));
    if (hb1) up(o_b1, hb1->start.data(), hb1->start.size() * sizeof(int));
    if (hb2) up(o_b2, hb2->start.data(), hb2->start.size() * sizeof(int));
    if (e != hipSuccess)
        return fail(BMND_E_HIP, std::string("upload to scratch: ") + hipGetErrorString(e));

    DevTables t1 = h1.t, t2 = h2.t;
    t1.f32 = reinterpret_cast<const float*>(base + o_t1f);
    t1.f64 = reinterpret_cast<const double*>(base + o_t1d);
    t2.f32 = reinterpret_cast<const float*>(base + o_t2f);
    t2.f64 = reinterpret_cast<const double*>(base + o_t2d);
    pl.t1 = &t1;
    pl.t2 = &t2;
    pl.r1 = reinterpret_cast<const int64_t*>(base + o_r1);
    pl.r2 = reinterpret_cast<const int64_t*>(base + o_r2);
    if (hb1) {
        pl.blk1 = hb1->blk;
        pl.blk1.start = reinterpret_cast<const int*>(base + o_b1);
    }
    if (hb2) {
        pl.blk2 = hb2->blk;
        pl.blk2.start = reinterpret_cast<const int*>(base + o_b2);
    }
    e = enqueue_denoise(pl, d_y, d_out, d_pilot, reinterpret_cast<char*>(base + o_ws), s, false);
    if (e != hipSuccess) return fail(BMND_E_HIP, std::string("denoise: ") + hipGetErrorString(e));
    return BMND_OK;
}
