// The launch plan of one two-stage denoise (section Method Overview), shared
// by bmnd_denoise, the batch call and the allocation-free entry point: the
// validated stage configurations, where the reference origins and the
// transform tables live on the device, and the workspace layout.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "bmnd_internal.h"
#include "filter_nd.h"

namespace bmnd {

struct DenoisePlan {
    StageCfg c1, c2;
    const int64_t* r1 = nullptr;
    const int64_t* r2 = nullptr;
    int64_t n1 = 0, n2 = 0;
    const DevTables* t1 = nullptr;
    const DevTables* t2 = nullptr;
    const MomentTables* m1 = nullptr;  // HT Poisson-likelihood matching
    // N-D filter with per-origin weights and LDS boxes: the stage's origins
    // are listed block by block (r1 / r2 then point to that order)
    bool nd1 = false, nd2 = false;
    NdBlocks blk1, blk2;
    size_t offs[10] = {};
    size_t total = 0;
    // owners of the library's device copies r1 / r2 point into, and the
    // events that mark the end of their uploads
    std::shared_ptr<const void> keep[2];
    hipEvent_t ready[2] = {nullptr, nullptr};
};

// Host part of a plan: stage configurations, reference counts and the
// workspace layout (no device pointers are set).
bmnd_status plan_denoise_host(const bmnd_geometry* geom, const bmnd_noise* noise,
                              const bmnd_params* params, DenoisePlan* pl);

// The two stages of one denoise on stream s; ws holds pl.total bytes laid
// out as pl.offs.  With spans, kernel times are recorded for tracing.  With
// from_pilot, d_pilot holds a pilot and only the Wiener stage runs.
hipError_t enqueue_denoise(const DenoisePlan& pl, const float* d_y, float* d_out,
                           float* d_pilot, char* ws, hipStream_t s, bool spans,
                           bool from_pilot = false);

// Transform, window and Haar tables of one stage configuration in host
// memory, with their offsets (t.f32 / t.f64 left null).
struct HostTables {
    std::vector<float> f;
    std::vector<double> f64;
    DevTables t;
};
void build_tables_host(const StageCfg& c, std::vector<float>& f, std::vector<double>& f64,
                       DevTables& t);

// Host caches.  The transform tables are kept for the process (a handful
// of configurations); origin lists and block lists are kept while recently
// used, within a byte budget, and shared with their users.
const HostTables& host_tables_cached(const StageCfg& c);
std::shared_ptr<const std::vector<int64_t>> host_origins_cached(const bmnd_geometry& geom,
                                                                const bmnd_stage_params& sp);

// Origins of a stage in the N-D filter's block order, with the block
// offsets and box geometry (blk.start left null).
struct HostBlocks {
    std::vector<int64_t> refs;
    std::vector<int> start;
    NdBlocks blk;
};
std::shared_ptr<const HostBlocks> host_blocks_cached(const bmnd_geometry& geom,
                                                     const bmnd_stage_params& sp, const Geo& g);
// whether a stage runs the N-D filter with per-origin weights
bool stage_uses_nd(const StageCfg& c);

}  // namespace bmnd
