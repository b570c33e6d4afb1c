// Arguments shared by the filtering kernels (generic and cube-patch paths).
#pragma once

#include "bmnd_internal.h"
#include "safe_index.h"

namespace bmnd {

struct FilterArgs {
    Geo g;
    int stage, shrink, noise;
    int spatial;   // the stage's spatial transform (BMND_SPATIAL_*)
    float s_p, sigma2, lambda, s_v, power_a;
    double s_p64, sigma2_64, lambda64;
    int wmodel, wscope;
    int wdomain;   // BMND_WDOMAIN_*
    int kex;       // exact covariance planes (leading Haar planes l < kex)
    int gmax, n_refs;
    int out_mode;  // 0 patches, 1 aggregate (FP64 sums), 2 mc sweep 1, 3 mc sweep 2
    const float* y;
    const float* pilot;
    const int* match;
    const int* count;
    const float* patches_in;  // aggregate-only launches
    const float* weights_in;
    DevTables t;
    float* patches;
    float* weights;
    double* numd;
    double* dend;
    double* wfield;   // per-origin weight sums (N-D filter: eta = W * window)
    // N-D filter, thresholding with mass conservation: per member (group *
    // gmax + slot) its final keep mask and the coefficients the FP64
    // re-decision kept (4 words), and its weight, written by sweep 1 and
    // read by sweep 2
    unsigned* hmask;
    float* hwt;
    // correlated Gaussian noise: variance table D(Delta, q) over the member
    // box of extents cbw (null otherwise)
    const double* cdtab;
    int cbw[kAx];
};

constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }

// diagonal of the windowed synthesis metric for spatial coefficient q (the
// product over the axes of sum_i (w_i U[i][q_d])^2)
__device__ inline float window_metric(const FilterArgs& a, int q)
{
    float h = 1.f;
#pragma unroll
    for (int d = kAx - 1; d >= 0; --d) {
        const int n = a.g.j[d];
        h *= a.t.f32[a.t.hw[d] + q % n];
        q /= n;
    }
    return h;
}


bool cube_filter_supported(const Geo& g, int gmax);
hipError_t launch_filter_cube(const FilterArgs& a, int step_last, hipStream_t s);
// 32-sample patches (leading patch extents 1), groups of at most 16, filtering
// launches only (not the aggregate-only entry point)
bool filter_1d_supported(const Geo& g, int gmax, bool patches_in, int kex);
hipError_t launch_filter_1d(const FilterArgs& a, int step_last, hipStream_t s);

}  // namespace bmnd
