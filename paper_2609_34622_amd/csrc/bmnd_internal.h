// Internal interfaces of the BMND HIP library (not installed, not part of
// the C ABI).  Canonical geometry: every array is viewed as 4 axes with
// leading singleton axes, so the kernels handle 1-, 2-, 3- and 4-axis
// arrays with one code path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bmnd.h"

namespace bmnd {

constexpr int kAx = 4;        // canonical number of axes in the kernels
constexpr int kMaxGroup = 32; // largest group (Haar on 2^5 members)
constexpr int kMaxKP = 4096;  // largest group size in samples
constexpr int kMaxPatch = 32; // largest patch extent per axis

// Canonical geometry of one array (all int32: batch * V < 2^31 is checked).
struct Geo {
    int L[kAx];    // shape
    int st[kAx];   // C-order strides
    int j[kAx];    // patch extents
    int W[kAx];    // search extents (candidate origins per axis)
    int ell[kAx];  // last valid origin L - j
    int P;         // samples per patch
    int V;         // samples per array
    int batch;     // arrays
};

// Stationary correlated Gaussian noise: one stage's device tables, inside
// the caller's prepared buffer.
struct CorrStage {
    const double* dtab = nullptr;       // D(Delta, q), [member box][P]
    const double* bias = nullptr;       // HT: gamma 2 P (c(0) - c(Delta)) per window offset
    const float* bias32 = nullptr;      // the same in FP32
    const double* bias_bound = nullptr; // >= every |bias| (one value)
    int bw[kAx] = {1, 1, 1, 1};         // member box extents 2 Wm_d - 1
};

// Host-side stage description after validation.
struct StageCfg {
    Geo g;
    int stage;       // BMND_STAGE_*
    int noise;       // BMND_NOISE_*
    bool integral;   // exact count-domain HT matching
    double s_p, sigma;
    double tau;      // resolved threshold, stored units
    double gamma;
    int gmin, gmax;
    int spatial, shrink;
    double lambda, s_v, power_a;
    int k_exact, wmodel, wscope, mc;
    double beta;
    int step_last;   // reference step along the last axis
    // HT matching distance and its acceptance calibration
    int metric = BMND_METRIC_SSD, policy = BMND_POLICY_FIXED;
    double match_t = 3.0, sbeta = 0.1, skappa = 1.0;
    bool counts_integral = false;
    int wdomain = BMND_WDOMAIN_COEFFICIENT;
    CorrStage corr;  // correlated noise only
};

// Device-resident immutable tables for one (spatial transform, patch, beta).
struct DevTables {
    const float* f32 = nullptr;   // packed float tables
    const double* f64 = nullptr;  // packed double tables
    int T[kAx], U[kAx], T2[kAx], win[kAx], rn[kAx];  // float offsets per axis
    int hw[kAx];  // float offsets: windowed synthesis metric diagonal per coefficient
    int T64[kAx], T264[kAx];                         // double offsets per axis
    // double offsets: autocorrelation of each row of T, A[q][tau + j - 1] =
    // sum_i T[q][i] T[q][i + tau], j x (2 j - 1) per axis
    int ac64[kAx];
    int haar;      // float offset of Haar H (32 x 32, row-major, for K = 32 .. 1 packed)
    int haar64;    // double offset of Haar H
    int f32_count = 0, f64_count = 0;
};

// Thread-local error message.
void set_error(const std::string& msg);

// Host schedule (section Reference-Patch Schedule).
std::vector<int64_t> reference_origins(const bmnd_geometry& geom, const bmnd_stage_params& sp);
std::vector<uint32_t> coverage_map(const bmnd_geometry& geom, const bmnd_stage_params& sp);

// Host tables (transform matrices, Kaiser window).
void spatial_matrices(int kind, int n, std::vector<double>& T, std::vector<double>& U);
void haar_matrix(int K, std::vector<double>& H);
std::vector<double> kaiser_window(int n, double beta);

// Exact finite-count moments mu(n), v(n) of a Poisson matching metric's
// per-entry contribution for pooled counts 0..nmax (device copies, FP32 and
// FP64; library owned).
struct MomentTables {
    const float* mu = nullptr;
    const float* v = nullptr;
    const double* mu64 = nullptr;
    const double* v64 = nullptr;
    int nmax = 0;
};
void count_moments_host(int metric, int nmax, std::vector<double>& mu, std::vector<double>& v);
const MomentTables* device_moments(int metric, std::string& err);

// Cached device copies of the transform tables (library owned, one per
// stage configuration, kept until the process ends).
const DevTables* device_tables(const StageCfg& c, std::string& err);

// Kernel launchers (kernels.hip).  Each returns hipSuccess or the launch error.
hipError_t launch_counts(const StageCfg& c, const float* y, int* kappa, int* psum, hipStream_t s);
// Matching; kappa/psum (workspace, one int per voxel each) are used by
// the generic count-domain path and may be NULL otherwise.
// blk (nullable): the reference list is in these spatial blocks' order
// (N-D matching then stages each block's search box once per workgroup)
struct NdBlocks;
hipError_t launch_match(const StageCfg& c, const float* src, int* kappa, int* psum,
                        const int64_t* refs, int n_refs, int* match, int* count, hipStream_t s,
                        const MomentTables* mom = nullptr, const NdBlocks* blk = nullptr);
// The score of every selected member (FP64, stored as float; 0 for the
// reference slot and beyond K) from the match lists bmnd_match wrote.
hipError_t launch_member_scores(const StageCfg& c, const float* src, const int* match,
                                const int* count, int n_refs, float* score,
                                const MomentTables* mom, hipStream_t s);
// out_mode: 0 write patches/weights, 1 aggregate (FP64 sums), 2 mc sweep 1, 3 mc sweep 2
hipError_t launch_filter(const StageCfg& c, const DevTables& t, int out_mode, const float* y,
                         const float* pilot, int n_refs, const int* match, const int* count,
                         float* patches, float* weights, void* num, void* den, hipStream_t s);
// N-D filter with per-origin weights W (FP64, one value per origin) and the
// numerator accumulated in LDS boxes of the spatial blocks `blk` (the
// origin list must be in blk's order); out_mode 1 (W and numerator), 2 (W
// only), 3 (numerator with the mass-conservation shift, eta in den).
// sweep_state: hard-threshold stages with out modes 2 and 3 pass each
// member's decisions and weight from sweep 1 to sweep 2 through it
// (nd_sweep_state_bytes); null otherwise
struct NdBlocks;
inline size_t nd_sweep_state_bytes(long groups, int gmax)
{
    return size_t(groups) * size_t(gmax) * (16 + sizeof(float));
}
hipError_t launch_filter_blocked(const StageCfg& c, const DevTables& t, int out_mode,
                                 const float* y, const float* pilot, int n_refs, const int* match,
                                 const int* count, void* num, void* den, double* wfield,
                                 const NdBlocks* blk, void* sweep_state, hipStream_t s);
hipError_t launch_aggregate(const StageCfg& c, const DevTables& t, int out_mode, const float* y,
                            int n_refs, const int* match, const int* count, const float* patches,
                            const float* weights, void* num, void* den, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_normalize(const StageCfg& c, const void* num, const void* den, float* out,
                            float* out2, hipStream_t s);
hipError_t read_and_clear_range_flag(int* flag);

// Correlated-noise tables (corr_noise.hip): layout size, preparation, and
// the lookup that validates a prepared buffer for a stage and fills
// StageCfg::corr.
bmnd_status correlated_size(const bmnd_geometry* geom, const bmnd_params* params, size_t* bytes);
bmnd_status correlated_prepare(const double* d_psd, const bmnd_geometry* geom,
                               const bmnd_params* params, void* d_tables, size_t bytes,
                               hipStream_t s);
bmnd_status correlated_bind(const void* d_corr, const bmnd_geometry* geom,
                            const bmnd_stage_params* sp, int stage, StageCfg& c);

}  // namespace bmnd
