// Arguments shared by the matching kernels (generic and 1-D paths).
#pragma once

#include "bmnd_internal.h"
#include "safe_index.h"

namespace bmnd {

enum MatchMode { kCount = 0, kPoissonF = 1, kGauss = 2, kPlain = 3 };

struct MatchArgs {
    Geo g;
    const float* src;    // batched observation (HT) or pilot (Wiener)
    const int* kappa;    // batched counts (kCount, generic path)
    const int* psum;     // batched patch sums of counts (kCount, generic path)
    const int64_t* refs;
    int n_refs;
    int* match;
    int* count;
    int gmin, gmax;
    int gamma_i;         // kCount: integral gamma
    float gamma_sp;      // kPoissonF: gamma * s_P
    float bias;          // kGauss: gamma * 2 P sigma^2
    int tau_i;           // kCount: accept iff score < tau_i
    float tau_f;         // float modes: accept iff score < tau_f
    float inv_sp;        // 1 / s_P
    int* range_flag;     // set when a count leaves the exact int32 range
    // float modes: FP64 twins of the constants for the re-scored near-ties
    double tau_d, bias_d, gamma_sp_d;
    // Poisson-likelihood matching (HT stage): policy, raw-count rule, the
    // policy's constants and the finite-count moment tables
    int policy;
    int integral;        // raw counts rint(y / s_P), else [y / s_P]_+
    double s_p_d;        // s_P
    double t_d, sbeta_d, skappa_d;
    const float* mu_f;
    const float* v_f;
    const double* mu_d;
    const double* v_d;
    int nmom;            // largest tabulated pooled count
    // correlated Gaussian noise (HT, kGauss): the bias of every window
    // offset (C-order over the W_d offsets, o_d = candidate - reference +
    // floor(W_d / 2)) in FP32 and FP64, and a bound on its magnitude
    const float* bias_t;
    const double* bias_td;
    const double* bias_bound;
};

// Float-mode scores within this relative band of the K-th value or of tau
// (relative to the magnitude of the terms) are re-scored in FP64, which
// decides membership, order and acceptance exactly as an FP64 evaluation
// would; FP32 round-off of a 32- to 64-term sum of squares stays below
// 1e-6 of the term magnitude.
constexpr double kTieBand = 1e-5;

bool match_1d_supported(const Geo& g, int mode);
// N-D arrays: P <= 64, last-axis patch extent 4, 8 or 16, staged window
// region and candidate count up to 4096
bool match_nd_supported(const Geo& g);
// blk (nullable): the reference list is in these spatial blocks' order; one
// workgroup per block then stages the block's box once
struct NdBlocks;
hipError_t launch_match_nd(const MatchArgs& a, int mode, int kmax, const NdBlocks* blk,
                           hipStream_t s);
hipError_t launch_match_1d(const MatchArgs& a, int mode, int step, int kmax, hipStream_t s);
// Poisson deviance / Pearson / Anscombe-SSD matching, any shape
hipError_t launch_match_pois(const MatchArgs& a, int metric, int kmax, hipStream_t s);

}  // namespace bmnd
