/*
 * bmnd.h -- C ABI of the BMND hot path on AMD Instinct MI355X (gfx950).
 *
 * BMND ("Direct Poisson Denoising by N-Dimensional Block Matching and
 * Collaborative Filtering") denoises an N-axis array in two stages that
 * share one structure (section Method Overview):
 *   block matching -> group gather -> separable group transform ->
 *   shrinkage (hard threshold, then Wiener) -> inverse transform ->
 *   Kaiser-windowed weighted overlap-add [-> mass conservation].
 * The first (hard-threshold, "HT") stage filters the observation y into a
 * pilot; the second ("Wiener") stage matches on the pilot and filters y.
 *
 * Every compute entry point is asynchronous on the caller's HIP stream
 * (passed as an opaque `void*`; NULL is the default stream) and runs
 * entirely in the library's HIP kernels.
 *
 * Memory and ownership
 *   - Pointers named d_* are device pointers owned by the caller.  The
 *     library never frees them and keeps no reference after the call.
 *   - Arrays are float32, C-order (axis 0 slowest).  A geometry with
 *     batch = B describes B independent arrays stored back to back; "lin"
 *     always means the C-order linear index inside one array.
 *   - Per-call scratch comes from a caller workspace sized by the matching
 *     *_workspace_size() call.  The library owns only immutable,
 *     process-lifetime tables (transform matrices, windows, reference
 *     origin lists) that it builds once per configuration.
 *
 * Errors
 *   - Every function returns a bmnd_status.  Invalid arguments are caught
 *     before any launch and leave device memory untouched; the message is
 *     available from bmnd_last_error() (thread-local, valid until the next
 *     call on the same thread).
 *   - Launch failures return BMND_E_HIP.  Asynchronous device faults and
 *     device-detected range errors surface from bmnd_stream_status().
 *   - Nothing throws or aborts across this interface.
 */
#ifndef BMND_H
#define BMND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BMND_MAX_AXES 8   /* geometry structs carry up to 8 axes            */
#define BMND_GPU_AXES 4   /* the GPU kernels take at most 4 axes of extent > 1 */

typedef int32_t bmnd_status;
enum {
    BMND_OK = 0,
    BMND_E_ARG = -1,          /* invalid argument or parameter combination     */
    BMND_E_SHAPE = -2,        /* geometry invalid or too large                 */
    BMND_E_UNSUPPORTED = -3,  /* valid for the method, not supported here      */
    BMND_E_NOMEM = -4,        /* host allocation or library table failed       */
    BMND_E_HIP = -5,          /* HIP runtime error                             */
    BMND_E_WORKSPACE = -6,    /* workspace pointer NULL or too small           */
    BMND_E_RANGE = -7,        /* device detected counts outside exact range    */
    BMND_E_BUDGET = -8        /* needs more device memory than the budget      */
};

enum { BMND_STAGE_HT = 0, BMND_STAGE_WIENER = 1 };
enum { BMND_NOISE_GAUSSIAN = 0, BMND_NOISE_POISSON = 1, BMND_NOISE_CORRELATED = 2 };
enum { BMND_SCHED_GENERATED = 0, BMND_SCHED_BALANCED = 1, BMND_SCHED_SPARSE = 2,
       BMND_SCHED_OFF = 3 };
enum { BMND_SPATIAL_IDENTITY = 0, BMND_SPATIAL_DCT = 1, BMND_SPATIAL_BIOR15 = 2 };
enum { BMND_SHRINK_HARD = 0, BMND_SHRINK_SOFT = 1, BMND_SHRINK_WIENER = 2 };
enum { BMND_WEIGHT_CLASSIC = 0, BMND_WEIGHT_VARIANCE = 1, BMND_WEIGHT_RISK = 2 };
enum { BMND_SCOPE_GROUP = 0, BMND_SCOPE_PATCH = 1 };
enum { BMND_PRESET_PLAIN = 0, BMND_PRESET_STANDARD = 1 };
/* HT matching distance (section Metrics) and, for the Poisson-likelihood
 * distances, the acceptance calibration (subsection Exact Finite-Count
 * Moment Calibration). */
enum { BMND_METRIC_SSD = 0, BMND_METRIC_DEVIANCE = 1, BMND_METRIC_PEARSON = 2,
       BMND_METRIC_ANSCOMBE = 3 };
enum { BMND_POLICY_FIXED = 0, BMND_POLICY_REFERENCE = 1, BMND_POLICY_STANDARDIZED = 2 };
/* domain of the aggregation-weight surrogates: the coefficient domain, or
 * the windowed synthesized domain (Def. windowed synthesized-domain
 * weighting models) */
enum { BMND_WDOMAIN_COEFFICIENT = 0, BMND_WDOMAIN_WINDOWED = 1 };
/* pooled counts up to which the finite-count moment tables are exact */
enum { BMND_MOMENT_MAX_COUNT = 4096 };

/* Observed array(s): sampling domain Omega of ndim axes (Notation, Method
 * Overview), `batch` arrays of that shape stored back to back.  Any ndim up
 * to BMND_MAX_AXES is accepted when at most BMND_GPU_AXES axes have extent
 * > 1 (otherwise BMND_E_UNSUPPORTED): the kernels then run on the axes of
 * extent > 1, which gives the same patches, windows and linear indices,
 * while the reference schedule is built on all ndim axes (a singleton axis
 * takes part in the generated schedule's axis hierarchy).  Patch extents
 * on singleton axes are 1.  Correlated noise takes ndim <= BMND_GPU_AXES. */
typedef struct {
    int32_t ndim;                    /* 1 .. BMND_MAX_AXES                     */
    int32_t reserved;                /* must be 0                              */
    int64_t batch;                   /* >= 1                                   */
    int64_t shape[BMND_MAX_AXES];    /* L_d >= 1; batch * prod(L_d) < 2^31     */
} bmnd_geometry;

/* Noise model (section Observation Models).
 *   Gaussian: y = x + n, white, standard deviation sigma (Def. additive
 *             Gaussian observation model).
 *   Poisson:  y = s_P K, K ~ Poi(lambda) (Def. scaled-Poisson observation
 *             model).  counts_integral != 0 declares that y / s_P is an
 *             integer up to float32 storage rounding; the HT-stage matching
 *             then runs exactly on the equivalent raw counts rint(y / s_P)
 *             (eq. raw-counts; unit invariance of count statistics).
 *   Correlated: y = x + n, n wide-sense stationary Gaussian (Def. wide-sense
 *             stationary Gaussian noise) with the power spectral density
 *             given to bmnd_correlated_prepare; d_corr points to the tables
 *             that call wrote, for the same geometry and parameters. */
typedef struct {
    int32_t kind;                    /* BMND_NOISE_*                           */
    int32_t counts_integral;         /* Poisson only: 0 / 1                    */
    double sigma;                    /* Gaussian: >= 0                         */
    double s_p;                      /* Poisson: > 0                           */
    const void* d_corr;              /* Correlated: prepared tables (device)   */
} bmnd_noise;

/* Parameters of one stage (Appendix A standard profile; Appendix B
 * ablation reference levels for the "plain" preset). */
typedef struct {
    int32_t patch[BMND_MAX_AXES];    /* j_d, 1 <= j_d <= min(L_d, 32)          */
    int32_t step[BMND_MAX_AXES];     /* h_d >= 1, reference lattice step      */
    int32_t search[BMND_MAX_AXES];   /* W_d >= 1 candidate origins per axis,   */
                                     /* window offsets [-W/2, W-1-W/2]         */
    int32_t schedule;                /* BMND_SCHED_*                           */
    int32_t passes;                  /* K_s >= 1 schedule passes               */
    double shift_density;            /* rho_s >= 0                             */
    int32_t group_min;               /* power of two, >= 1                     */
    int32_t group_max;               /* power of two, <= 32; group_max*P<=4096 */
    double tau;                      /* matching threshold (stored units);     */
                                     /* < 0 selects c*P/255^2, c = 3000 (HT),  */
                                     /* 400 (Wiener)                           */
    double gamma;                    /* SSD noise-bias factor (HT); 0 Wiener  */
    int32_t spatial;                 /* BMND_SPATIAL_*                         */
    int32_t shrink;                  /* HT: HARD | SOFT;  Wiener: WIENER       */
    double lambda;                   /* HT threshold multiplier                */
    double s_v;                      /* Wiener variance scale >= 0             */
    double power_a;                  /* pilot-power correction a >= 0          */
    int32_t k_exact;                 /* exact shared-source planes, >= 0       */
    int32_t weight_model;            /* BMND_WEIGHT_*; RISK only in Wiener     */
    int32_t weight_scope;            /* BMND_SCOPE_*                           */
    int32_t mass_conservation;       /* 0 / 1                                  */
    double kaiser_beta;              /* Kaiser window beta                     */
    /* HT matching on Poisson data (ignored by SSD with the fixed policy):  */
    int32_t match_metric;            /* BMND_METRIC_*; non-SSD: HT, Poisson    */
    int32_t match_policy;            /* BMND_POLICY_*; non-FIXED needs a       */
                                     /* Poisson metric and integral counts     */
    double match_t;                  /* threshold multiplier t >= 0            */
    double struct_beta;              /* structural allowance beta_s >= 0       */
    double struct_kappa;             /* its intensity exponent kappa_s > 0     */
    int32_t weight_domain;           /* BMND_WDOMAIN_*                         */
    int32_t reserved2;               /* must be 0                              */
} bmnd_stage_params;

typedef struct {
    bmnd_stage_params ht;
    bmnd_stage_params wiener;
} bmnd_params;

/* Message describing the last failed call on this thread ("" if none). */
const char* bmnd_last_error(void);

/* Library version string. */
const char* bmnd_version(void);

/* Fill *out with a preset for an ndim-axis array.
 *   PLAIN: the ablation reference levels (Appendix B): generated schedule
 *     (rho_s = 2, K_s = 2), HT: SSD with gamma = 3, hard threshold
 *     lambda = 3, bior1.5 spatial transform, group 2..16; Wiener: DCT,
 *     classic gain (a = 0), s_v = 0.4, group 2..32; k_exact = 0, classic
 *     group weights, no mass conservation, Kaiser beta = 2.
 *   STANDARD: Appendix A: as PLAIN but k_exact = 4 and variance / patch
 *     weights in both stages.
 * Patch 8 (2-D), 4 (3-D), 32 (1-D) per axis, step 3 (4 in 1-D), search
 * 19 (2-D) / 7 (3-D) / 256 (1-D) per axis.  BMND_E_ARG for a bad preset or
 * ndim. */
bmnd_status bmnd_params_default(int32_t preset, int32_t ndim, bmnd_params* out);

/* Reference origins of one array (section Reference-Patch Schedule:
 * Def. clipped reference origin, the K_s passes, Defs. generated /
 * balanced / sparse / off schedule), deduplicated, ascending lin.  Host
 * call.  Writes up to `cap` origins to out_lin (host, may be NULL with
 * cap = 0) and the total count to *n_out. */
bmnd_status bmnd_reference_origins(const bmnd_geometry* geom, const bmnd_stage_params* sp,
                                   int64_t* out_lin, int64_t cap, int64_t* n_out);

/* Byte budgets of the library's per-shape caches: host_bytes for the
 * reference-origin and block lists of each (shape, stage parameters) seen,
 * device_bytes for their device copies (all devices together); 0 restores
 * the default of 1 GiB each.  Least recently used entries beyond a budget
 * are dropped; a device copy is freed only once no call that uses it is
 * being planned or captured in a cached batch graph, and after the device
 * has finished its queued work.  A new copy is uploaded asynchronously on
 * the stream of the call that first needs it; calls on other streams wait
 * for that upload on the device.  Host call, any time. */
bmnd_status bmnd_cache_limits(size_t host_bytes, size_t device_bytes);

/* Coverage map of a stage's reference schedule (section Experiments, Shift
 * Schedule Analysis): C(x), the number of scheduled reference patches
 * (origin r, patch support B) with x in r + B, for every sample x of one
 * array, and stats[0..2] = the spatial mean of C, its population standard
 * deviation and their ratio, the coefficient of variation (0 when the
 * mean is 0).  Host call.  out_map: host, prod(shape) uint32 in C order
 * (may be NULL); stats: host, 3 doubles (may be NULL).  Errors: those of
 * bmnd_reference_origins. */
bmnd_status bmnd_reference_coverage(const bmnd_geometry* geom, const bmnd_stage_params* sp,
                                    uint32_t* out_map, double* stats);

/* The library's transform and window tables (host call, double precision):
 * T (n x n, row-major) the spatial analysis matrix of `spatial` on n points
 * (orthonormal DCT-II; full multilevel periodised bior1.5 DWT; identity)
 * and U = T^-1 (Appendix A transforms), and the n-point Kaiser window of
 * `beta` (Method Overview).  Any output pointer may be NULL. */
bmnd_status bmnd_transform_matrices(int32_t spatial, int32_t n, double* T, double* U);
bmnd_status bmnd_haar_matrix(int32_t K, double* H);
bmnd_status bmnd_kaiser_window(int32_t n, double beta, double* w);

/* Exact finite-count moments of a Poisson matching metric's per-entry
 * contribution (Prop. universal finite-count moments), the tables the
 * calibrated policies use: mu[n], v[n] for pooled counts n = 0..nmax (host
 * arrays of nmax + 1 doubles, caller owned).  Host call.  BMND_E_ARG for a
 * metric other than DEVIANCE / PEARSON / ANSCOMBE or nmax outside
 * [0, BMND_MOMENT_MAX_COUNT]. */
bmnd_status bmnd_count_moments(int32_t metric, int32_t nmax, double* mu, double* v);

/* Stationary correlated Gaussian noise (section Observation Models: Def.
 * wide-sense stationary Gaussian noise and the discrete Wiener-Khinchin
 * relation c = ifftn(S) / |Omega|; Prop. Gaussian SSD noise bias; Lemma
 * covariance propagation).
 *
 * bmnd_correlated_size: bytes of the device tables for one array shape
 * (geom->batch is ignored: every array of a batch has the same noise) and
 * both stages of `params`.
 *
 * bmnd_correlated_prepare: from the power spectral density S on the
 * array's own DFT grid (d_psd: device, prod(shape) doubles, C-order,
 * S(omega) >= 0 is not checked), compute into d_tables (device, caller
 * owned, `bytes` >= the size above, 256-byte aligned):
 *   - the autocovariance c(tau) = Re ifftn(S)(tau) / |Omega| for every
 *     displacement the method needs, tau taken modulo the shape;
 *   - per stage, the variance table D(Delta, q) = sum_tau A_q(tau)
 *     c(Delta + tau) over the member displacements Delta of the search
 *     window and the spatial coefficients q, with A_q the autocorrelation of
 *     row q of the stage's spatial transform, so that a group's coefficient
 *     variances are sigma^2_(l,q) = sum_(j,j') H_lj H_lj' D(u_j' - u_j, q),
 *     the diagonal of T Sigma_g T^T with Sigma_g[a][b] = c(u_b - u_a);
 *   - for the HT stage, the matching bias gamma 2 P (c(0) - c(Delta)) of
 *     every window offset.
 * Stream-ordered on `stream`.  The tables stay valid until d_tables is
 * freed or prepared again; bmnd_match / bmnd_filter / bmnd_denoise check
 * that a noise model's d_corr was prepared by this call for the same shape
 * and the same patch, search, spatial transform and gamma of the stage.
 * Errors: BMND_E_ARG (NULL pointers, bad geometry or parameters),
 * BMND_E_WORKSPACE (bytes too small or d_tables misaligned), BMND_E_HIP. */
bmnd_status bmnd_correlated_size(const bmnd_geometry* geom, const bmnd_params* params,
                                 size_t* bytes);
bmnd_status bmnd_correlated_prepare(const double* d_psd, const bmnd_geometry* geom,
                                    const bmnd_params* params, void* d_tables, size_t bytes,
                                    void* stream);

/* Workspace bytes for bmnd_match / bmnd_aggregate / bmnd_denoise. */
bmnd_status bmnd_match_workspace_size(const bmnd_geometry* geom, const bmnd_stage_params* sp,
                                      size_t* bytes);
bmnd_status bmnd_aggregate_workspace_size(const bmnd_geometry* geom,
                                          const bmnd_stage_params* sp, size_t* bytes);
bmnd_status bmnd_workspace_size(const bmnd_geometry* geom, const bmnd_noise* noise,
                                const bmnd_params* params, size_t* bytes);

/* Where bmnd_denoise leaves the FP64 sums of its last (Wiener) stage in
 * its workspace (Def. weighted overlap-add; section Aggregation-Aware Mass
 * Conservation): byte offsets into d_ws of two [batch][V] double arrays,
 * the numerator (sum over groups and members of w omega (p + alpha), alpha
 * = 0 without mass conservation) and the denominator eta; the output is
 * their ratio rounded to float, 0 where eta = 0.  They let a caller check
 * the conservation of the total in FP64, before the float rounding.  The
 * arrays hold these sums from the end of a bmnd_denoise call (in stream
 * order) until the workspace is used again.  Host call.  Errors: those of
 * bmnd_workspace_size. */
bmnd_status bmnd_workspace_sums(const bmnd_geometry* geom, const bmnd_noise* noise,
                                const bmnd_params* params, size_t* num_offset,
                                size_t* den_offset);

/* Device memory one bmnd_denoise request holds while it runs (admission
 * against an HBM budget when serving): the input and output arrays
 * (2 batch V floats) plus bmnd_workspace_size(); the library's own device
 * copies of origin lists are shared between requests of one shape and
 * bounded by bmnd_cache_limits, and are not counted.  Host call.  *bytes is
 * always written on success of the size computation; BMND_E_BUDGET when
 * budget > 0 and the request needs more than budget bytes (it can never be
 * admitted within it); other errors as bmnd_workspace_size. */
bmnd_status bmnd_request_bytes(const bmnd_geometry* geom, const bmnd_noise* noise,
                               const bmnd_params* params, size_t budget, size_t* bytes);

/* Block matching for one stage (section Block Matching).
 * For every array b < batch and reference g < n_refs with origin
 * d_refs[g] (lin, same origins for every array), score every candidate
 * origin of the clipped search window:
 *   HT, Gaussian: SSD - gamma 2 P sigma^2 (Prop. Gaussian SSD noise bias,
 *                 white noise; Def. noise-bias-corrected SSD);
 *   HT, Correlated: SSD - gamma 2 P (c(0) - c(Delta)), Delta the
 *                 displacement from the reference origin to the candidate's
 *                 (Prop. Gaussian SSD noise bias);
 *   HT, Poisson:  SSD - gamma s_P sum[p + q]_+ (Prop. scaled-Poisson SSD
 *                 noise bias; Def. noise-bias-corrected SSD), computed on
 *                 the raw counts when counts_integral is set;
 *   Wiener:       SSD on d_src, the pilot (Def. paired pilot and
 *                 observation groups).
 * With a Poisson-likelihood metric (HT stage, Poisson noise) the score of
 * a candidate is built from the raw counts r = [p / s_P]_+, c = [q / s_P]_+
 * (eq. raw-counts; rint(y / s_P) with integral counts) and the per-entry
 * contributions phi of the deviance, Pearson or Anscombe-SSD statistic
 * (eq. varphi):
 *   FIXED:        d = sum phi / P, accepted if d < 1 + t sqrt(2 / P), the
 *                 high-count mean 1 and variance 2 per entry (Thm. common
 *                 high-count limit);
 *   REFERENCE:    d accepted if d < mean mu(2 r_i) + t sqrt(sum v(2 r_i)) / P
 *                 + beta_s rbar^kappa_s (Def. reference finite-count
 *                 threshold);
 *   STANDARDIZED: Z = (sum phi - sum mu(r_i + c_i)) / sqrt(sum v(r_i +
 *                 c_i)) (0 if the variance sum is 0), accepted if Z < t
 *                 (Def. candidate-standardized distance);
 * with the exact finite-count moments mu, v of phi (Prop. universal
 * finite-count moments) for pooled counts up to BMND_MOMENT_MAX_COUNT.
 * The group is the reference in slot 0 followed by the other candidates
 * in ascending (score, lin); its size K is pow2floor(min(1 + #{score <
 * tau}, group_max)), clamped to [group_min, pow2floor(1 + candidates)].
 *   d_src   [batch][V] HT: the observation y; Wiener: the pilot
 *   d_refs  [n_refs] int64 origins (lin)
 *   d_match [batch][n_refs][group_max] int32 lin of the members; -1 beyond K
 *   d_count [batch][n_refs] int32 K
 *   d_score [batch][n_refs][group_max] float, or NULL: the distance of each
 *           member to its reference in the units tau is compared in (the
 *           corrected SSD, or the Poisson-likelihood statistic of the
 *           policy: d/P for FIXED and REFERENCE, Z for STANDARDIZED),
 *           evaluated in FP64 from d_src by a second kernel and rounded
 *           to float; 0 for the reference slot and at or beyond K
 *   d_ws    workspace of bmnd_match_workspace_size() bytes
 * Non-finite scores are never selected; a group then shrinks to the
 * largest power of two its selected members fill, so every entry below K
 * is a valid origin.  Reference origins are clamped into the array.
 * Errors: BMND_E_ARG / _SHAPE / _UNSUPPORTED / _WORKSPACE / _HIP;
 * counts too large for exact int32 scoring, non-finite observations in
 * count-domain HT matching, and pooled counts beyond the moment tables
 * raise BMND_E_RANGE from bmnd_stream_status(). */
bmnd_status bmnd_match(int32_t stage, const float* d_src, const bmnd_geometry* geom,
                       const bmnd_noise* noise, const bmnd_stage_params* sp,
                       const int64_t* d_refs, int64_t n_refs, int32_t* d_match,
                       int32_t* d_count, float* d_score, void* d_ws, size_t ws_bytes,
                       void* stream);

/* Collaborative filtering of the matched groups (sections Hard
 * Thresholding, Wiener Shrinkage, Aggregation Weights).  For each group:
 * gather y (and the pilot in the Wiener stage) at the members' origins
 * (Def. paired pilot and observation groups), apply T = Haar (x) spatial
 * (x) ..., propagate the noise variances sigma_k^2 = sum |T_ki|^2 m_v(u_i)
 * (Prop. diagonal Poisson variance propagation) with the leading k_exact
 * Haar planes from the shared-source model (Def. partial shared-source
 * Poisson variance model); under correlated noise sigma_k^2 is the
 * diagonal of T Sigma_g T^T for every plane (k_exact is ignored), and every
 * member must lie within the search window of the group's reference (as
 * bmnd_match places them; displacements beyond it are clamped), shrink (eq. hard-threshold / soft-threshold,
 * or eq. wiener-gain with eq. pilot-power-family), compute the patch
 * reliability weights (Defs. coefficient-domain hard-thresholding /
 * Wiener weighting models, Def. aggregation-weight scope; with
 * BMND_WDOMAIN_WINDOWED every coefficient's term is weighted by the
 * diagonal of the windowed synthesis metric H = U^H W^2 U, Def. windowed
 * synthesis metrics, Def. windowed synthesized-domain weighting models,
 * using the diagonal of the noise model) and synthesize p = U C with
 * U = T^-1 (Def. pilot group).
 *   d_pilot    [batch][V] (Wiener only; NULL in the HT stage)
 *   d_match, d_count as produced by bmnd_match (other contents are read
 *              memory-safely: K is cut to a power of two in [1, group_max]
 *              and origins into the array; the result is then unspecified)
 *   d_patches  [batch][n_refs][group_max][P] synthesized patches, no window
 *   d_weights  [batch][n_refs][group_max] patch weights (0 beyond K)
 * Errors: BMND_E_ARG / _SHAPE / _UNSUPPORTED / _HIP. */
bmnd_status bmnd_filter(int32_t stage, const float* d_y, const float* d_pilot,
                        const bmnd_geometry* geom, const bmnd_noise* noise,
                        const bmnd_stage_params* sp, int64_t n_refs, const int32_t* d_match,
                        const int32_t* d_count, float* d_patches, float* d_weights,
                        void* stream);

/* Kaiser-windowed weighted overlap-add of given patches (Def. weighted
 * overlap-add), optionally with aggregation-aware mass conservation
 * (section Aggregation-Aware Mass Conservation): with the weights and the
 * denominator eta of a first sweep held fixed, every group is shifted by
 * the constant alpha_g = zeta_g^T (y_g - p_g) / zeta_g^T 1 that satisfies
 * eq. dc-group-constraint, so that sum x^ = sum y (Thm. mass conservation
 * after normalized overlap-add).  Voxels no patch covers are set to 0.
 *   d_match, d_count as for bmnd_filter
 *   d_y    [batch][V] observation (read only with mass conservation)
 *   d_out  [batch][V] result
 *   d_ws   workspace of bmnd_aggregate_workspace_size() bytes */
bmnd_status bmnd_aggregate(const float* d_y, const bmnd_geometry* geom,
                           const bmnd_stage_params* sp, int64_t n_refs,
                           const int32_t* d_match, const int32_t* d_count,
                           const float* d_patches, const float* d_weights, float* d_out,
                           void* d_ws, size_t ws_bytes, void* stream);

/* The two-stage BMND (section Method Overview), fused: per stage the
 * matching kernel, then one filtering kernel that aggregates directly
 * (two sweeps with mass conservation), then normalisation.  The pilot is
 * written to d_pilot if it is not NULL.  Reference origins come from the
 * library's schedule cache.
 *   d_y, d_out [batch][V];  d_ws of bmnd_workspace_size() bytes. */
bmnd_status bmnd_denoise(const float* d_y, const bmnd_geometry* geom,
                         const bmnd_noise* noise, const bmnd_params* params, float* d_out,
                         float* d_pilot, void* d_ws, size_t ws_bytes, void* stream);

/* The Wiener stage of bmnd_denoise alone, from a supplied pilot (section
 * Method Overview: the second stage matches on the first stage's pilot and
 * filters y with gains from it): for replaying or resuming a denoise from a
 * stored pilot, or for a pilot from elsewhere.  With the pilot that
 * bmnd_denoise wrote, d_out equals that call's output bit for bit.
 *   d_y, d_pilot [batch][V] inputs (read only); d_out [batch][V];
 *   d_ws of bmnd_workspace_size() bytes.
 * Errors: those of bmnd_denoise; BMND_E_ARG when d_pilot is NULL. */
bmnd_status bmnd_denoise_from_pilot(const float* d_y, const float* d_pilot,
                                    const bmnd_geometry* geom, const bmnd_noise* noise,
                                    const bmnd_params* params, float* d_out, void* d_ws,
                                    size_t ws_bytes, void* stream);

/* Autotuning of the spatial blocks of references that the 2-D and 3-D
 * kernels of bmnd_denoise walk (the matcher stages a block's search box
 * once per workgroup; the filter accumulates a block's numerators in an
 * LDS box): each of BMND_BLOCK_RULES candidate rules for the block size
 * (the largest box, the references per block) is timed on this input with
 * two bmnd_denoise runs on `stream` after one warm-up, and the fastest (a
 * rule replaces rule 0, the default, or an earlier rule only when at least
 * 3 % faster) is kept in the library's tuning table for this shape, patch,
 * step, schedule
 * and search window: every later call with them uses it.  The call waits
 * for the timings (host-synchronous) and leaves the chosen rule's result
 * in d_out.  ms (host, BMND_BLOCK_RULES doubles, nullable): the best time
 * of each rule (-1 where a rule was not run); *chosen (nullable): the
 * chosen rule, -1 when the arrays run no blocked kernels (nothing tuned).
 * Errors: those of bmnd_denoise. */
#define BMND_BLOCK_RULES 6
bmnd_status bmnd_autotune(const float* d_y, const bmnd_geometry* geom, const bmnd_noise* noise,
                          const bmnd_params* params, float* d_out, void* d_ws, size_t ws_bytes,
                          void* stream, int32_t* chosen, double* ms);

/* A batch of independent denoises (the serving and batching form of
 * bmnd_denoise, section Method Overview applied per array): any mix of
 * dimensionality, size, noise model and parameters.  Each job is exactly
 * the computation of bmnd_denoise on its own arrays.
 *   d_y, d_out  [geom.batch][V] device arrays of the job
 *   d_pilot     [geom.batch][V] receives the pilot, or NULL */
typedef struct {
    const float* d_y;
    float* d_out;
    float* d_pilot;
    bmnd_geometry geom;
    bmnd_noise noise;
    bmnd_params params;
} bmnd_job;

enum { BMND_BATCH_GRAPH = 1 };  /* capture the launch sequence, replay it */

/* Workspace bytes for bmnd_denoise_batch on this job table.  Jobs are
 * assigned to the library's concurrent streams (longest first, least
 * loaded stream); jobs on one stream share that stream's workspace, so the
 * size is the sum over streams of the largest job workspace on each.
 * Errors: those of bmnd_workspace_size, naming the job. */
bmnd_status bmnd_batch_workspace_size(int32_t n_jobs, const bmnd_job* jobs, size_t* bytes);

/* Queue all jobs: the library's streams (default priority, one per
 * hardware queue) wait for the work already on `stream`, run the jobs
 * concurrently, and `stream` waits for all of them, so the call behaves as
 * an ordinary stream-ordered operation on `stream`.  With
 * BMND_BATCH_GRAPH the launch sequence of a job table (pointers, shapes,
 * parameters and d_ws alike) is captured once into a hipGraph and
 * replayed by later calls with the same table; graphs are cached per
 * device (the 16 most recent tables).  Calls are serialized by the
 * library.  The caller owns every buffer; d_ws must hold
 * bmnd_batch_workspace_size() bytes.
 * Errors: BMND_E_ARG (NULL pointers, unknown flags), BMND_E_WORKSPACE,
 * per-job validation errors, BMND_E_HIP. */
bmnd_status bmnd_denoise_batch(int32_t n_jobs, const bmnd_job* jobs, void* d_ws, size_t ws_bytes,
                               int32_t flags, void* stream);

/* Allocation-free denoise, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes exactly what bmnd_denoise computes, with the same
 * kernels, but takes every piece of device scratch -- match lists, counts,
 * the FP64 numerator and denominator, the pilot when d_pilot is NULL, the
 * reference-origin lists and the transform tables -- from one static device
 * array of BMND_NOALLOC_SCRATCH_BYTES bytes that the library holds on each
 * device it runs on until the process ends.  The library allocates no
 * device memory in this call (host-side plan caches only); tables and
 * origin lists are copied into the array on `stream` each call.
 *   d_y, d_out  [batch][V] caller arrays;  d_pilot [batch][V] or NULL
 * Every call on one device shares that device's array and overwrites it:
 * calls that overlap in time on one device (different streams or threads)
 * race and give undefined results; calls on one stream are ordered.
 * Errors: those of bmnd_denoise; BMND_E_WORKSPACE when the denoise needs
 * more than BMND_NOALLOC_SCRATCH_BYTES of scratch (the message states the
 * need); BMND_E_UNSUPPORTED for Poisson-likelihood matching metrics. */
#define BMND_NOALLOC_SCRATCH_BYTES (64u << 20)
bmnd_status bmnd_denoise_noalloc(const float* d_y, const bmnd_geometry* geom,
                                 const bmnd_noise* noise, const bmnd_params* params, float* d_out,
                                 float* d_pilot, void* stream);

/* Kernel tracing.  Between bmnd_profile_begin() and bmnd_profile_end() the
 * library records a pair of HIP events on the launch stream around every
 * kernel that bmnd_denoise launches.  bmnd_profile_end() synchronises those
 * events, writes per kernel id the summed duration in milliseconds and the
 * number of launches (arrays of n_ids entries, ids BMND_KID_*), and stops
 * recording.  Tracing is process-wide and meant for one thread. */
enum { BMND_KID_COUNTS = 0, BMND_KID_PATCH_SUMS = 1, BMND_KID_MATCH_HT = 2,
       BMND_KID_MATCH_WIENER = 3, BMND_KID_FILTER_HT = 4, BMND_KID_FILTER_WIENER = 5,
       BMND_KID_ZERO = 6, BMND_KID_NORMALIZE = 7, BMND_KID_COUNT = 8 };
bmnd_status bmnd_profile_begin(void);
bmnd_status bmnd_profile_end(double* ms, int64_t* launches, int32_t n_ids);

/* Synchronise `stream` and report asynchronous failures: BMND_E_HIP for a
 * device fault, BMND_E_RANGE if a matching kernel saw counts outside the
 * exact int32 range (or non-finite counts) since the last call.  Clears the
 * range flag. */
bmnd_status bmnd_stream_status(void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BMND_H */
