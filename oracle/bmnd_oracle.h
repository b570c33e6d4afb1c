/*
 * BMND reference oracle (FP64, single-threaded, plain C99).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct CPU
 * statement of what the BMND hot path computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  The GPU
 * library never includes, links or calls anything here, and the oracle
 * shares no code, header, table or constant generator with it.
 *
 * Paper: "BMND: Direct Poisson Denoising by N-Dimensional Block Matching and
 * Collaborative Filtering".  Every function in bmnd_oracle.c names the
 * section / definition / equation it follows.
 *
 * Conventions (all of them readings of points the paper leaves open):
 *   - arrays are C-order, axis 0 slowest; "lin" is the C-order linear index;
 *   - a patch origin is the coordinate of its first sample (Reference-Patch
 *     Schedule section), the patch is the box origin + [0, j_d) per axis;
 *   - the search window holds W_d candidate origins per axis, centred:
 *     delta_d in [-floor(W_d/2), W_d - 1 - floor(W_d/2)], clipped to the
 *     valid origins [0, L_d - j_d];
 *   - the reference is always slot 0 of its own group, the other members are
 *     ranked by (score, lin), group size = pow2floor(min(1 + accepted, Nmax))
 *     clamped to [Nmin, pow2floor(1 + candidates)].
 */
#ifndef BMND_ORACLE_H
#define BMND_ORACLE_H

#include <stdint.h>

#define ORC_MAXD 8

enum { ORC_SCHED_GENERATED = 0, ORC_SCHED_BALANCED = 1, ORC_SCHED_SPARSE = 2, ORC_SCHED_OFF = 3 };
enum { ORC_SPATIAL_IDENTITY = 0, ORC_SPATIAL_DCT = 1, ORC_SPATIAL_BIOR15 = 2 };
enum { ORC_SHRINK_HARD = 0, ORC_SHRINK_SOFT = 1, ORC_SHRINK_WIENER = 2 };
enum { ORC_W_CLASSIC = 0, ORC_W_VARIANCE = 1, ORC_W_RISK = 2 };
enum { ORC_SCOPE_GROUP = 0, ORC_SCOPE_PATCH = 1 };
/* noise models: white Gaussian, scaled Poisson, and stationary correlated
 * Gaussian given by its periodic autocovariance (Def. wide-sense stationary
 * Gaussian noise) */
enum { ORC_NOISE_GAUSSIAN = 0, ORC_NOISE_POISSON = 1, ORC_NOISE_CORRELATED = 2 };
enum { ORC_STAGE_HT = 0, ORC_STAGE_WIENER = 1 };
/* HT matching distance and acceptance policy (section Metrics, subsection
 * Exact Finite-Count Moment Calibration) */
enum { ORC_METRIC_SSD = 0, ORC_METRIC_DEVIANCE = 1, ORC_METRIC_PEARSON = 2,
       ORC_METRIC_ANSCOMBE = 3 };
enum { ORC_POLICY_FIXED = 0, ORC_POLICY_REFERENCE = 1, ORC_POLICY_STANDARDIZED = 2 };
/* domain of the aggregation-weight surrogates (Def. windowed synthesized-
 * domain weighting models) */
enum { ORC_WDOMAIN_COEFFICIENT = 0, ORC_WDOMAIN_WINDOWED = 1 };

/* One stage's full configuration (geometry + noise + stage profile). */
typedef struct {
    int32_t ndim;
    int32_t pad0;
    int64_t shape[ORC_MAXD];
    int32_t patch[ORC_MAXD];
    int32_t step[ORC_MAXD];
    int32_t search[ORC_MAXD];
    int32_t schedule;
    int32_t passes;          /* K_s, number of schedule passes            */
    double  shift_density;   /* rho_s                                     */
    int32_t group_min;
    int32_t group_max;
    double  tau;             /* matching threshold, stored units          */
    double  gamma;           /* SSD noise-bias correction strength        */
    int32_t spatial;         /* ORC_SPATIAL_*                             */
    int32_t shrink;          /* ORC_SHRINK_*                              */
    double  lambda;          /* hard/soft threshold multiplier            */
    double  s_v;             /* Wiener variance scale                     */
    double  power_a;         /* pilot-power correction a                  */
    int32_t k_exact;         /* exact shared-source covariance planes     */
    int32_t weight_model;    /* ORC_W_*                                   */
    int32_t weight_scope;    /* ORC_SCOPE_*                               */
    int32_t mass_conservation;
    double  kaiser_beta;
    int32_t noise_kind;      /* ORC_NOISE_*                               */
    int32_t counts_integral; /* y / s_P is integral (Poisson)             */
    double  sigma;           /* Gaussian standard deviation               */
    double  s_p;             /* Poisson scale                             */
    int32_t metric;          /* ORC_METRIC_* (HT stage, Poisson noise)    */
    int32_t policy;          /* ORC_POLICY_*                              */
    double  match_t;         /* threshold multiplier t                    */
    double  struct_beta;     /* structural allowance beta_s               */
    double  struct_kappa;    /* its intensity exponent kappa_s            */
    int32_t weight_domain;   /* ORC_WDOMAIN_*                             */
    int32_t pad1;
    /* correlated Gaussian noise: the autocovariance c(tau) sampled on the
     * array's own grid (prod(shape) doubles, C-order, tau_d in [0, L_d)),
     * periodic, as the inverse DFT of the power spectral density gives it */
    const double* acov;
} orc_cfg;

/* All functions return 0 on success, <0 on bad arguments / allocation. */
int     orc_shift_list(int32_t j, int32_t h, double rho, int32_t* out, int32_t cap);
int64_t orc_schedule(const orc_cfg* c, int64_t* out, int64_t cap);
int     orc_coverage(const orc_cfg* c, uint32_t* cov, double* stats);
int     orc_haar_matrix(int32_t K, double* H);
int     orc_spatial_matrices(int32_t kind, int32_t n, double* T, double* U);
int     orc_bior15_filters(double* dec_lo10, double* rec_lo2);
int     orc_kaiser(int32_t n, double beta, double* w);
/* Per-entry contribution phi_m(r, c) of a Poisson metric (eq. varphi), the
 * finite-count moments mu_m(n), v_m(n) (eq. finite-count-moments), and the
 * score and acceptance threshold of one reference / candidate pair of P
 * entries under a policy (fixed, Def. reference finite-count threshold,
 * Def. candidate-standardized distance). */
double  orc_phi(int32_t metric, double r, double c);
int     orc_count_moments(int32_t metric, int32_t n, double* mu, double* v);
int     orc_pair_score(int32_t metric, int32_t policy, double t, double beta, double kappa,
                       int32_t P, const double* r, const double* c, double* score,
                       double* threshold);
int     orc_match(const orc_cfg* c, int32_t stage, const double* src, const double* y,
                  const int64_t* refs, int64_t nrefs, int32_t* match, int32_t* count,
                  double* score, int32_t* accepted);
int     orc_filter(const orc_cfg* c, int32_t stage, const double* y, const double* pilot,
                   int64_t nrefs, const int32_t* match, const int32_t* count,
                   double* patches, double* weights);
int     orc_group_coeffs(const orc_cfg* c, int32_t stage, const double* y, const double* pilot,
                         int32_t K, const int32_t* origins, double* Y, double* var,
                         double* C, double* w);
int     orc_aggregate(const orc_cfg* c, const double* y, int64_t nrefs, const int32_t* match,
                      const int32_t* count, const double* patches, const double* weights,
                      double* out, double* eta);
int     orc_run_stage(const orc_cfg* c, int32_t stage, const double* y, const double* pilot,
                      double* out);
int     orc_denoise(const orc_cfg* ht, const orc_cfg* wie, const double* y, double* pilot,
                    double* out);

#endif
