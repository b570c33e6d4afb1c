/*
 * BMND reference oracle (FP64, single-threaded, plain C99).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the benchmark's CPU-baseline leg; never by the GPU library.  See
 * bmnd_oracle.h for the conventions this file fixes where the paper is
 * silent.  Everything is written as the paper states it, step by step,
 * with no blocking or fusion: one reference at a time, one group at a time.
 */
#include "bmnd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_TIE_REL 1e-9

/* ------------------------------------------------------------------ */
/* geometry helpers                                                    */
/* ------------------------------------------------------------------ */

static void strides_of(const orc_cfg* c, int64_t* st)
{
    st[c->ndim - 1] = 1;
    for (int d = c->ndim - 2; d >= 0; --d) st[d] = st[d + 1] * c->shape[d + 1];
}

static int64_t volume_of(const orc_cfg* c)
{
    int64_t v = 1;
    for (int d = 0; d < c->ndim; ++d) v *= c->shape[d];
    return v;
}

static int patch_size_of(const orc_cfg* c)
{
    int p = 1;
    for (int d = 0; d < c->ndim; ++d) p *= c->patch[d];
    return p;
}

/* Linear offsets of the P patch samples relative to the patch origin,
 * patch samples enumerated in C-order (vectorised patch, Def. patch-group
 * observation model). */
static void patch_offsets(const orc_cfg* c, const int64_t* st, int64_t* off)
{
    int P = patch_size_of(c);
    for (int i = 0; i < P; ++i) {
        int rem = i;
        int64_t o = 0;
        for (int d = c->ndim - 1; d >= 0; --d) {
            int id = rem % c->patch[d];
            rem /= c->patch[d];
            o += (int64_t)id * st[d];
        }
        off[i] = o;
    }
}

static int check_cfg(const orc_cfg* c)
{
    if (!c || c->ndim < 1 || c->ndim > ORC_MAXD) return -1;
    for (int d = 0; d < c->ndim; ++d) {
        if (c->shape[d] < 1 || c->patch[d] < 1 || c->patch[d] > c->shape[d]) return -1;
        if (c->step[d] < 1 || c->search[d] < 1) return -1;
    }
    if (c->group_min < 1 || c->group_max < c->group_min) return -1;
    if ((c->group_max & (c->group_max - 1)) != 0) return -1;
    if ((c->group_min & (c->group_min - 1)) != 0) return -1;
    if (c->group_max > 32 || c->group_max * patch_size_of(c) > 4096) return -1;
    if (c->spatial < ORC_SPATIAL_IDENTITY || c->spatial > ORC_SPATIAL_BIOR15) return -1;
    if (c->shrink < ORC_SHRINK_HARD || c->shrink > ORC_SHRINK_WIENER) return -1;
    if (c->weight_model < ORC_W_CLASSIC || c->weight_model > ORC_W_RISK) return -1;
    if (c->noise_kind == ORC_NOISE_POISSON && !(c->s_p > 0.0)) return -1;
    if (c->noise_kind == ORC_NOISE_GAUSSIAN && !(c->sigma >= 0.0)) return -1;
    if (c->noise_kind == ORC_NOISE_CORRELATED && !c->acov) return -1;
    if (c->noise_kind < ORC_NOISE_GAUSSIAN || c->noise_kind > ORC_NOISE_CORRELATED) return -1;
    return 0;
}

/* Autocovariance at a displacement (Def. wide-sense stationary Gaussian
 * noise): the inverse DFT of the power spectral density samples c on the
 * discrete torus, so every component is taken modulo the axis length. */
static double acov_at(const orc_cfg* c, const int64_t* tau)
{
    int64_t idx = 0;
    for (int d = 0; d < c->ndim; ++d) {
        int64_t t = tau[d] % c->shape[d];
        if (t < 0) t += c->shape[d];
        idx = idx * c->shape[d] + t;
    }
    return c->acov[idx];
}

static void coords_of(const orc_cfg* c, int64_t lin, int64_t* co)
{
    for (int d = c->ndim - 1; d >= 0; --d) { co[d] = lin % c->shape[d]; lin /= c->shape[d]; }
}

static int64_t pow2floor64(int64_t x)
{
    int64_t p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

/* ------------------------------------------------------------------ */
/* Reference-patch schedule (section Reference-Patch Schedule)         */
/* ------------------------------------------------------------------ */

/* Candidate shift list S_d, eq. number-shifts and eq. candidate-shift-list:
 *   n_d = min{ j_d, max(1, ceil(rho (j_d - 1) / h_d)) }
 *   s_{d,i} = floor(i (j_d - 1) / (n_d - 1) + 1/2)   (0 when n_d = 1).     */
int orc_shift_list(int32_t j, int32_t h, double rho, int32_t* out, int32_t cap)
{
    if (j < 1 || h < 1) return -1;
    long n = (long)ceil(rho * (double)(j - 1) / (double)h);
    if (n < 1) n = 1;
    if (n > j) n = j;
    if (n > cap) return -1;
    if (n == 1) {
        out[0] = 0;
        return 1;
    }
    for (long i = 0; i < n; ++i) {
        /* floor(i(j-1)/(n-1) + 1/2) in exact integer arithmetic */
        long num = 2 * i * (long)(j - 1) + (n - 1);
        out[i] = (int32_t)(num / (2 * (n - 1)));
    }
    return (int)n;
}

static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Reference origins: Def. clipped reference origin (eq. clipped-origin),
 * the K_s passes with one offset vector per pass, and the four schedules
 * (Defs. generated / balanced / sparse / off reference schedule).  Repeated
 * origins are kept once; the result is sorted by lin.
 * Returns the number of origins (fills out[] if cap suffices), <0 on error. */
int64_t orc_schedule(const orc_cfg* c, int64_t* out, int64_t cap)
{
    if (check_cfg(c) != 0) return -1;
    const int D = c->ndim;
    int64_t st[ORC_MAXD], ell[ORC_MAXD], Z[ORC_MAXD];
    int32_t S[ORC_MAXD][64];
    int nS[ORC_MAXD];
    strides_of(c, st);
    int64_t nslots = 1;
    for (int d = 0; d < D; ++d) {
        ell[d] = c->shape[d] - c->patch[d];
        Z[d] = (ell[d] + c->step[d] - 1) / c->step[d] + 1;   /* ceil(ell/h) + 1 */
        nslots *= Z[d];
        if (c->patch[d] > 64) return -1;
        nS[d] = orc_shift_list(c->patch[d], c->step[d], c->shift_density, S[d], 64);
        if (nS[d] < 1) return -1;
    }
    int passes = c->schedule == ORC_SCHED_OFF ? 1 : c->passes;
    if (passes < 1) return -1;

    /* active axes for the sparse schedule */
    int active[ORC_MAXD], next_active[ORC_MAXD];
    for (int d = 0; d < D; ++d) active[d] = (Z[d] > 1 || c->patch[d] > 1);
    for (int d = 0; d < D; ++d) {
        next_active[d] = -1;
        for (int e = d + 1; e < D; ++e)
            if (active[e]) { next_active[d] = e; break; }
    }

    int64_t total = nslots * passes;
    int64_t* all = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    if (!all) return -2;
    int64_t nall = 0;
    int64_t q[ORC_MAXD];
    for (int64_t s = 0; s < nslots; ++s) {
        int64_t rem = s;
        for (int d = D - 1; d >= 0; --d) { q[d] = rem % Z[d]; rem /= Z[d]; }
        int64_t Qsum = 0;
        for (int d = 0; d < D; ++d) Qsum += q[d];
        for (int k = 0; k < passes; ++k) {
            int64_t lin = 0;
            for (int d = 0; d < D; ++d) {
                int64_t o = 0;
                switch (c->schedule) {
                case ORC_SCHED_GENERATED:
                    if (d < D - 1) o = S[d][(q[d + 1] + k) % nS[d]];
                    break;
                case ORC_SCHED_BALANCED:
                    o = S[d][(k + Qsum - q[d]) % nS[d]];
                    break;
                case ORC_SCHED_SPARSE:
                    if (active[d] && next_active[d] >= 0) o = S[d][(q[next_active[d]] + k) % nS[d]];
                    break;
                case ORC_SCHED_OFF:
                default:
                    o = 0;
                }
                int64_t slot = q[d] * c->step[d];
                if (slot > ell[d]) slot = ell[d];
                int64_t r = slot - o;
                if (r < 0) r = 0;
                if (r > ell[d]) r = ell[d];
                if (q[d] == Z[d] - 1) r = ell[d];   /* last slot anchors the far boundary */
                lin += r * st[d];
            }
            all[nall++] = lin;
        }
    }
    qsort(all, (size_t)nall, sizeof(int64_t), cmp_i64);
    int64_t nu = 0;
    for (int64_t i = 0; i < nall; ++i)
        if (nu == 0 || all[i] != all[nu - 1]) all[nu++] = all[i];
    if (out && cap >= nu) memcpy(out, all, sizeof(int64_t) * (size_t)nu);
    free(all);
    return nu;
}

/* Coverage map of a schedule (section Experiments, Shift Schedule
 * Analysis): C(x) counts the scheduled reference patches r + B (r an origin
 * of the schedule, B the patch support) that contain sample x; mean and
 * population standard deviation of C over the whole array, and their ratio,
 * the coefficient of variation.  Written as the definition: every origin
 * adds one over its patch.  cov (V entries, may be NULL) receives C;
 * stats[0..2] = mean, standard deviation, CV.  Returns 0, <0 on error. */
int orc_coverage(const orc_cfg* c, uint32_t* cov, double* stats)
{
    int64_t n = orc_schedule(c, NULL, 0);
    if (n < 0) return (int)n;
    const int D = c->ndim;
    int64_t st[ORC_MAXD];
    strides_of(c, st);
    int64_t V = 1, P = 1;
    for (int d = 0; d < D; ++d) {
        V *= c->shape[d];
        P *= c->patch[d];
    }
    int64_t* refs = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    uint32_t* C = (uint32_t*)calloc((size_t)V, sizeof(uint32_t));
    if (!refs || !C) {
        free(refs);
        free(C);
        return -2;
    }
    orc_schedule(c, refs, n);
    for (int64_t i = 0; i < n; ++i) {
        /* every sample of the patch at origin refs[i] */
        for (int64_t k = 0; k < P; ++k) {
            int64_t rem = k, lin = refs[i];
            for (int d = D - 1; d >= 0; --d) {
                lin += (rem % c->patch[d]) * st[d];
                rem /= c->patch[d];
            }
            C[lin] += 1u;
        }
    }
    double sum = 0.0;
    for (int64_t x = 0; x < V; ++x) sum += (double)C[x];
    const double mean = sum / (double)V;
    double ss = 0.0;
    for (int64_t x = 0; x < V; ++x) {
        const double dv = (double)C[x] - mean;
        ss += dv * dv;
    }
    const double sd = sqrt(ss / (double)V);
    if (stats) {
        stats[0] = mean;
        stats[1] = sd;
        stats[2] = mean > 0.0 ? sd / mean : 0.0;
    }
    if (cov) memcpy(cov, C, sizeof(uint32_t) * (size_t)V);
    free(refs);
    free(C);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Transforms (Appendix A: Haar group transform, bior1.5 / DCT spatial) */
/* ------------------------------------------------------------------ */

/* Orthonormal multilevel Haar on K = 2^m members.  Row order: scaling row,
 * then detail rows from the coarsest level (support K) to the finest
 * (support 2, pairing members (0,1), (2,3), ...).  Built recursively:
 * H_K = [ H_{K/2} * A ; B ] with A the pairwise averages and B the pairwise
 * differences, both scaled by 1/sqrt(2). */
int orc_haar_matrix(int32_t K, double* H)
{
    if (K < 1 || (K & (K - 1)) != 0) return -1;
    memset(H, 0, sizeof(double) * (size_t)K * (size_t)K);
    if (K == 1) {
        H[0] = 1.0;
        return 0;
    }
    int h = K / 2;
    double* Hh = (double*)malloc(sizeof(double) * (size_t)h * (size_t)h);
    if (!Hh) return -2;
    orc_haar_matrix(h, Hh);
    const double r = 1.0 / sqrt(2.0);
    /* top block: H_h applied to the averages a_i = (x_{2i} + x_{2i+1})/sqrt2 */
    for (int a = 0; a < h; ++a)
        for (int i = 0; i < h; ++i) {
            H[a * K + 2 * i] += Hh[a * h + i] * r;
            H[a * K + 2 * i + 1] += Hh[a * h + i] * r;
        }
    /* bottom block: finest details d_i = (x_{2i} - x_{2i+1})/sqrt2 */
    for (int i = 0; i < h; ++i) {
        H[(h + i) * K + 2 * i] = r;
        H[(h + i) * K + 2 * i + 1] = -r;
    }
    free(Hh);
    return 0;
}

/* bior1.5 filter pair from the Cohen-Daubechies-Feauveau spline
 * construction with (N, N~) = (1, 5), l = (N + N~)/2 = 3:
 *   synthesis lowpass   m0(z)  = ((1 + z)/2)^1
 *   analysis  lowpass   m~0(z) = ((1 + z)/2)^5 * z^-2 * sum_{n<l} C(l-1+n, n) s(z)^n,
 *   s(z) = (2 - z - 1/z)/4  (i.e. sin^2 of half the frequency),
 * both scaled by sqrt(2).  dec_lo10 receives the 10 analysis taps at
 * z^-4 .. z^5 (the two central taps at z^0, z^1), rec_lo2 the synthesis taps
 * at z^0, z^1. */
int orc_bior15_filters(double* dec_lo10, double* rec_lo2)
{
    /* Laurent polynomials stored with an index offset */
    double q[5] = {0, 0, 0, 0, 0};   /* powers -2..2 */
    double spow[5] = {0, 0, 1, 0, 0}; /* s^0 */
    const double s[3] = {-0.25, 0.5, -0.25};
    const int l = 3;
    for (int n = 0; n < l; ++n) {
        /* binomial C(l-1+n, n) */
        double b = 1.0;
        for (int t = 1; t <= n; ++t) b = b * (double)(l - 1 + t) / (double)t;
        for (int p = 0; p < 5; ++p) q[p] += b * spow[p];
        if (n + 1 == l) break;
        /* spow *= s */
        double nxt[5] = {0, 0, 0, 0, 0};
        for (int p = 0; p < 5; ++p)
            for (int t = 0; t < 3; ++t) {
                int idx = p + t - 1;
                if (spow[p] != 0.0 && (idx < 0 || idx >= 5)) return -1;
                if (idx >= 0 && idx < 5) nxt[idx] += spow[p] * s[t];
            }
        memcpy(spow, nxt, sizeof nxt);
    }
    /* ((1+z)/2)^5, powers 0..5 */
    double bnm[6] = {1, 0, 0, 0, 0, 0};
    for (int t = 0; t < 5; ++t) {
        for (int p = 5; p >= 1; --p) bnm[p] = 0.5 * (bnm[p] + bnm[p - 1]);
        bnm[0] *= 0.5;
    }
    /* product: powers -2..7, then shift by z^-2 -> powers -4..5 */
    double prod[10];
    memset(prod, 0, sizeof prod);
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 6; ++b) prod[a + b] += q[a] * bnm[b];
    for (int i = 0; i < 10; ++i) dec_lo10[i] = sqrt(2.0) * prod[i];
    rec_lo2[0] = sqrt(2.0) * 0.5;
    rec_lo2[1] = sqrt(2.0) * 0.5;
    return 0;
}

/* One periodised analysis level on n points (n even):
 *   a[k] = sum_t lo~[t] x[(2k + t) mod n],  d[k] = sum_t hi~[t] x[(2k + t) mod n],
 * hi~[t] = (-1)^t lo[1 - t] (alternating flip of the synthesis lowpass).
 * Writes the n x n matrix with the approximation rows first. */
static void bior_analysis_level(int n, const double* lo10, const double* lo2, double* A)
{
    memset(A, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int k = 0; k < n / 2; ++k) {
        for (int t = -4; t <= 5; ++t) {
            int m = ((2 * k + t) % n + n) % n;
            A[k * n + m] += lo10[t + 4];
        }
        for (int t = 0; t <= 1; ++t) {
            /* hi~[t] for t in {0, 1}: hi~[0] = lo[1], hi~[1] = -lo[0] */
            double v = (t == 0) ? lo2[1] : -lo2[0];
            int m = ((2 * k + t) % n + n) % n;
            A[(n / 2 + k) * n + m] += v;
        }
    }
}

/* One periodised synthesis level on n points:
 *   x[m] = sum_k a[k] lo[(m - 2k)] + sum_k d[k] hi[(m - 2k)]   (indices mod n),
 * hi[t] = (-1)^t lo~[1 - t].  Writes S (n x n) with x = S [a; d]. */
static void bior_synthesis_level(int n, const double* lo10, const double* lo2, double* S)
{
    memset(S, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int k = 0; k < n / 2; ++k) {
        for (int t = 0; t <= 1; ++t) {
            int m = ((2 * k + t) % n + n) % n;
            S[m * n + k] += lo2[t];
        }
        /* hi[t] = (-1)^t lo~[1 - t]; lo~ lives on t' = 1 - t in [-4, 5] -> t in [-4, 5] */
        for (int t = -4; t <= 5; ++t) {
            int tp = 1 - t;
            double v = ((t % 2 == 0) ? 1.0 : -1.0) * lo10[tp + 4];
            int m = ((2 * k + t) % n + n) % n;
            S[m * n + (n / 2 + k)] += v;
        }
    }
}

static void matmul(int n, const double* A, const double* B, double* C)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
            C[i * n + j] = s;
        }
}

/* Spatial transform matrices T (analysis) and U = T^-1 (synthesis), n x n,
 * row-major, for one patch axis.
 *   IDENTITY: T = U = I.
 *   DCT: orthonormal DCT-II, T[k][m] = c_k cos(pi (2m+1) k / (2n)), U = T^T.
 *   BIOR15: full multilevel periodised bior1.5 DWT (levels while the length
 *   is even), approximation coefficients first; U built from the synthesis
 *   filters level by level (not by inverting T). */
int orc_spatial_matrices(int32_t kind, int32_t n, double* T, double* U)
{
    if (n < 1) return -1;
    const size_t nn = (size_t)n * (size_t)n;
    memset(T, 0, sizeof(double) * nn);
    memset(U, 0, sizeof(double) * nn);
    if (kind == ORC_SPATIAL_IDENTITY || n == 1) {
        for (int i = 0; i < n; ++i) T[i * n + i] = U[i * n + i] = 1.0;
        return 0;
    }
    if (kind == ORC_SPATIAL_DCT) {
        for (int k = 0; k < n; ++k) {
            double ck = sqrt((k == 0 ? 1.0 : 2.0) / (double)n);
            for (int m = 0; m < n; ++m) {
                /* cos(pi q / (2n)), q = k (2m + 1), is exactly 0 when q / n is
                 * an odd integer (an odd multiple of pi/2) */
                const long q = (long)k * (2L * m + 1L);
                const int zero = (q % n == 0) && ((q / n) % 2 == 1);
                T[k * n + m] = zero ? 0.0 : ck * cos(ORC_PI * (2.0 * m + 1.0) * k / (2.0 * n));
                U[m * n + k] = T[k * n + m];
            }
        }
        return 0;
    }
    if (kind != ORC_SPATIAL_BIOR15) return -1;
    double lo10[10], lo2[2];
    if (orc_bior15_filters(lo10, lo2) != 0) return -1;
    double* L = (double*)malloc(sizeof(double) * nn);
    double* tmp = (double*)malloc(sizeof(double) * nn);
    double* lvl = (double*)malloc(sizeof(double) * nn);
    if (!L || !tmp || !lvl) { free(L); free(tmp); free(lvl); return -2; }
    for (int i = 0; i < n; ++i) T[i * n + i] = U[i * n + i] = 1.0;
    int len = n;
    while (len % 2 == 0 && len >= 2) {
        /* embed the level operator acting on the first len coefficients */
        double* A = (double*)malloc(sizeof(double) * (size_t)len * (size_t)len);
        double* Sy = (double*)malloc(sizeof(double) * (size_t)len * (size_t)len);
        if (!A || !Sy) { free(A); free(Sy); free(L); free(tmp); free(lvl); return -2; }
        bior_analysis_level(len, lo10, lo2, A);
        bior_synthesis_level(len, lo10, lo2, Sy);
        /* T <- blockdiag(A, I) * T */
        memset(lvl, 0, sizeof(double) * nn);
        for (int i = 0; i < n; ++i) lvl[i * n + i] = 1.0;
        for (int i = 0; i < len; ++i)
            for (int j = 0; j < len; ++j) lvl[i * n + j] = A[i * len + j];
        matmul(n, lvl, T, tmp);
        memcpy(T, tmp, sizeof(double) * nn);
        /* U <- U * blockdiag(Sy, I) */
        memset(lvl, 0, sizeof(double) * nn);
        for (int i = 0; i < n; ++i) lvl[i * n + i] = 1.0;
        for (int i = 0; i < len; ++i)
            for (int j = 0; j < len; ++j) lvl[i * n + j] = Sy[i * len + j];
        matmul(n, U, lvl, tmp);
        memcpy(U, tmp, sizeof(double) * nn);
        free(A);
        free(Sy);
        len /= 2;
    }
    free(L);
    free(tmp);
    free(lvl);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Kaiser aggregation window (Method Overview; Appendix A, beta = 2)    */
/* ------------------------------------------------------------------ */

/* Modified Bessel function of the first kind, order 0, by its power series
 * I0(x) = sum_k ((x/2)^k / k!)^2. */
static double bessel_i0(double x)
{
    double term = 1.0, sum = 1.0, half = 0.5 * x;
    for (int k = 1; k < 200; ++k) {
        term *= half / (double)k;
        double t2 = term * term;
        sum += t2;
        if (t2 < 1e-18 * sum) break;
    }
    return sum;
}

/* w[m] = I0(beta sqrt(1 - (2m/(n-1) - 1)^2)) / I0(beta);  w = [1] for n = 1. */
int orc_kaiser(int32_t n, double beta, double* w)
{
    if (n < 1) return -1;
    if (n == 1) { w[0] = 1.0; return 0; }
    double den = bessel_i0(beta);
    for (int m = 0; m < n; ++m) {
        double r = 2.0 * m / (double)(n - 1) - 1.0;
        double a = 1.0 - r * r;
        if (a < 0.0) a = 0.0;
        w[m] = bessel_i0(beta * sqrt(a)) / den;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Block matching (section Block Matching)                              */
/* ------------------------------------------------------------------ */

typedef struct {
    double score;
    int64_t lin;
} cand_t;

static int cmp_cand(const void* a, const void* b)
{
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (x->score < y->score) return -1;
    if (x->score > y->score) return 1;
    return (x->lin > y->lin) - (x->lin < y->lin);
}

/* ---- Poisson-likelihood matching (section Metrics; subsection Exact
 * Finite-Count Moment Calibration) */

/* Anscombe transform A(n) = 2 sqrt(n + 3/8) (Def. Anscombe-SSD matching
 * statistic) */
static double anscombe(double n) { return 2.0 * sqrt(n + 0.375); }

/* Per-entry contribution phi_m(r, c) (eq. varphi) on raw counts r, c >= 0
 * (eq. raw-counts): the entrywise likelihood-ratio statistic of the
 * symmetric deviance (Prop. deviance as likelihood ratio; 0 log 0 = 0 and
 * zero when r + c = 0), the pooled Pearson term (zero when r + c = 0), or
 * half the squared difference of Anscombe transforms. */
double orc_phi(int32_t metric, double r, double c)
{
    const double s = r + c;
    if (metric == ORC_METRIC_DEVIANCE) {
        if (s <= 0.0) return 0.0;
        double v = 0.0;
        if (r > 0.0) v += r * log(2.0 * r / s);
        if (c > 0.0) v += c * log(2.0 * c / s);
        return 2.0 * v;
    }
    if (metric == ORC_METRIC_PEARSON) {
        if (s <= 0.0) return 0.0;
        return (c - r) * (c - r) / s;
    }
    if (metric == ORC_METRIC_ANSCOMBE) {
        const double d = anscombe(c) - anscombe(r);
        return 0.5 * d * d;
    }
    return (c - r) * (c - r);
}

/* Exact conditional moments of phi_m given the pooled count n (Prop.
 * universal finite-count moments): under the equal-rate null the reference
 * count is Bin(n, 1/2) given r + c = n (Lemma conditional Poisson
 * splitting), so mu = sum_x C(n, x) 2^-n phi(x, n - x) and v = sum_x
 * C(n, x) 2^-n phi(x, n - x)^2 - mu^2. */
int orc_count_moments(int32_t metric, int32_t n, double* mu, double* v)
{
    if (n < 0 || !mu || !v) return -1;
    double m1 = 0.0, m2 = 0.0;
    for (int32_t x = 0; x <= n; ++x) {
        const double w = exp(lgamma(n + 1.0) - lgamma(x + 1.0) - lgamma(n - x + 1.0) -
                             n * log(2.0));
        const double f = orc_phi(metric, (double)x, (double)(n - x));
        m1 += w * f;
        m2 += w * f * f;
    }
    *mu = m1;
    *v = m2 - m1 * m1;
    return 0;
}

/* Score and threshold of one pair under a policy, given the moments of
 * every pooled count that occurs (mu_tab, v_tab for n <= nmax):
 *   fixed:        d_m = sum phi / P against 1 + t sqrt(2 / P), the
 *                 high-count mean 1 and variance 2 per entry (Thm. common
 *                 high-count limit);
 *   reference:    d_m against T_ref = mean mu(2 r_i) + t sqrt(sum v(2 r_i)
 *                 / P^2) + beta rbar^kappa (Def. reference finite-count
 *                 threshold);
 *   standardized: Z = (sum phi - sum mu(r_i + c_i)) / sqrt(sum v(r_i +
 *                 c_i)), 0 when the variance sum is 0, against t (Def.
 *                 candidate-standardized distance).
 * The calibrated policies need integral counts. */
static int pair_score_tab(int32_t metric, int32_t policy, double t, double beta, double kappa,
                          int32_t P, const double* r, const double* c, const double* mu_tab,
                          const double* v_tab, int64_t nmax, double* score, double* threshold)
{
    double A = 0.0;
    for (int32_t i = 0; i < P; ++i) A += orc_phi(metric, r[i], c[i]);
    if (policy == ORC_POLICY_FIXED) {
        *score = A / P;
        *threshold = 1.0 + t * sqrt(2.0 / P);
        return 0;
    }
    if (policy == ORC_POLICY_REFERENCE) {
        double mu = 0.0, v = 0.0, rs = 0.0;
        for (int32_t i = 0; i < P; ++i) {
            const int64_t n = (int64_t)(2.0 * r[i]);
            if (n < 0 || n > nmax) return -1;
            mu += mu_tab[n];
            v += v_tab[n];
            rs += r[i];
        }
        *score = A / P;
        *threshold = mu / P + t * sqrt(v / ((double)P * P)) + beta * pow(rs / P, kappa);
        return 0;
    }
    double M = 0.0, S = 0.0;
    for (int32_t i = 0; i < P; ++i) {
        const int64_t n = (int64_t)(r[i] + c[i]);
        if (n < 0 || n > nmax) return -1;
        M += mu_tab[n];
        S += v_tab[n];
    }
    *score = S > 0.0 ? (A - M) / sqrt(S) : 0.0;
    *threshold = t;
    return 0;
}

static int moment_tables(int32_t metric, int64_t nmax, double** mu, double** v)
{
    *mu = (double*)malloc(sizeof(double) * (size_t)(nmax + 1));
    *v = (double*)malloc(sizeof(double) * (size_t)(nmax + 1));
    if (!*mu || !*v) return -2;
    for (int64_t n = 0; n <= nmax; ++n)
        if (orc_count_moments(metric, (int32_t)n, &(*mu)[n], &(*v)[n]) != 0) return -1;
    return 0;
}

int orc_pair_score(int32_t metric, int32_t policy, double t, double beta, double kappa,
                   int32_t P, const double* r, const double* c, double* score, double* threshold)
{
    if (P < 1 || !r || !c || !score || !threshold) return -1;
    if (metric < ORC_METRIC_DEVIANCE || metric > ORC_METRIC_ANSCOMBE) return -1;
    double nmax = 0.0;
    for (int32_t i = 0; i < P; ++i) {
        if (r[i] < 0.0 || c[i] < 0.0) return -1;
        if (2.0 * r[i] > nmax) nmax = 2.0 * r[i];
        if (r[i] + c[i] > nmax) nmax = r[i] + c[i];
    }
    double *mu = NULL, *v = NULL;
    int rc = 0;
    if (policy != ORC_POLICY_FIXED) rc = moment_tables(metric, (int64_t)nmax, &mu, &v);
    if (rc == 0)
        rc = pair_score_tab(metric, policy, t, beta, kappa, P, r, c, mu, v, (int64_t)nmax, score,
                            threshold);
    free(mu);
    free(v);
    return rc;
}

/* For every reference origin: score every candidate origin of the clipped
 * search window (section Block Matching), keep the reference in slot 0 and
 * the best others by (score, lin).
 *   HT stage, Gaussian:  d = SSD - gamma * 2 P sigma^2           (Prop. Gaussian
 *                        SSD noise bias with white noise, Def. corrected SSD)
 *   HT stage, Poisson:   d = SSD - gamma * s_P sum [p_i + q_i]_+ (Prop. scaled-
 *                        Poisson SSD noise bias, Def. corrected SSD).  With
 *                        integral counts the sums run on the equivalent raw
 *                        counts kappa = rint(y / s_P), eq. raw-counts, which
 *                        gives d = s_P^2 (SSD_kappa - gamma sum[kappa_p+kappa_q]_+)
 *                        exactly (unit invariance of count statistics).
 *   Wiener stage:        d = SSD on the pilot (paired groups definition).
 * Acceptance is d < tau (tau compared in the same units as the score).
 * score[] receives d in stored units (reference: 0).  accepted[] (nullable)
 * receives the number of accepted non-reference candidates. */
int orc_match(const orc_cfg* c, int32_t stage, const double* src, const double* y,
              const int64_t* refs, int64_t nrefs, int32_t* match, int32_t* count,
              double* score, int32_t* accepted)
{
    if (check_cfg(c) != 0 || !src || !refs || !match || !count) return -1;
    const int D = c->ndim;
    const int P = patch_size_of(c);
    const int gmax = c->group_max;
    int64_t st[ORC_MAXD];
    strides_of(c, st);
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)P);
    int64_t wn = 1;
    for (int d = 0; d < D; ++d) wn *= c->search[d];
    cand_t* cand = (cand_t*)malloc(sizeof(cand_t) * (size_t)wn);
    double* kap = NULL;
    const int64_t V = volume_of(c);
    const int integral = (stage == ORC_STAGE_HT && c->noise_kind == ORC_NOISE_POISSON &&
                          c->counts_integral);
    if (!off || !cand) { free(off); free(cand); return -2; }
    patch_offsets(c, st, off);
    if (integral) {
        kap = (double*)malloc(sizeof(double) * (size_t)V);
        if (!kap) { free(off); free(cand); return -2; }
        for (int64_t u = 0; u < V; ++u) kap[u] = nearbyint(y[u] / c->s_p);
    }
    double tau_eff = c->tau;
    if (integral) tau_eff = c->tau / (c->s_p * c->s_p);
    /* Poisson-likelihood metrics in the HT stage: raw counts [y / s_P]_+
     * (integral counts rounded), scores and thresholds per pair */
    const int pois = stage == ORC_STAGE_HT && c->noise_kind == ORC_NOISE_POISSON &&
                     c->metric != ORC_METRIC_SSD;
    double *rawc = NULL, *mu_tab = NULL, *v_tab = NULL, *rr = NULL, *cc = NULL;
    int64_t nmax = 0;
    if (stage == ORC_STAGE_HT && c->metric != ORC_METRIC_SSD && !pois) {
        free(kap); free(off); free(cand);
        return -1;
    }
    if (pois) {
        if (c->policy != ORC_POLICY_FIXED && !c->counts_integral) {
            free(kap); free(off); free(cand);
            return -1;
        }
        rawc = (double*)malloc(sizeof(double) * (size_t)V);
        rr = (double*)malloc(sizeof(double) * (size_t)P);
        cc = (double*)malloc(sizeof(double) * (size_t)P);
        if (!rawc || !rr || !cc) {
            free(kap); free(off); free(cand); free(rawc); free(rr); free(cc);
            return -2;
        }
        double mx = 0.0;
        for (int64_t u = 0; u < V; ++u) {
            double k = c->counts_integral ? nearbyint(y[u] / c->s_p) : y[u] / c->s_p;
            rawc[u] = k > 0.0 ? k : 0.0;
            if (rawc[u] > mx) mx = rawc[u];
        }
        nmax = (int64_t)(2.0 * mx);
        if (c->policy != ORC_POLICY_FIXED &&
            moment_tables(c->metric, nmax, &mu_tab, &v_tab) != 0) {
            free(kap); free(off); free(cand); free(rawc); free(rr); free(cc);
            free(mu_tab); free(v_tab);
            return -2;
        }
    }

    for (int64_t g = 0; g < nrefs; ++g) {
        const int64_t r = refs[g];
        int64_t rc[ORC_MAXD], lo[ORC_MAXD], hi[ORC_MAXD], ext[ORC_MAXD];
        int64_t rem = r;
        for (int d = D - 1; d >= 0; --d) { rc[d] = rem % c->shape[d]; rem /= c->shape[d]; }
        int64_t ncand_box = 1;
        for (int d = 0; d < D; ++d) {
            int64_t ell = c->shape[d] - c->patch[d];
            lo[d] = rc[d] - c->search[d] / 2;
            hi[d] = rc[d] + c->search[d] - 1 - c->search[d] / 2;
            if (lo[d] < 0) lo[d] = 0;
            if (hi[d] > ell) hi[d] = ell;
            ext[d] = hi[d] - lo[d] + 1;
            ncand_box *= ext[d];
        }
        int64_t nc = 0;
        double thr_ref = 0.0;  /* Poisson metrics: the reference's threshold */
        for (int64_t t = 0; t < ncand_box; ++t) {
            int64_t tr = t, clin = 0;
            for (int d = D - 1; d >= 0; --d) {
                clin += (lo[d] + tr % ext[d]) * st[d];
                tr /= ext[d];
            }
            if (clin == r) continue;
            double s = 0.0;
            if (pois) {
                for (int i = 0; i < P; ++i) {
                    rr[i] = rawc[r + off[i]];
                    cc[i] = rawc[clin + off[i]];
                }
                double thr = 0.0;
                if (pair_score_tab(c->metric, c->policy, c->match_t, c->struct_beta,
                                   c->struct_kappa, P, rr, cc, mu_tab, v_tab, nmax, &s, &thr) != 0) {
                    free(kap); free(off); free(cand); free(rawc); free(rr); free(cc);
                    free(mu_tab); free(v_tab);
                    return -1;
                }
                thr_ref = thr;
            } else if (stage == ORC_STAGE_WIENER) {
                for (int i = 0; i < P; ++i) {
                    double df = src[clin + off[i]] - src[r + off[i]];
                    s += df * df;
                }
            } else if (integral) {
                double ssd = 0.0, b = 0.0;
                for (int i = 0; i < P; ++i) {
                    double kp = kap[r + off[i]], kq = kap[clin + off[i]];
                    ssd += (kq - kp) * (kq - kp);
                    b += (kp + kq > 0.0) ? (kp + kq) : 0.0;
                }
                s = ssd - c->gamma * b;
            } else if (c->noise_kind == ORC_NOISE_POISSON) {
                double ssd = 0.0, b = 0.0;
                for (int i = 0; i < P; ++i) {
                    double p = src[r + off[i]], q = src[clin + off[i]];
                    ssd += (q - p) * (q - p);
                    b += (p + q > 0.0) ? (p + q) : 0.0;
                }
                s = ssd - c->gamma * c->s_p * b;
            } else if (c->noise_kind == ORC_NOISE_CORRELATED) {
                /* Prop. Gaussian SSD noise bias: B_G(Delta) = 2 P (c(0) -
                 * c(Delta)), Delta the displacement from the reference's
                 * origin to the candidate's */
                double ssd = 0.0;
                for (int i = 0; i < P; ++i) {
                    double df = src[clin + off[i]] - src[r + off[i]];
                    ssd += df * df;
                }
                int64_t cq[ORC_MAXD], dl[ORC_MAXD], z[ORC_MAXD];
                coords_of(c, clin, cq);
                for (int d = 0; d < D; ++d) { dl[d] = cq[d] - rc[d]; z[d] = 0; }
                double bg = 2.0 * (double)P * (acov_at(c, z) - acov_at(c, dl));
                s = ssd - c->gamma * bg;
            } else {
                double ssd = 0.0;
                for (int i = 0; i < P; ++i) {
                    double df = src[clin + off[i]] - src[r + off[i]];
                    ssd += df * df;
                }
                s = ssd - c->gamma * 2.0 * (double)P * c->sigma * c->sigma;
            }
            cand[nc].score = s;
            cand[nc].lin = clin;
            ++nc;
        }
        qsort(cand, (size_t)nc, sizeof(cand_t), cmp_cand);
        int64_t acc = 0;
        const double tau_g = pois ? thr_ref : tau_eff;
        for (int64_t i = 0; i < nc; ++i)
            if (cand[i].score < tau_g) ++acc;
        int64_t kacc = 1 + acc;
        if (kacc > gmax) kacc = gmax;
        int64_t K = pow2floor64(kacc);
        if (K < c->group_min) K = c->group_min;
        int64_t kcap = pow2floor64(1 + nc);
        if (K > kcap) K = kcap;
        count[g] = (int32_t)K;
        if (accepted) accepted[g] = (int32_t)acc;
        for (int t = 0; t < gmax; ++t) {
            match[g * gmax + t] = -1;
            if (score) score[g * gmax + t] = 0.0;
        }
        match[g * gmax] = (int32_t)r;
        for (int64_t t = 1; t < K; ++t) {
            match[g * gmax + t] = (int32_t)cand[t - 1].lin;
            if (score)
                score[g * gmax + t] = (integral && !pois) ? cand[t - 1].score * c->s_p * c->s_p
                                               : cand[t - 1].score;
        }
    }
    free(kap);
    free(off);
    free(cand);
    free(rawc);
    free(rr);
    free(cc);
    free(mu_tab);
    free(v_tab);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Collaborative filtering of one group                                 */
/* ------------------------------------------------------------------ */

/* Tensor with dims (K, j_0, ..., j_{D-1}) in C-order; apply the n x n
 * matrix M along `axis` (out[a] = sum_b M[a][b] in[b]). */
static void mode_product(double* x, const int* dims, int nd, int axis, const double* M,
                         double* tmp)
{
    int64_t outer = 1, inner = 1;
    for (int a = 0; a < axis; ++a) outer *= dims[a];
    for (int a = axis + 1; a < nd; ++a) inner *= dims[a];
    const int n = dims[axis];
    for (int64_t o = 0; o < outer; ++o)
        for (int64_t i = 0; i < inner; ++i) {
            for (int a = 0; a < n; ++a) {
                double s = 0.0;
                for (int b = 0; b < n; ++b) s += M[a * n + b] * x[(o * n + b) * inner + i];
                tmp[a] = s;
            }
            for (int a = 0; a < n; ++a) x[(o * n + a) * inner + i] = tmp[a];
        }
}

/* Per-stage constant data: transform matrices, window, offsets. */
typedef struct {
    int D, P, K;
    int dims[ORC_MAXD + 1];
    double* Tsp[ORC_MAXD];   /* spatial analysis per axis   */
    double* Usp[ORC_MAXD];   /* spatial synthesis per axis  */
    double* T2sp[ORC_MAXD];  /* elementwise squares of Tsp  */
    double* TspT[ORC_MAXD];  /* transpose of Usp (for U^T)  */
    double* H;               /* Haar K x K                  */
    double* Ht;              /* H^T                         */
    double* H2;              /* elementwise squares of H    */
    double* Hbuf[6];         /* Haar matrices for K = 1..32 */
    double* omega;           /* P-sample Kaiser window      */
    double* Tkron;           /* P x P spatial Kronecker     */
    int64_t* off;
    int64_t st[ORC_MAXD];
    double* tmp;
} stage_ctx;

static void ctx_free(stage_ctx* x)
{
    for (int d = 0; d < ORC_MAXD; ++d) {
        free(x->Tsp[d]); free(x->Usp[d]); free(x->T2sp[d]); free(x->TspT[d]);
    }
    for (int i = 0; i < 6; ++i) free(x->Hbuf[i]);
    free(x->H); free(x->Ht); free(x->H2);
    free(x->omega); free(x->Tkron); free(x->off); free(x->tmp);
    memset(x, 0, sizeof *x);
}

static int ctx_init(stage_ctx* x, const orc_cfg* c)
{
    memset(x, 0, sizeof *x);
    x->D = c->ndim;
    x->P = patch_size_of(c);
    strides_of(c, x->st);
    x->off = (int64_t*)malloc(sizeof(int64_t) * (size_t)x->P);
    x->omega = (double*)malloc(sizeof(double) * (size_t)x->P);
    x->tmp = (double*)malloc(sizeof(double) * 4096);
    x->Tkron = (double*)malloc(sizeof(double) * (size_t)x->P * (size_t)x->P);
    if (!x->off || !x->omega || !x->tmp || !x->Tkron) return -2;
    patch_offsets(c, x->st, x->off);
    double* wax[ORC_MAXD];
    for (int d = 0; d < x->D; ++d) {
        int n = c->patch[d];
        x->Tsp[d] = (double*)malloc(sizeof(double) * (size_t)n * n);
        x->Usp[d] = (double*)malloc(sizeof(double) * (size_t)n * n);
        x->T2sp[d] = (double*)malloc(sizeof(double) * (size_t)n * n);
        x->TspT[d] = (double*)malloc(sizeof(double) * (size_t)n * n);
        wax[d] = (double*)malloc(sizeof(double) * (size_t)n);
        if (!x->Tsp[d] || !x->Usp[d] || !x->T2sp[d] || !x->TspT[d] || !wax[d]) return -2;
        if (orc_spatial_matrices(c->spatial, n, x->Tsp[d], x->Usp[d]) != 0) return -1;
        for (int i = 0; i < n * n; ++i) x->T2sp[d][i] = x->Tsp[d][i] * x->Tsp[d][i];
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) x->TspT[d][a * n + b] = x->Usp[d][b * n + a];
        orc_kaiser(n, c->kaiser_beta, wax[d]);
    }
    /* window and spatial Kronecker product, patch samples in C-order */
    for (int i = 0; i < x->P; ++i) {
        int rem = i;
        int id[ORC_MAXD];
        for (int d = x->D - 1; d >= 0; --d) { id[d] = rem % c->patch[d]; rem /= c->patch[d]; }
        double w = 1.0;
        for (int d = 0; d < x->D; ++d) w *= wax[d][id[d]];
        x->omega[i] = w;
        for (int q = 0; q < x->P; ++q) {
            int rq = q;
            double t = 1.0;
            for (int d = x->D - 1; d >= 0; --d) {
                int qd = rq % c->patch[d];
                rq /= c->patch[d];
                t *= x->Tsp[d][qd * c->patch[d] + id[d]];
            }
            x->Tkron[q * x->P + i] = t;
        }
    }
    for (int d = 0; d < x->D; ++d) free(wax[d]);
    for (int m = 0; m < 6; ++m) {
        int K = 1 << m;
        x->Hbuf[m] = (double*)malloc(sizeof(double) * (size_t)K * K);
        if (!x->Hbuf[m]) return -2;
        orc_haar_matrix(K, x->Hbuf[m]);
    }
    x->H = (double*)malloc(sizeof(double) * 32 * 32);
    x->Ht = (double*)malloc(sizeof(double) * 32 * 32);
    x->H2 = (double*)malloc(sizeof(double) * 32 * 32);
    if (!x->H || !x->Ht || !x->H2) return -2;
    return 0;
}

static int ctx_set_group(stage_ctx* x, int K)
{
    int m = 0;
    while ((1 << m) < K) ++m;
    if ((1 << m) != K || m > 5) return -1;
    x->K = K;
    memcpy(x->H, x->Hbuf[m], sizeof(double) * (size_t)K * K);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            x->Ht[a * K + b] = x->H[b * K + a];
            x->H2[a * K + b] = x->H[a * K + b] * x->H[a * K + b];
        }
    return 0;
}

/* Apply the full group transform T = H_K (x) T_0 (x) ... (x) T_{D-1}. */
static void apply_forward(stage_ctx* x, double* t)
{
    mode_product(t, x->dims, x->D + 1, 0, x->H, x->tmp);
    for (int d = 0; d < x->D; ++d) mode_product(t, x->dims, x->D + 1, d + 1, x->Tsp[d], x->tmp);
}

/* Apply the full inverse U = T^-1 = H_K^T (x) U_0 (x) ... */
static void apply_inverse(stage_ctx* x, double* t)
{
    mode_product(t, x->dims, x->D + 1, 0, x->Ht, x->tmp);
    for (int d = 0; d < x->D; ++d) mode_product(t, x->dims, x->D + 1, d + 1, x->Usp[d], x->tmp);
}

/* Apply U^T = H_K (x) U_0^T (x) ... (for the aggregation functional h_g). */
static void apply_inverse_transpose(stage_ctx* x, double* t)
{
    mode_product(t, x->dims, x->D + 1, 0, x->H, x->tmp);
    for (int d = 0; d < x->D; ++d) mode_product(t, x->dims, x->D + 1, d + 1, x->TspT[d], x->tmp);
}

/* Filter one group (sections Hard Thresholding, Wiener Shrinkage,
 * Aggregation Weights).  Produces the transformed observation Y, the
 * coefficient noise variances, the shrunk coefficients C and the per-patch
 * reliability weights w. */
static int filter_group(stage_ctx* x, const orc_cfg* c, int stage, const double* y,
                        const double* pilot, int K, const int32_t* org, double* Yc,
                        double* var, double* C, double* w)
{
    const int P = x->P;
    const int n = K * P;
    if (ctx_set_group(x, K) != 0) return -1;
    x->dims[0] = K;
    for (int d = 0; d < x->D; ++d) x->dims[d + 1] = c->patch[d];

    double* mv = (double*)malloc(sizeof(double) * (size_t)n);
    double* gam = (double*)malloc(sizeof(double) * (size_t)n);
    double* shat = (double*)malloc(sizeof(double) * (size_t)n);
    double* att = (double*)malloc(sizeof(double) * (size_t)n);
    if (!mv || !gam || !shat || !att) { free(mv); free(gam); free(shat); free(att); return -2; }

    /* gather (Def. patch-group observation model; paired groups for Wiener) */
    for (int j = 0; j < K; ++j)
        for (int i = 0; i < P; ++i) {
            int64_t u = (int64_t)org[j] + x->off[i];
            Yc[j * P + i] = y[u];
            if (stage == ORC_STAGE_WIENER) gam[j * P + i] = pilot[u];
            /* variance map: Poisson m_v(u) = s_P [X^(u)]_+ with X^ = y in the
             * HT stage and the pilot in the Wiener stage (Def. Poisson
             * variance map); white Gaussian: sigma^2 everywhere */
            if (c->noise_kind == ORC_NOISE_POISSON) {
                double xs = (stage == ORC_STAGE_WIENER) ? pilot[u] : y[u];
                mv[j * P + i] = c->s_p * (xs > 0.0 ? xs : 0.0);
            } else {
                mv[j * P + i] = c->sigma * c->sigma;
            }
        }

    /* Y = T y_g, Gamma = T gamma_g (eq. paired-wiener-transforms) */
    apply_forward(x, Yc);
    if (stage == ORC_STAGE_WIENER) apply_forward(x, gam);

    /* sigma_k^2 = sum_i |T_ki|^2 m_v(u_i): diagonal propagation
     * (Prop. diagonal Poisson variance propagation); for separable T the
     * squared matrix is the Kronecker product of the squared factors. */
    memcpy(var, mv, sizeof(double) * (size_t)n);
    mode_product(var, x->dims, x->D + 1, 0, x->H2, x->tmp);
    for (int d = 0; d < x->D; ++d) mode_product(var, x->dims, x->D + 1, d + 1, x->T2sp[d], x->tmp);

    /* stationary correlated Gaussian noise: the group covariance is
     * Sigma_g[a][b] = c(u_b - u_a) over the source locations of the group
     * entries (Def. wide-sense stationary Gaussian noise; repeated voxels
     * give c(0) and are fully correlated), and the coefficient variances are
     * the diagonal of T Sigma_g T^H (Lemma covariance propagation), for
     * every plane */
    if (c->noise_kind == ORC_NOISE_CORRELATED) {
        double* S = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
        int64_t* uc = (int64_t*)malloc(sizeof(int64_t) * (size_t)n * ORC_MAXD);
        if (!S || !uc) { free(S); free(uc); free(mv); free(gam); free(shat); free(att); return -2; }
        for (int e = 0; e < n; ++e)
            coords_of(c, (int64_t)org[e / P] + x->off[e % P], uc + (size_t)e * ORC_MAXD);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                int64_t dl[ORC_MAXD];
                for (int d = 0; d < x->D; ++d)
                    dl[d] = uc[(size_t)b * ORC_MAXD + d] - uc[(size_t)a * ORC_MAXD + d];
                S[(size_t)a * n + b] = acov_at(c, dl);
            }
        /* rows of S (each a group-shaped array) times T^T, then the same on
         * the transpose: the result is (T S T^T)^T */
        for (int a = 0; a < n; ++a) apply_forward(x, S + (size_t)a * n);
        for (int a = 0; a < n; ++a)
            for (int b = a + 1; b < n; ++b) {
                double t = S[(size_t)a * n + b];
                S[(size_t)a * n + b] = S[(size_t)b * n + a];
                S[(size_t)b * n + a] = t;
            }
        for (int a = 0; a < n; ++a) apply_forward(x, S + (size_t)a * n);
        for (int e = 0; e < n; ++e) var[e] = S[(size_t)e * n + e];
        free(S);
        free(uc);
    }

    /* exact shared-source planes l < k_ex (Def. effective transform weights,
     * Def. partial shared-source Poisson variance model): group entries from
     * the same voxel are combined before squaring.  The correlated model is
     * exact already. */
    int kex = c->k_exact < K ? c->k_exact : K;
    if (c->noise_kind == ORC_NOISE_CORRELATED) kex = 0;
    if (kex > 0) {
        int64_t* ulin = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        int* order = (int*)malloc(sizeof(int) * (size_t)n);
        double* mvu = (double*)malloc(sizeof(double) * (size_t)n);
        if (!ulin || !order || !mvu) { free(ulin); free(order); free(mvu); return -2; }
        for (int e = 0; e < n; ++e) {
            ulin[e] = (int64_t)org[e / P] + x->off[e % P];
            order[e] = e;
        }
        /* sort entries by source voxel (insertion sort: n <= 4096) */
        for (int a = 1; a < n; ++a) {
            int v = order[a];
            int b = a - 1;
            while (b >= 0 && ulin[order[b]] > ulin[v]) { order[b + 1] = order[b]; --b; }
            order[b + 1] = v;
        }
        for (int e = 0; e < n; ++e) mvu[e] = mv[e];
        for (int l = 0; l < kex; ++l)
            for (int q = 0; q < P; ++q) {
                double s = 0.0;
                int a = 0;
                while (a < n) {
                    int b = a;
                    double t = 0.0;
                    while (b < n && ulin[order[b]] == ulin[order[a]]) {
                        int e = order[b];
                        t += x->H[l * K + e / P] * x->Tkron[q * P + e % P];
                        ++b;
                    }
                    s += t * t * mvu[order[a]];
                    a = b;
                }
                var[l * P + q] = s;
            }
        free(ulin);
        free(order);
        free(mvu);
    }

    /* magnitude of the terms of every coefficient, M_k = sum_i |T_ki| |y_i|
     * (the transform with absolute entries applied to |y|): the scale of
     * the rounding residue of Y_k, used by the hard threshold when
     * sigma_k = 0 */
    double* mag = NULL;
    if (c->shrink == ORC_SHRINK_HARD) {
        mag = (double*)malloc(sizeof(double) * (size_t)n);
        double* aH = (double*)malloc(sizeof(double) * (size_t)K * K);
        double* aT[ORC_MAXD] = {0};
        int ok = mag && aH;
        for (int d = 0; d < x->D && ok; ++d) {
            const int m = c->patch[d];
            aT[d] = (double*)malloc(sizeof(double) * (size_t)m * m);
            ok = aT[d] != NULL;
            for (int i = 0; ok && i < m * m; ++i) aT[d][i] = fabs(x->Tsp[d][i]);
        }
        if (ok) {
            for (int i = 0; i < K * K; ++i) aH[i] = fabs(x->H[i]);
            for (int j = 0; j < K; ++j)
                for (int i = 0; i < P; ++i) mag[j * P + i] = fabs(y[(int64_t)org[j] + x->off[i]]);
            mode_product(mag, x->dims, x->D + 1, 0, aH, x->tmp);
            for (int d = 0; d < x->D; ++d) mode_product(mag, x->dims, x->D + 1, d + 1, aT[d], x->tmp);
        }
        free(aH);
        for (int d = 0; d < x->D; ++d) free(aT[d]);
        if (!ok) { free(mag); free(mv); free(gam); free(shat); free(att); return -2; }
    }

    /* shrinkage */
    for (int e = 0; e < n; ++e) {
        double sig2 = var[e] > 0.0 ? var[e] : 0.0;
        double Y = Yc[e];
        if (c->shrink == ORC_SHRINK_HARD) {
            /* eq. hard-threshold: keep iff |Y_k| > lambda sigma_k.  With
             * integral counts exact ties occur (a coefficient fed by one
             * sample with kappa = lambda^2 has |Y| = lambda sigma exactly),
             * and the strict inequality drops them; the comparison is made
             * with a relative margin of 1e-9 so that a tie is not decided by
             * the rounding of Y and sigma.  With sigma_k = 0 the threshold is
             * 0 and a coefficient that is 0 in exact arithmetic keeps a
             * rounding residue; |Y_k| up to 1e-9 M_k counts as 0. */
            double a;
            if (sig2 > 0.0)
                a = (fabs(Y) > c->lambda * sqrt(sig2) * (1.0 + ORC_TIE_REL)) ? 1.0 : 0.0;
            else
                a = (fabs(Y) > ORC_TIE_REL * mag[e]) ? 1.0 : 0.0;
            att[e] = a;
            C[e] = a * Y;
            shat[e] = 0.0;
        } else if (c->shrink == ORC_SHRINK_SOFT) {
            /* eq. soft-threshold */
            double m = fabs(Y) - c->lambda * sqrt(sig2);
            if (m < 0.0) m = 0.0;
            C[e] = (Y > 0.0) ? m : ((Y < 0.0) ? -m : 0.0);
            att[e] = (Y != 0.0) ? m / fabs(Y) : 0.0;
            shat[e] = 0.0;
        } else {
            /* eq. pilot-power-family and eq. wiener-gain; the gain is 0 when
             * its denominator vanishes */
            double g2 = gam[e] * gam[e];
            double S = g2 - c->power_a * sig2;
            if (S < 0.0) S = 0.0;
            double den = S + c->s_v * sig2;
            double G = den > 0.0 ? S / den : 0.0;
            att[e] = G;
            shat[e] = S;
            C[e] = G * Y;   /* eq. wiener-diagonal-filter */
        }
    }

    /* reliability weights (Defs. hard-thresholding / Wiener weighting
     * models, coefficient domain; Def. aggregation-weight scope).
     * Windowed synthesized domain (Def. windowed synthesis metrics, Def.
     * windowed synthesized-domain weighting models): the surrogate is
     * tr(H F Sigma F^H) with the diagonal filter F and the diagonal of the
     * selected noise model, i.e. sum_k H_kk t_k with t_k the coefficient
     * term.  H = L^H L, L = W_g U_g; the column of L for coefficient k =
     * (l, q) is U_g e_k windowed: member j holds H_lj (U_sp e_q)(i) w(i),
     * so the patch-j diagonal entry is H_lj^2 h_q with h_q = sum_i (w(i)
     * (U_sp e_q)(i))^2, and the group entry sums it over j. */
    double* hq = NULL;
    if (c->weight_domain == ORC_WDOMAIN_WINDOWED) {
        hq = (double*)malloc(sizeof(double) * (size_t)P);
        if (!hq) { free(mag); free(mv); free(gam); free(shat); free(att); return -2; }
        for (int q = 0; q < P; ++q) {
            int qd[ORC_MAXD];
            int rem = q;
            for (int d = x->D - 1; d >= 0; --d) { qd[d] = rem % c->patch[d]; rem /= c->patch[d]; }
            double s = 0.0;
            for (int i = 0; i < P; ++i) {
                int ri = i;
                double col = 1.0;
                for (int d = x->D - 1; d >= 0; --d) {
                    const int n = c->patch[d];
                    col *= x->Usp[d][(ri % n) * n + qd[d]];
                    ri /= n;
                }
                const double v = x->omega[i] * col;
                s += v * v;
            }
            hq[q] = s;
        }
    }
    double* rl = x->tmp + 2048;   /* per-plane surrogates r_l, K <= 32 */
    for (int l = 0; l < K; ++l) {
        double s = 0.0;
        for (int q = 0; q < P; ++q) {
            int e = l * P + q;
            double a2 = att[e] * att[e];
            double sig2 = var[e] > 0.0 ? var[e] : 0.0;
            double tk;
            if (c->weight_model == ORC_W_CLASSIC) tk = a2;
            else if (c->weight_model == ORC_W_VARIANCE) tk = a2 * sig2;
            else tk = a2 * sig2 + (1.0 - att[e]) * (1.0 - att[e]) * shat[e];
            s += hq ? hq[q] * tk : tk;
        }
        rl[l] = s;
    }
    if (hq && c->weight_scope == ORC_SCOPE_GROUP) {
        /* group diagonal: sum_j H_lj^2 h_q */
        double R = 0.0;
        for (int l = 0; l < K; ++l) {
            double hl = 0.0;
            for (int j = 0; j < K; ++j) hl += x->H2[l * K + j];
            R += hl * rl[l];
        }
        double wg = R > 0.0 ? 1.0 / R : 1.0;
        for (int j = 0; j < K; ++j) w[j] = wg;
    } else if (c->weight_scope == ORC_SCOPE_GROUP) {
        double R = 0.0;
        for (int l = 0; l < K; ++l) R += rl[l];
        double wg = R > 0.0 ? 1.0 / R : 1.0;
        for (int j = 0; j < K; ++j) w[j] = wg;
    } else {
        /* R_j = sum_l |V_{j l}|^2 r_l with V = H^-1 = H^T, so V_{j l} = H_{l j} */
        for (int j = 0; j < K; ++j) {
            double R = 0.0;
            for (int l = 0; l < K; ++l) R += x->H2[l * K + j] * rl[l];
            w[j] = R > 0.0 ? 1.0 / R : 1.0;
        }
    }
    free(hq);
    free(mag);
    free(mv);
    free(gam);
    free(shat);
    free(att);
    return 0;
}

int orc_group_coeffs(const orc_cfg* c, int32_t stage, const double* y, const double* pilot,
                     int32_t K, const int32_t* origins, double* Y, double* var, double* C,
                     double* w)
{
    if (check_cfg(c) != 0) return -1;
    stage_ctx x;
    int rc = ctx_init(&x, c);
    if (rc == 0) rc = filter_group(&x, c, stage, y, pilot, K, origins, Y, var, C, w);
    ctx_free(&x);
    return rc;
}

/* Stage-isolated filtering on given match lists: per group the synthesized
 * (windowless) patches p = U C (Def. pilot group) and the patch weights. */
int orc_filter(const orc_cfg* c, int32_t stage, const double* y, const double* pilot,
               int64_t nrefs, const int32_t* match, const int32_t* count, double* patches,
               double* weights)
{
    if (check_cfg(c) != 0) return -1;
    if (stage == ORC_STAGE_WIENER && !pilot) return -1;
    stage_ctx x;
    int rc = ctx_init(&x, c);
    const int P = x.P, gmax = c->group_max;
    double* Y = (double*)malloc(sizeof(double) * 4096 * 4);
    double* var = Y + 4096;
    double* C = Y + 8192;
    double* w = Y + 12288;
    if (!Y) rc = -2;
    for (int64_t g = 0; rc == 0 && g < nrefs; ++g) {
        int K = count[g];
        rc = filter_group(&x, c, stage, y, pilot, K, match + g * gmax, Y, var, C, w);
        if (rc != 0) break;
        apply_inverse(&x, C);
        for (int j = 0; j < gmax; ++j) {
            weights[g * gmax + j] = j < K ? w[j] : 0.0;
            for (int i = 0; i < P; ++i)
                patches[(g * gmax + j) * P + i] = j < K ? C[j * P + i] : 0.0;
        }
    }
    free(Y);
    ctx_free(&x);
    return rc;
}

/* Weighted overlap-add of given patches (Def. weighted overlap-add).  With
 * mass conservation the per-group offset alpha_g is the unique constant
 * that satisfies the group constraint zeta_g^T (p_g + alpha 1) = zeta_g^T y_g
 * (Prop. exactness of the constant-synthesis correction) with the weights
 * and denominator eta of the first sweep held fixed (Remark fixed
 * aggregation weights).  eta (nullable) receives the denominator. */
int orc_aggregate(const orc_cfg* c, const double* y, int64_t nrefs, const int32_t* match,
                  const int32_t* count, const double* patches, const double* weights,
                  double* out, double* eta)
{
    if (check_cfg(c) != 0) return -1;
    stage_ctx x;
    int rc = ctx_init(&x, c);
    const int64_t V = volume_of(c);
    const int P = x.P, gmax = c->group_max;
    double* num = (double*)calloc((size_t)V, sizeof(double));
    double* den = (double*)calloc((size_t)V, sizeof(double));
    if (!num || !den) rc = -2;
    for (int64_t g = 0; rc == 0 && g < nrefs; ++g)
        for (int j = 0; j < count[g]; ++j) {
            double wj = weights[g * gmax + j];
            for (int i = 0; i < P; ++i) {
                int64_t u = (int64_t)match[g * gmax + j] + x.off[i];
                den[u] += wj * x.omega[i];
                if (!c->mass_conservation)
                    num[u] += wj * x.omega[i] * patches[(g * gmax + j) * P + i];
            }
        }
    if (rc == 0 && c->mass_conservation) {
        for (int64_t g = 0; g < nrefs; ++g) {
            double zs = 0.0, zr = 0.0;
            for (int j = 0; j < count[g]; ++j)
                for (int i = 0; i < P; ++i) {
                    int64_t u = (int64_t)match[g * gmax + j] + x.off[i];
                    double zeta = weights[g * gmax + j] * x.omega[i] / den[u];
                    zs += zeta;
                    zr += zeta * (y[u] - patches[(g * gmax + j) * P + i]);
                }
            double alpha = zs > 0.0 ? zr / zs : 0.0;
            for (int j = 0; j < count[g]; ++j)
                for (int i = 0; i < P; ++i) {
                    int64_t u = (int64_t)match[g * gmax + j] + x.off[i];
                    num[u] += weights[g * gmax + j] * x.omega[i] *
                              (patches[(g * gmax + j) * P + i] + alpha);
                }
        }
    }
    if (rc == 0)
        for (int64_t u = 0; u < V; ++u) {
            out[u] = den[u] > 0.0 ? num[u] / den[u] : 0.0;
            if (eta) eta[u] = den[u];
        }
    free(num);
    free(den);
    ctx_free(&x);
    return rc;
}

/* One complete stage: schedule, matching, filtering, aggregation.  With
 * mass conservation the stage runs in two sweeps (Remark fixed aggregation
 * weights): the first gives the weights and eta, the second applies the
 * coefficient-domain correction C + (d_g / zeta^T 1) m_g with
 * h_g = U^T zeta_g, d_g = zeta^T y_g - h_g^T C_g, m_g = U^-1 1 = T 1
 * (Defs. normalized aggregation functional, aggregation-aware
 * constant-synthesis correction) and aggregates the corrected patches. */
int orc_run_stage(const orc_cfg* c, int32_t stage, const double* y, const double* pilot,
                  double* out)
{
    if (check_cfg(c) != 0) return -1;
    if (stage == ORC_STAGE_WIENER && !pilot) return -1;
    int64_t nrefs = orc_schedule(c, NULL, 0);
    if (nrefs < 0) return (int)nrefs;
    const int64_t V = volume_of(c);
    const int gmax = c->group_max;
    int64_t* refs = (int64_t*)malloc(sizeof(int64_t) * (size_t)nrefs);
    int32_t* match = (int32_t*)malloc(sizeof(int32_t) * (size_t)nrefs * gmax);
    int32_t* count = (int32_t*)malloc(sizeof(int32_t) * (size_t)nrefs);
    double* num = (double*)calloc((size_t)V, sizeof(double));
    double* den = (double*)calloc((size_t)V, sizeof(double));
    double* buf = (double*)malloc(sizeof(double) * 4096 * 6);
    int rc = 0;
    stage_ctx x;
    memset(&x, 0, sizeof x);
    if (!refs || !match || !count || !num || !den || !buf) rc = -2;
    if (rc == 0) orc_schedule(c, refs, nrefs);
    if (rc == 0)
        rc = orc_match(c, stage, stage == ORC_STAGE_WIENER ? pilot : y, y, refs, nrefs, match,
                       count, NULL, NULL);
    if (rc == 0) rc = ctx_init(&x, c);
    const int P = x.P;
    double *Y = buf, *var = buf + 4096, *C = buf + 8192, *w = buf + 12288, *z = buf + 16384,
           *m = buf + 20480;
    for (int sweep = 0; rc == 0 && sweep < (c->mass_conservation ? 2 : 1); ++sweep) {
        for (int64_t g = 0; rc == 0 && g < nrefs; ++g) {
            const int K = count[g];
            const int32_t* org = match + g * gmax;
            rc = filter_group(&x, c, stage, y, pilot, K, org, Y, var, C, w);
            if (rc != 0) break;
            if (c->mass_conservation && sweep == 0) {
                for (int j = 0; j < K; ++j)
                    for (int i = 0; i < P; ++i) den[(int64_t)org[j] + x.off[i]] += w[j] * x.omega[i];
                continue;
            }
            if (c->mass_conservation) {
                /* zeta_{g,j}(u) = w_j omega(u) / eta(u) in stacking order */
                double zsum = 0.0, zy = 0.0;
                for (int j = 0; j < K; ++j)
                    for (int i = 0; i < P; ++i) {
                        int64_t u = (int64_t)org[j] + x.off[i];
                        z[j * P + i] = w[j] * x.omega[i] / den[u];
                        zsum += z[j * P + i];
                        zy += z[j * P + i] * y[u];
                    }
                /* h_g = U^T zeta_g ; d_g = zeta^T y_g - h_g^T C_g */
                apply_inverse_transpose(&x, z);
                double hC = 0.0;
                for (int e = 0; e < K * P; ++e) hC += z[e] * C[e];
                double dg = zy - hC;
                /* m_g = U^-1 1 = T 1 */
                for (int e = 0; e < K * P; ++e) m[e] = 1.0;
                apply_forward(&x, m);
                if (zsum > 0.0)
                    for (int e = 0; e < K * P; ++e) C[e] += dg / zsum * m[e];
            }
            apply_inverse(&x, C);
            for (int j = 0; j < K; ++j)
                for (int i = 0; i < P; ++i) {
                    int64_t u = (int64_t)org[j] + x.off[i];
                    num[u] += w[j] * x.omega[i] * C[j * P + i];
                    if (!c->mass_conservation) den[u] += w[j] * x.omega[i];
                }
        }
    }
    if (rc == 0)
        for (int64_t u = 0; u < V; ++u) out[u] = den[u] > 0.0 ? num[u] / den[u] : 0.0;
    ctx_free(&x);
    free(refs);
    free(match);
    free(count);
    free(num);
    free(den);
    free(buf);
    return rc;
}

/* Two-stage driver (section Method Overview): the hard-threshold stage on
 * y gives the pilot, the Wiener stage matches on the pilot and filters y. */
int orc_denoise(const orc_cfg* ht, const orc_cfg* wie, const double* y, double* pilot,
                double* out)
{
    int rc = orc_run_stage(ht, ORC_STAGE_HT, y, NULL, pilot);
    if (rc != 0) return rc;
    return orc_run_stage(wie, ORC_STAGE_WIENER, y, pilot, out);
}
