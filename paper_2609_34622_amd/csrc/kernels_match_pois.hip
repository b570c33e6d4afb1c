// Block matching with the Poisson-likelihood metrics (section Metrics:
// Defs. Poisson deviance, Poisson Pearson and Anscombe-SSD matching
// statistics, eq. varphi; subsection Exact Finite-Count Moment
// Calibration: Def. reference finite-count threshold, Def.
// candidate-standardized distance), any array shape.
//
// One thread owns one reference.  Raw counts are rint(y / s_P) for integral
// counts and [y / s_P]_+ otherwise (eq. raw-counts).  Pass 1 scores every
// candidate of the clipped window in FP32 together with a bound on its
// round-off (the band), counts the accepted candidates and keeps the M + 1
// smallest scores.  The group size follows (acceptance re-decided in FP64
// for scores within their band of the threshold when that can change it).
// Pass 2 re-scores in FP64 every candidate whose FP32 score is within twice
// the largest band of the K-1-th smallest value, and keeps the best K-1 by
// (FP64 score, lin): the FP64 ranking's members all lie in that range, so
// the list is the FP64 ranking itself.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

#include "bmnd_internal.h"
#include "match_common.h"
#include "safe_index.h"

namespace bmnd {

namespace {

constexpr int kPoisThreads = 64;

// 1-D arrays: a block's 64 references (one array, grid.y) stage the counts
// of the union of their windows once in LDS, with a per-count term of the
// metric, when that region holds at most kStageCap samples
constexpr int kStageCap = 1024;

// per-count term staged beside the counts: n ln n for the deviance, the
// Anscombe transform 2 sqrt(n + 3/8) (its FP32 value, as phi32 forms it)
template <int METRIC>
__device__ __forceinline__ float pois_term(float n)
{
    if constexpr (METRIC == BMND_METRIC_DEVIANCE) return n > 0.f ? n * logf(n) : 0.f;
    else if constexpr (METRIC == BMND_METRIC_ANSCOMBE) return 2.f * sqrtf(n + 0.375f);
    else return 0.f;
}

// phi32 from staged counts r, c and their terms tr, tc: the deviance as
// 2 (s ln 2 + r ln r + c ln c - s ln s), s = r + c (the same value up to
// FP32 round-off, within the score's band); Anscombe and Pearson as phi32
template <int METRIC>
__device__ __forceinline__ float phi32s(float r, float c, float tr, float tc)
{
    if constexpr (METRIC == BMND_METRIC_DEVIANCE) {
        const float s = r + c;
        // s ln s from the hardware base-2 logarithm (about 1 ulp): its error
        // is far inside the score's round-off band
        const float ts = s > 0.f ? s * (__builtin_amdgcn_logf(s) * 0.69314718f) : 0.f;
        return 2.f * (__builtin_fmaf(s, 0.69314718f, tr + tc) - ts);
    } else if constexpr (METRIC == BMND_METRIC_ANSCOMBE) {
        const float d = tc - tr;
        return 0.5f * d * d;
    } else {
        const float s = r + c;
        const float d = c - r;
        return s > 0.f ? d * d * __builtin_amdgcn_rcpf(s) : 0.f;
    }
}

// per-entry contribution phi(r, c) (eq. varphi) in FP32: the deviance's
// 2 (r ln(2r/s) + c ln(2c/s)), Pearson's (c - r)^2 / s (both 0 for s = 0),
// and (A(c) - A(r))^2 / 2 with A(n) = 2 sqrt(n + 3/8)
template <int METRIC>
__device__ __forceinline__ float phi32(float r, float c)
{
    const float s = r + c;
    if constexpr (METRIC == BMND_METRIC_DEVIANCE) {
        const float is = __builtin_amdgcn_rcpf(s);
        const float t1 = r > 0.f ? r * logf(2.f * r * is) : 0.f;
        const float t2 = c > 0.f ? c * logf(2.f * c * is) : 0.f;
        return 2.f * (t1 + t2);
    } else if constexpr (METRIC == BMND_METRIC_PEARSON) {
        const float d = c - r;
        return s > 0.f ? d * d * __builtin_amdgcn_rcpf(s) : 0.f;
    } else {
        const float d = 2.f * sqrtf(c + 0.375f) - 2.f * sqrtf(r + 0.375f);
        return 0.5f * d * d;
    }
}

// the same in FP64 with separately rounded operations, in the statement's
// order (the plain FP64 value)
template <int METRIC>
__device__ __forceinline__ double phi64(double r, double c)
{
    const double s = __dadd_rn(r, c);
    if constexpr (METRIC == BMND_METRIC_DEVIANCE) {
        if (!(s > 0.0)) return 0.0;
        double v = 0.0;
        if (r > 0.0) v = __dadd_rn(v, __dmul_rn(r, log(__ddiv_rn(__dmul_rn(2.0, r), s))));
        if (c > 0.0) v = __dadd_rn(v, __dmul_rn(c, log(__ddiv_rn(__dmul_rn(2.0, c), s))));
        return __dmul_rn(2.0, v);
    } else if constexpr (METRIC == BMND_METRIC_PEARSON) {
        if (!(s > 0.0)) return 0.0;
        const double d = __dsub_rn(c, r);
        return __ddiv_rn(__dmul_rn(d, d), s);
    } else {
        const double d = __dsub_rn(__dmul_rn(2.0, sqrt(__dadd_rn(c, 0.375))),
                                   __dmul_rn(2.0, sqrt(__dadd_rn(r, 0.375))));
        return __dmul_rn(0.5, __dmul_rn(d, d));
    }
}

__device__ __forceinline__ int p2floor_p(int x) { return x <= 1 ? 1 : (1 << (31 - __clz(x))); }

// STAGED (1-D arrays): blocks of 64 references of one array (grid.y the
// array), the counts of their windows' union and their terms in LDS when
// the union holds at most kStageCap samples (else read from the array)
template <int METRIC, int GM, bool STAGED>
__global__ __launch_bounds__(kPoisThreads) void k_match_pois(MatchArgs a, int kmax)
{
    constexpr int M = GM > 1 ? GM - 1 : 1;
    constexpr int NS = M + 1;
    __shared__ double sel_s[M][kPoisThreads];
    __shared__ int sel_l[M][kPoisThreads];
    __shared__ float st_c[STAGED ? kStageCap : 1], st_t[STAGED ? kStageCap : 1];
    __shared__ int st_lo, st_hi;

    const Geo& g = a.g;
    long t;
    int b, gi;
    if constexpr (STAGED) {
        b = int(blockIdx.y);
        gi = int(blockIdx.x) * kPoisThreads + int(threadIdx.x);
        t = long(b) * a.n_refs + gi;
    } else {
        t = long(blockIdx.x) * kPoisThreads + threadIdx.x;
        if (t >= long(g.batch) * a.n_refs) return;
        b = int(t / a.n_refs);
        gi = int(t - long(b) * a.n_refs);
    }
    const bool valid = !STAGED || gi < a.n_refs;
    const int r = safe_origin(int(a.refs[valid ? gi : 0]), last_origin(g));
    const float* src = a.src + long(b) * g.V;
    const int P = g.P;

    // raw counts of a sample (non-finite or out-of-range integral counts are
    // flagged and read as 0)
    auto cnt32 = [&](float x) -> float {
        if (a.integral) {
            const float k = rintf(x * a.inv_sp);
            const bool ok = k >= 0.f ? k <= float(kmax) : k > -1e30f;
            if (!ok) atomicOr(a.range_flag, 1);
            return ok ? fmaxf(k, 0.f) : 0.f;
        }
        const float k = x * a.inv_sp;
        return k > 0.f ? k : 0.f;
    };
    auto cnt64 = [&](float x) -> double {
        if (a.integral) {
            const double k = rint(__ddiv_rn(double(x), a.s_p_d));
            return (k > 0.0 && k <= double(kmax)) ? k : 0.0;
        }
        const double k = __ddiv_rn(double(x), a.s_p_d);
        return k > 0.0 ? k : 0.0;
    };
    // pooled counts index the moment tables (beyond them: flagged, clamped)
    auto tab = [&](float n) -> int {
        const int k = int(n);
        if (k > a.nmom) {
            atomicOr(a.range_flag, 1);
            return a.nmom;
        }
        return k;
    };

    // STAGED: the union of the block's windows (window origins plus a patch
    // along the one array axis)
    bool staged = false;
    int slo = 0;
    if constexpr (STAGED) {
        if (threadIdx.x == 0) {
            st_lo = INT_MAX;
            st_hi = INT_MIN;
        }
        __syncthreads();
        if (valid) {
            const int L3 = g.L[kAx - 1], W3 = g.W[kAx - 1];
            const int rc = r % L3;
            atomicMin(&st_lo, max(rc - W3 / 2, 0));
            atomicMax(&st_hi, min(rc + W3 - 1 - W3 / 2, g.ell[kAx - 1]) + g.j[kAx - 1] - 1);
        }
        __syncthreads();
        slo = st_lo;
        const int n_st = st_hi - st_lo + 1;
        staged = n_st <= kStageCap;   // uniform over the block
        if (staged) {
            for (int e = threadIdx.x; e < n_st; e += kPoisThreads) {
                const float k = cnt32(src[slo + e]);
                st_c[e] = k;
                st_t[e] = pois_term<METRIC>(k);
            }
        }
        __syncthreads();
        if (!valid) return;
    }

    int lo[kAx], hi[kAx];
    int ncand = 1;
    for (int d = 0; d < kAx; ++d) {
        const int rc = (r / g.st[d]) % g.L[d];
        lo[d] = max(rc - g.W[d] / 2, 0);
        hi[d] = min(rc + g.W[d] - 1 - g.W[d] / 2, g.ell[d]);
        ncand *= hi[d] - lo[d] + 1;
    }
    ncand -= 1;

    // the reference's threshold in FP64 (fixed: the high-count calibration;
    // reference: mean mu(2 r_i) + t sqrt(sum v(2 r_i)) / P + beta rbar^kappa;
    // standardized: t)
    double tau_d = a.tau_d;
    if (a.policy == BMND_POLICY_REFERENCE) {
        double mu = 0.0, v = 0.0, rs = 0.0;
        for (int i0 = 0; i0 < g.j[0]; ++i0)
            for (int i1 = 0; i1 < g.j[1]; ++i1)
                for (int i2 = 0; i2 < g.j[2]; ++i2)
                    for (int i3 = 0; i3 < g.j[3]; ++i3) {
                        const double rr = cnt64(src[r + i0 * g.st[0] + i1 * g.st[1] +
                                                    i2 * g.st[2] + i3]);
                        const int n = tab(float(2.0 * rr));
                        mu = __dadd_rn(mu, a.mu_d[n]);
                        v = __dadd_rn(v, a.v_d[n]);
                        rs = __dadd_rn(rs, rr);
                    }
        tau_d = __dadd_rn(__dadd_rn(__ddiv_rn(mu, double(P)),
                                    __dmul_rn(a.t_d, sqrt(__ddiv_rn(v, __dmul_rn(double(P), double(P)))))),
                          __dmul_rn(a.sbeta_d, pow(__ddiv_rn(rs, double(P)), a.skappa_d)));
    }
    const float tau_f = float(tau_d);
    const float tau_eps = 1e-6f * fabsf(tau_f) + 1e-30f;
    const float invP = 1.f / float(P);

    // FP32 score and its round-off bound
    auto score = [&](int c, float* band) -> float {
        float A = 0.f, Mu = 0.f, S = 0.f, ssum = 0.f;
        if (STAGED && staged) {
            // 1-D: the patch is one run along the last axis
            const int pr = r - slo, pc = c - slo;
            for (int i3 = 0; i3 < g.j[kAx - 1]; ++i3) {
                const float rr = st_c[pr + i3], cc = st_c[pc + i3];
                A += phi32s<METRIC>(rr, cc, st_t[pr + i3], st_t[pc + i3]);
                ssum += rr + cc;
                if (a.policy == BMND_POLICY_STANDARDIZED) {
                    const int n = tab(rr + cc);
                    Mu += a.mu_f[n];
                    S += a.v_f[n];
                }
            }
        } else
        for (int i0 = 0; i0 < g.j[0]; ++i0)
            for (int i1 = 0; i1 < g.j[1]; ++i1)
                for (int i2 = 0; i2 < g.j[2]; ++i2) {
                    const int o = i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2];
                    for (int i3 = 0; i3 < g.j[3]; ++i3) {
                        const float rr = cnt32(src[r + o + i3]), cc = cnt32(src[c + o + i3]);
                        A += phi32<METRIC>(rr, cc);
                        ssum += rr + cc;
                        if (a.policy == BMND_POLICY_STANDARDIZED) {
                            const int n = tab(rr + cc);
                            Mu += a.mu_f[n];
                            S += a.v_f[n];
                        }
                    }
                }
        const float bA = 4e-5f * (ssum + float(P));
        if (a.policy == BMND_POLICY_STANDARDIZED) {
            if (!(S > 0.f)) {
                *band = 0.f;
                return 0.f;
            }
            const float is = __builtin_amdgcn_rsqf(S);
            const float z = (A - Mu) * is;
            *band = (bA + 1e-5f * (Mu + float(P))) * is + 1e-5f * fabsf(z);
            return z;
        }
        const float d = A * invP;
        *band = bA * invP + 1e-6f * fabsf(d);
        return d;
    };
    // FP64 score in the statement's order (the oracle's value)
    auto score64 = [&](int c) -> double {
        double A = 0.0, Mu = 0.0, S = 0.0;
        for (int i0 = 0; i0 < g.j[0]; ++i0)
            for (int i1 = 0; i1 < g.j[1]; ++i1)
                for (int i2 = 0; i2 < g.j[2]; ++i2) {
                    const int o = i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2];
                    for (int i3 = 0; i3 < g.j[3]; ++i3) {
                        const double rr = cnt64(src[r + o + i3]), cc = cnt64(src[c + o + i3]);
                        A = __dadd_rn(A, phi64<METRIC>(rr, cc));
                        if (a.policy == BMND_POLICY_STANDARDIZED) {
                            const int n = tab(float(__dadd_rn(rr, cc)));
                            Mu = __dadd_rn(Mu, a.mu_d[n]);
                            S = __dadd_rn(S, a.v_d[n]);
                        }
                    }
                }
        if (a.policy == BMND_POLICY_STANDARDIZED)
            return S > 0.0 ? __ddiv_rn(__dsub_rn(A, Mu), sqrt(S)) : 0.0;
        return __ddiv_rn(A, double(P));
    };

    // ---- pass 1
    float s[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) s[m] = FLT_MAX;
    int acc = 0, namb = 0;
    float bmax = 0.f;
    for (int c0 = lo[0]; c0 <= hi[0]; ++c0)
        for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
            for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
                for (int c3 = lo[3]; c3 <= hi[3]; ++c3) {
                    const int c = c0 * g.st[0] + c1 * g.st[1] + c2 * g.st[2] + c3;
                    if (c == r) continue;
                    float bx;
                    float x = score(c, &bx);
                    if (!(fabsf(x) <= FLT_MAX)) x = FLT_MAX;  // never selected
                    // acc: certain acceptances; namb: the band around tau
                    const bool amb = fabsf(x - tau_f) <= bx + tau_eps;
                    acc += x < tau_f && !amb ? 1 : 0;
                    namb += amb ? 1 : 0;
                    bmax = fmaxf(bmax, bx);
#pragma unroll
                    for (int m = NS - 1; m >= 1; --m) s[m] = fminf(s[m], fmaxf(s[m - 1], x));
                    s[0] = fminf(s[0], x);
                }

    auto group_size = [&](int acc_) {
        int k = p2floor_p(min(1 + acc_, a.gmax));
        k = max(k, a.gmin);
        return min(k, p2floor_p(1 + ncand));
    };
    int K = group_size(acc);
    if (namb > 0 && group_size(acc + namb) != K) {
        acc = 0;
        for (int c0 = lo[0]; c0 <= hi[0]; ++c0)
            for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
                for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
                    for (int c3 = lo[3]; c3 <= hi[3]; ++c3) {
                        const int c = c0 * g.st[0] + c1 * g.st[1] + c2 * g.st[2] + c3;
                        if (c == r) continue;
                        float bx;
                        const float x = score(c, &bx);
                        if (!(fabsf(x) <= FLT_MAX)) continue;
                        if (fabsf(x - tau_f) <= bx + tau_eps)
                            acc += score64(c) < tau_d ? 1 : 0;
                        else
                            acc += x < tau_f ? 1 : 0;
                    }
        K = group_size(acc);
    }
    const int need = GM > 1 ? K - 1 : 0;
    int* out = a.match + t * a.gmax;
    out[0] = r;
    for (int m = 1; m < a.gmax; ++m) out[m] = -1;
    if (need == 0) {
        a.count[t] = K;
        return;
    }

    // ---- pass 2: FP64 ranking of every candidate that can be a member
    float theta = s[0];
#pragma unroll
    for (int m = 0; m < NS; ++m)
        if (m == need - 1) theta = s[m];
    const float thr = theta + 2.f * bmax;
    int got = 0;
    for (int c0 = lo[0]; c0 <= hi[0]; ++c0)
        for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
            for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
                for (int c3 = lo[3]; c3 <= hi[3]; ++c3) {
                    const int c = c0 * g.st[0] + c1 * g.st[1] + c2 * g.st[2] + c3;
                    if (c == r) continue;
                    float bx;
                    const float x = score(c, &bx);
                    if (!(x <= thr) || !(fabsf(x) <= FLT_MAX)) continue;
                    const double xd = score64(c);
                    if (!(fabs(xd) <= DBL_MAX)) continue;
                    if (got == need && !(xd < sel_s[need - 1][threadIdx.x])) continue;
                    int p = got < need ? got : need - 1;
                    while (p > 0 && sel_s[p - 1][threadIdx.x] > xd) {
                        sel_s[p][threadIdx.x] = sel_s[p - 1][threadIdx.x];
                        sel_l[p][threadIdx.x] = sel_l[p - 1][threadIdx.x];
                        --p;
                    }
                    sel_s[p][threadIdx.x] = xd;
                    sel_l[p][threadIdx.x] = c;
                    if (got < need) ++got;
                }
    // non-finite scores select fewer members than asked: the group is cut to
    // the largest power of two they fill
    if (got < need) K = p2floor_p(1 + got);
    a.count[t] = K;
    for (int m = 0; m < K - 1; ++m) out[1 + m] = sel_l[m][threadIdx.x];
}

template <int METRIC, bool STAGED>
hipError_t launch_metric_st(const MatchArgs& a, int kmax, dim3 grid, hipStream_t s)
{
    switch (a.gmax) {
    case 1: hipLaunchKernelGGL((k_match_pois<METRIC, 1, STAGED>), grid, dim3(kPoisThreads), 0, s, a, kmax); break;
    case 2: hipLaunchKernelGGL((k_match_pois<METRIC, 2, STAGED>), grid, dim3(kPoisThreads), 0, s, a, kmax); break;
    case 4: hipLaunchKernelGGL((k_match_pois<METRIC, 4, STAGED>), grid, dim3(kPoisThreads), 0, s, a, kmax); break;
    case 8: hipLaunchKernelGGL((k_match_pois<METRIC, 8, STAGED>), grid, dim3(kPoisThreads), 0, s, a, kmax); break;
    case 16: hipLaunchKernelGGL((k_match_pois<METRIC, 16, STAGED>), grid, dim3(kPoisThreads), 0, s, a, kmax); break;
    default: hipLaunchKernelGGL((k_match_pois<METRIC, 32, STAGED>), grid, dim3(kPoisThreads), 0, s, a, kmax); break;
    }
    return hipGetLastError();
}

template <int METRIC>
hipError_t launch_metric(const MatchArgs& a, int kmax, hipStream_t s)
{
    bool one_axis = true;   // the patch and the window run along the last axis only
    for (int d = 0; d < kAx - 1; ++d) one_axis = one_axis && a.g.L[d] == 1;
    if (one_axis) {
        const dim3 grid(unsigned((a.n_refs + kPoisThreads - 1) / kPoisThreads),
                        unsigned(a.g.batch));
        return launch_metric_st<METRIC, true>(a, kmax, grid, s);
    }
    const long n = long(a.g.batch) * a.n_refs;
    return launch_metric_st<METRIC, false>(a, kmax, dim3(unsigned((n + kPoisThreads - 1) / kPoisThreads)), s);
}

// ---- member scores (the optional score output of matching)

// The distance of every selected member to its reference, in the units the
// acceptance test compares with tau (section Block Matching: Def. corrected
// SSD and its bias terms, the Wiener stage's SSD on the pilot, the
// Poisson-likelihood statistics with their policies), evaluated in FP64
// from the source array: one thread per (array, reference, slot).  Slot 0
// (the reference) and slots at or beyond K hold 0.
enum ScoreKind { kScCount = 0, kScPoissonF = 1, kScGauss = 2, kScCorr = 3, kScPlain = 4,
                 kScMetric = 5 };

struct ScoreArgs {
    Geo g;
    const float* src;
    const int* match;
    const int* count;
    float* score;
    int n_refs, gmax;
    int kind, metric, policy, integral;
    double s_p, gamma, bias;     // bias: white Gaussian gamma 2 P sigma^2
    const double* bias_td;       // correlated Gaussian: per window offset
    const double* mu_d;
    const double* v_d;
    int nmom;
};

// offset of patch sample i (C order over the patch axes) from the origin
__device__ __forceinline__ int patch_sample_offset(const Geo& g, int i)
{
    int o = 0;
    for (int d = kAx - 1; d >= 0; --d) {
        o += (i % g.j[d]) * g.st[d];
        i /= g.j[d];
    }
    return o;
}

template <int METRIC>
__device__ double metric_score(const ScoreArgs& a, const float* y, int r, int q)
{
    const int P = a.g.P;
    double A = 0.0, M = 0.0, S = 0.0;
    for (int i = 0; i < P; ++i) {
        const int o = patch_sample_offset(a.g, i);
        double rk = __ddiv_rn(double(y[r + o]), a.s_p);
        double ck = __ddiv_rn(double(y[q + o]), a.s_p);
        if (a.integral) {
            rk = rint(rk);
            ck = rint(ck);
        }
        rk = fmax(rk, 0.0);
        ck = fmax(ck, 0.0);
        A = __dadd_rn(A, phi64<METRIC>(rk, ck));
        if (a.policy == BMND_POLICY_STANDARDIZED) {
            const double n = __dadd_rn(rk, ck);
            if (!(n <= double(a.nmom))) return __longlong_as_double(0x7FF8000000000000LL);
            M = __dadd_rn(M, a.mu_d[int(n)]);
            S = __dadd_rn(S, a.v_d[int(n)]);
        }
    }
    if (a.policy == BMND_POLICY_STANDARDIZED) return S > 0.0 ? __ddiv_rn(__dsub_rn(A, M), sqrt(S)) : 0.0;
    return __ddiv_rn(A, double(P));
}

__global__ __launch_bounds__(256) void k_member_scores(ScoreArgs a)
{
    const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
    const long total = long(a.g.batch) * a.n_refs * a.gmax;
    if (idx >= total) return;
    const int m = int(idx % a.gmax);
    const long t = idx / a.gmax;
    const int b = int(t / a.n_refs);
    const Geo& g = a.g;
    const int K = safe_count(a.count[t], a.gmax);
    double x = 0.0;
    if (m > 0 && m < K) {
        const int omax = last_origin(g);
        const int r = safe_origin(a.match[t * a.gmax], omax);
        const int q = safe_origin(a.match[t * a.gmax + m], omax);
        const float* y = a.src + long(b) * g.V;
        if (a.kind == kScMetric) {
            if (a.metric == BMND_METRIC_DEVIANCE) x = metric_score<BMND_METRIC_DEVIANCE>(a, y, r, q);
            else if (a.metric == BMND_METRIC_PEARSON) x = metric_score<BMND_METRIC_PEARSON>(a, y, r, q);
            else x = metric_score<BMND_METRIC_ANSCOMBE>(a, y, r, q);
        } else {
            double ssd = 0.0, bsum = 0.0;
            for (int i = 0; i < g.P; ++i) {
                const int o = patch_sample_offset(g, i);
                double p = double(y[r + o]), c = double(y[q + o]);
                if (a.kind == kScCount) {
                    p = rint(__ddiv_rn(p, a.s_p));
                    c = rint(__ddiv_rn(c, a.s_p));
                }
                const double df = __dsub_rn(c, p);
                ssd = __dadd_rn(ssd, __dmul_rn(df, df));
                const double pc = __dadd_rn(p, c);
                if (pc > 0.0) bsum = __dadd_rn(bsum, pc);
            }
            if (a.kind == kScCount) {
                x = __dmul_rn(__dmul_rn(a.s_p, a.s_p), __dsub_rn(ssd, __dmul_rn(a.gamma, bsum)));
            } else if (a.kind == kScPoissonF) {
                x = __dsub_rn(ssd, __dmul_rn(__dmul_rn(a.gamma, a.s_p), bsum));
            } else if (a.kind == kScGauss) {
                x = __dsub_rn(ssd, a.bias);
            } else if (a.kind == kScCorr) {
                // window offset of the displacement, C order over the W_d offsets
                int wo = 0, wst = 1;
                for (int d = kAx - 1; d >= 0; --d) {
                    const int rc = (r / g.st[d]) % g.L[d], qc = (q / g.st[d]) % g.L[d];
                    wo += (qc - rc + g.W[d] / 2) * wst;
                    wst *= g.W[d];
                }
                x = __dsub_rn(ssd, a.bias_td[wo]);
            } else {
                x = ssd;
            }
        }
    }
    a.score[idx] = float(x);
}

}  // namespace

hipError_t launch_member_scores(const StageCfg& c, const float* src, const int* match,
                                const int* count, int n_refs, float* score,
                                const MomentTables* mom, hipStream_t s)
{
    ScoreArgs a{};
    a.g = c.g;
    a.src = src;
    a.match = match;
    a.count = count;
    a.score = score;
    a.n_refs = n_refs;
    a.gmax = c.gmax;
    a.s_p = c.s_p;
    a.gamma = c.gamma;
    a.metric = c.metric;
    a.policy = c.policy;
    a.integral = c.counts_integral ? 1 : 0;
    if (c.stage == BMND_STAGE_WIENER) {
        a.kind = kScPlain;
    } else if (c.metric != BMND_METRIC_SSD) {
        if (!mom) return hipErrorInvalidValue;
        a.kind = kScMetric;
        a.mu_d = mom->mu64;
        a.v_d = mom->v64;
        a.nmom = mom->nmax;
    } else if (c.integral) {
        a.kind = kScCount;
    } else if (c.noise == BMND_NOISE_POISSON) {
        a.kind = kScPoissonF;
    } else if (c.noise == BMND_NOISE_CORRELATED) {
        a.kind = kScCorr;
        a.bias_td = c.corr.bias;
    } else {
        a.kind = kScGauss;
        a.bias = c.gamma * 2.0 * c.g.P * c.sigma * c.sigma;
    }
    const long total = long(c.g.batch) * n_refs * c.gmax;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_member_scores, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_match_pois(const MatchArgs& a, int metric, int kmax, hipStream_t s)
{
    if (metric == BMND_METRIC_DEVIANCE) return launch_metric<BMND_METRIC_DEVIANCE>(a, kmax, s);
    if (metric == BMND_METRIC_PEARSON) return launch_metric<BMND_METRIC_PEARSON>(a, kmax, s);
    return launch_metric<BMND_METRIC_ANSCOMBE>(a, kmax, s);
}

}  // namespace bmnd
