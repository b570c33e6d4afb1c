// BMND HIP kernels for gfx950 (MI355X).
//
// Layout conventions: every array is viewed with 4 canonical axes (leading
// singleton axes pad lower dimensionalities); arrays of a batch are stored
// back to back, V samples each.  A group of K members is a K x j0 x j1 x
// j2 x j3 tensor in LDS (member axis slowest).
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>

#include "bmnd_internal.h"
#include "filter_common.h"
#include "filter_nd.h"
#include "exact_planes.h"
#include "corr_noise.h"
#include "match_common.h"

namespace bmnd {

// Set by the matching kernels when a count lies outside the range in which
// the int32 count-domain score is exact (read by bmnd_stream_status).
__device__ int g_range_flag;

namespace {

constexpr int kMatchThreads = 64;
constexpr int kFilterThreads = 256;
constexpr double kTieRel = 1e-9;  // relative tie margin of the hard threshold

// ---------------------------------------------------------------------------
// Equivalent raw counts and their patch sums (eq. raw-counts; the plug-in
// Poisson bias needs sum_i [p_i + q_i]_+ = S(p) + S(q) for counts >= 0).
// ---------------------------------------------------------------------------

__global__ void k_counts(Geo g, const float* __restrict__ y, float inv_sp, int kmax,
                         int* __restrict__ kappa, int* __restrict__ flag)
{
    const long n = long(g.batch) * g.V;
    for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += long(gridDim.x) * blockDim.x) {
        // non-finite or out-of-range counts are flagged (and scored as 0)
        const float rk = rintf(y[i] * inv_sp);
        const bool ok = rk >= 0.f && rk <= float(kmax);
        if (!ok) atomicOr(flag, 1);
        kappa[i] = ok ? int(rk) : 0;
    }
}

__global__ void k_patch_sums(Geo g, const int* __restrict__ kappa, int* __restrict__ psum)
{
    const long n = long(g.batch) * g.V;
    for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += long(gridDim.x) * blockDim.x) {
        const int b = int(i / g.V);
        const int u = int(i - long(b) * g.V);
        int c[kAx];
        bool valid = true;
        for (int d = 0; d < kAx; ++d) {
            c[d] = (u / g.st[d]) % g.L[d];
            valid = valid && c[d] <= g.ell[d];
        }
        int s = 0;
        if (valid) {
            const int* base = kappa + long(b) * g.V + u;
            for (int i0 = 0; i0 < g.j[0]; ++i0)
                for (int i1 = 0; i1 < g.j[1]; ++i1)
                    for (int i2 = 0; i2 < g.j[2]; ++i2) {
                        const int* row = base + i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2];
                        for (int i3 = 0; i3 < g.j[3]; ++i3) s += row[i3];
                    }
        }
        psum[i] = s;
    }
}

// ---------------------------------------------------------------------------
// Block matching (section Block Matching).
// One thread owns one reference.  Pass 1 scores every candidate of the
// clipped window, counts the accepted ones (score < tau) and keeps the
// M = group_max - 1 smallest score values with a branch-free median-of-three
// insertion network.  The group size K follows; the (K-1)-th smallest value
// theta splits the candidates.  Pass 2 recomputes the (bit-identical)
// scores and collects, in ascending lin order, every candidate below theta
// and the first ties at theta, which is exactly the (score, lin) order's
// first K-1 members; they are then sorted by (score, lin).
// ---------------------------------------------------------------------------



template <int MODE>
struct ScoreT { using type = float; };
template <>
struct ScoreT<kCount> { using type = int; };

// Window-offset index of candidate c of reference r (C-order over the W_d
// offsets, o_d = c_d - r_d + floor(W_d / 2)): the row of the correlated-noise
// bias table.
__device__ inline int window_offset(const Geo& g, int r, int c)
{
    int o = 0, st = 1;
    for (int d = kAx - 1; d >= 0; --d) {
        o += ((c / g.st[d]) % g.L[d] - (r / g.st[d]) % g.L[d] + g.W[d] / 2) * st;
        st *= g.W[d];
    }
    return o;
}

template <int MODE>
__device__ __forceinline__ typename ScoreT<MODE>::type score_of(const MatchArgs& a,
                                                                 const float* src,
                                                                 const int* kap, int r, int c)
{
    const Geo& g = a.g;
    if constexpr (MODE == kCount) {
        int ssd = 0;
        for (int i0 = 0; i0 < g.j[0]; ++i0)
            for (int i1 = 0; i1 < g.j[1]; ++i1)
                for (int i2 = 0; i2 < g.j[2]; ++i2) {
                    const int o = i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2];
                    const int* pr = kap + r + o;
                    const int* pc = kap + c + o;
                    for (int i3 = 0; i3 < g.j[3]; ++i3) {
                        const int d = pc[i3] - pr[i3];
                        ssd += __mul24(d, d);
                    }
                }
        return ssd - a.gamma_i * (a.psum[r + (kap - a.kappa)] + a.psum[c + (kap - a.kappa)]);
    } else {
        float ssd = 0.f, b = 0.f;
        for (int i0 = 0; i0 < g.j[0]; ++i0)
            for (int i1 = 0; i1 < g.j[1]; ++i1)
                for (int i2 = 0; i2 < g.j[2]; ++i2) {
                    const int o = i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2];
                    const float* pr = src + r + o;
                    const float* pc = src + c + o;
                    for (int i3 = 0; i3 < g.j[3]; ++i3) {
                        const float p = pr[i3], q = pc[i3];
                        const float d = q - p;
                        ssd = __builtin_fmaf(d, d, ssd);
                        if constexpr (MODE == kPoissonF) b += fmaxf(p + q, 0.f);
                    }
                }
        if constexpr (MODE == kPoissonF) return __builtin_fmaf(-a.gamma_sp, b, ssd);
        if constexpr (MODE == kGauss)
            return ssd - (a.bias_t ? a.bias_t[window_offset(g, r, c)] : a.bias);
        return ssd;
    }
}

// FP64 score of a float-mode candidate (the re-scored near-ties)
template <int MODE>
__device__ inline double score64_of(const MatchArgs& a, const float* src, int r, int c)
{
    const Geo& g = a.g;
    double ssd = 0.0, b = 0.0;
    for (int i0 = 0; i0 < g.j[0]; ++i0)
        for (int i1 = 0; i1 < g.j[1]; ++i1)
            for (int i2 = 0; i2 < g.j[2]; ++i2) {
                const int o = i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2];
                for (int i3 = 0; i3 < g.j[3]; ++i3) {
                    // separately rounded products and sums (no contraction):
                    // the plain FP64 sum in patch order
                    const double p = src[r + o + i3], q = src[c + o + i3];
                    const double d = __dsub_rn(q, p);
                    ssd = __dadd_rn(ssd, __dmul_rn(d, d));
                    if constexpr (MODE == kPoissonF) b = __dadd_rn(b, fmax(__dadd_rn(p, q), 0.0));
                }
            }
    if constexpr (MODE == kPoissonF) return __dsub_rn(ssd, __dmul_rn(a.gamma_sp_d, b));
    if constexpr (MODE == kGauss)
        return __dsub_rn(ssd, a.bias_td ? a.bias_td[window_offset(g, r, c)] : a.bias_d);
    return ssd;
}

template <typename S>
__device__ __forceinline__ S max_score();
template <>
__device__ __forceinline__ int max_score<int>() { return INT_MAX; }
template <>
__device__ __forceinline__ float max_score<float>() { return FLT_MAX; }


__device__ __forceinline__ int smin(int a, int b) { return min(a, b); }
__device__ __forceinline__ int smax(int a, int b) { return max(a, b); }
__device__ __forceinline__ float smin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ float smax(float a, float b) { return fmaxf(a, b); }

__device__ __forceinline__ int pow2floor(int x)
{
    return x <= 1 ? 1 : (1 << (31 - __clz(x)));
}

template <int MODE, int GM>
__global__ __launch_bounds__(kMatchThreads) void k_match(MatchArgs a)
{
    using S = typename ScoreT<MODE>::type;
    constexpr bool kF = MODE != kCount;  // float scores, FP64 near-tie re-scoring
    using Key = typename std::conditional<kF, double, int>::type;
    constexpr int M = GM > 1 ? GM - 1 : 1;
    __shared__ Key sel_s[M][kMatchThreads];
    __shared__ int sel_l[M][kMatchThreads];

    const Geo& g = a.g;
    const long t = long(blockIdx.x) * kMatchThreads + threadIdx.x;
    if (t >= long(g.batch) * a.n_refs) return;
    const int b = int(t / a.n_refs);
    const int gi = int(t - long(b) * a.n_refs);
    const int r = safe_origin(int(a.refs[gi]), last_origin(g));
    const float* src = a.src + long(b) * g.V;
    const int* kap = MODE == kCount ? a.kappa + long(b) * g.V : nullptr;

    int lo[kAx], hi[kAx];
    int ncand = 1;
    for (int d = 0; d < kAx; ++d) {
        const int rc = (r / g.st[d]) % g.L[d];
        lo[d] = max(rc - g.W[d] / 2, 0);
        hi[d] = min(rc + g.W[d] - 1 - g.W[d] / 2, g.ell[d]);
        ncand *= hi[d] - lo[d] + 1;
    }
    ncand -= 1;  // the reference itself is not a candidate

    // magnitude of the terms beside the score (bias, Poisson correction) for
    // the float-mode tie band: near the K-th value q ~ p, so the correction
    // is at most about twice the reference's
    float bmag = 0.f;
    if constexpr (MODE == kGauss) bmag = a.bias_t ? float(*a.bias_bound) : fabsf(a.bias);
    if constexpr (MODE == kPoissonF) {
        float sp = 0.f;
        for (int i0 = 0; i0 < g.j[0]; ++i0)
            for (int i1 = 0; i1 < g.j[1]; ++i1)
                for (int i2 = 0; i2 < g.j[2]; ++i2)
                    for (int i3 = 0; i3 < g.j[3]; ++i3)
                        sp += fmaxf(src[r + i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2] + i3], 0.f);
        bmag = 4.f * fabsf(a.gamma_sp) * sp;
    }
    auto band = [&](float v) { return float(kTieBand) * (fabsf(v) + bmag); };

    // ---- pass 1: accepted count and the M smallest values (in float modes
    // one more: the value after the K-th tells whether the K-th boundary is
    // a near-tie)
    constexpr int NS = kF ? M + 1 : M;
    S s[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) s[m] = max_score<S>();
    int acc = 0, namb = 0;
    float tau_band = 0.f;
    if constexpr (kF) tau_band = band(a.tau_f);
    for (int c0 = lo[0]; c0 <= hi[0]; ++c0)
        for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
            for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
                for (int c3 = lo[3]; c3 <= hi[3]; ++c3) {
                    const int c = c0 * g.st[0] + c1 * g.st[1] + c2 * g.st[2] + c3;
                    if (c == r) continue;
                    const S x = score_of<MODE>(a, src, kap, r, c);
                    if constexpr (MODE == kCount) {
                        acc += x < a.tau_i;
                    } else {
                        // acc: certain acceptances; namb: the band around
                        // tau, decided in FP64 when it matters
                        const bool amb = fabsf(x - a.tau_f) <= tau_band;
                        acc += x < a.tau_f && !amb;
                        namb += amb;
                    }
#pragma unroll
                    for (int m = NS - 1; m >= 1; --m) s[m] = smin(s[m], smax(s[m - 1], x));
                    s[0] = smin(s[0], x);
                }

    auto group_size = [&](int acc_) {
        int k = pow2floor(min(1 + acc_, a.gmax));
        k = max(k, a.gmin);
        return min(k, pow2floor(1 + ncand));
    };
    int K = group_size(acc);
    if constexpr (kF) {
        // scores within the band of tau are accepted or not in FP64, when
        // that can change the group size
        if (namb > 0 && group_size(acc + namb) != K) {
            acc = 0;
            for (int c0 = lo[0]; c0 <= hi[0]; ++c0)
                for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
                    for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
                        for (int c3 = lo[3]; c3 <= hi[3]; ++c3) {
                            const int c = c0 * g.st[0] + c1 * g.st[1] + c2 * g.st[2] + c3;
                            if (c == r) continue;
                            const float x = score_of<MODE>(a, src, kap, r, c);
                            if (fabsf(x - a.tau_f) <= tau_band)
                                acc += score64_of<MODE>(a, src, r, c) < a.tau_d;
                            else
                                acc += x < a.tau_f;
                        }
            K = group_size(acc);
        }
    }
    const int need = GM > 1 ? K - 1 : 0;

    int* out = a.match + t * a.gmax;
    out[0] = r;
    for (int m = 1; m < a.gmax; ++m) out[m] = -1;
    if (need == 0) {
        a.count[t] = K;
        return;
    }

    S theta = s[0], next = s[0];
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        if (m == need - 1) theta = s[m];
        if (m == need) next = s[m];
    }

    // ---- pass 2: the members below theta and the first ties at theta, in
    // lin order; then sorted by (score, lin)
    int got = 0;
    {
        int n_less = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) n_less += (m < need && s[m] < theta) ? 1 : 0;
        int eq_left = need - n_less;
        for (int c0 = lo[0]; c0 <= hi[0] && got < need; ++c0)
            for (int c1 = lo[1]; c1 <= hi[1] && got < need; ++c1)
                for (int c2 = lo[2]; c2 <= hi[2] && got < need; ++c2)
                    for (int c3 = lo[3]; c3 <= hi[3] && got < need; ++c3) {
                        const int c = c0 * g.st[0] + c1 * g.st[1] + c2 * g.st[2] + c3;
                        if (c == r) continue;
                        const S x = score_of<MODE>(a, src, kap, r, c);
                        bool take = x < theta;
                        if (!take && x == theta && eq_left > 0) {
                            take = true;
                            --eq_left;
                        }
                        if (take) {
                            sel_s[got][threadIdx.x] = Key(x);
                            sel_l[got][threadIdx.x] = c;
                            ++got;
                        }
                    }
        for (int m = 1; m < got; ++m) {
            const Key ks = sel_s[m][threadIdx.x];
            const int kl = sel_l[m][threadIdx.x];
            int p = m - 1;
            while (p >= 0 && sel_s[p][threadIdx.x] > ks) {
                sel_s[p + 1][threadIdx.x] = sel_s[p][threadIdx.x];
                sel_l[p + 1][threadIdx.x] = sel_l[p][threadIdx.x];
                --p;
            }
            sel_s[p + 1][threadIdx.x] = ks;
            sel_l[p + 1][threadIdx.x] = kl;
        }
    }
    if constexpr (kF) {
        // The FP32 ranking equals the FP64 one unless the value after the
        // K-th, or two neighbours in the list, lie within the round-off band
        // (equal zeros are exact).  Otherwise every candidate up to theta
        // plus the band is re-scored in FP64 and the best `need` are kept by
        // (FP64 score, lin); candidates arrive in lin order, so a strict
        // comparison keeps the lower lin first on equal scores.
        auto near = [&](float lo_, float hi_) {
            return hi_ - lo_ <= band(hi_) && !(lo_ == 0.f && hi_ == 0.f);
        };
        bool amb = got == need && near(float(theta), float(next));
        for (int m = 1; m < got; ++m)
            amb = amb || near(float(sel_s[m - 1][threadIdx.x]), float(sel_s[m][threadIdx.x]));
        if (amb) {
            got = 0;
            const float thr = float(theta) + band(float(theta));
            for (int c0 = lo[0]; c0 <= hi[0]; ++c0)
                for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
                    for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
                        for (int c3 = lo[3]; c3 <= hi[3]; ++c3) {
                            const int c = c0 * g.st[0] + c1 * g.st[1] + c2 * g.st[2] + c3;
                            if (c == r) continue;
                            const float x = score_of<MODE>(a, src, kap, r, c);
                            if (!(x <= thr)) continue;
                            const double xd = score64_of<MODE>(a, src, r, c);
                            if (!(xd == xd)) continue;
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
        }
    }
    // non-finite scores select fewer members than asked: the group is cut to
    // the largest power of two they fill, so every listed member is valid
    if (got < need) K = pow2floor(1 + got);
    a.count[t] = K;
    for (int m = 0; m < K - 1; ++m) out[1 + m] = sel_l[m][threadIdx.x];
}

// ---------------------------------------------------------------------------
// Collaborative filtering (sections Hard Thresholding, Wiener Shrinkage,
// Aggregation Weights, Aggregation-Aware Mass Conservation).
// One workgroup filters one group.
// ---------------------------------------------------------------------------



// LDS carve-up shared by host (size) and device (pointers).
struct FilterLds {
    int kp, p, gm;
    size_t off_red, off_A, off_B, off_V, off_T, off_tab, off_H, off_H2, off_win, off_r, off_w,
        off_off, off_org, off_misc, off_key, off_pix, bytes;
    __host__ __device__ FilterLds(const Geo& g, int gmax)
    {
        p = g.P;
        gm = gmax;
        kp = gmax * g.P;
        size_t o = 0;
        off_red = o; o += sizeof(double) * 2 * kFilterThreads;
        off_A = o; o += sizeof(float) * kp;
        off_B = o; o += sizeof(float) * kp;
        off_V = o; o += sizeof(float) * kp;
        off_T = o; o += sizeof(float) * kp;
        off_tab = o;
        for (int d = 0; d < kAx; ++d) o += sizeof(float) * 3 * g.j[d] * g.j[d];
        off_H = o; o += sizeof(float) * gmax * gmax;
        off_H2 = o; o += sizeof(float) * gmax * gmax;
        off_win = o; o += sizeof(float) * g.P;
        off_r = o; o += sizeof(float) * gmax;
        off_w = o; o += sizeof(float) * gmax;
        off_off = o; o += sizeof(int) * g.P;
        off_org = o; o += sizeof(int) * gmax;
        off_misc = o; o += sizeof(int) * 8;
        // correlated noise: member keys and the table rows of member pairs
        off_key = o; o += sizeof(unsigned) * gmax;
        off_pix = o; o += sizeof(int) * size_t(corr_npairs(gmax));
        bytes = (o + 15) & ~size_t(15);
    }
};

// Mode product along `axis` of the K x j0 x j1 x j2 x j3 tensor:
// out[.., a, ..] = sum_t M[a][t] in[.., t, ..].
__device__ void mode_product(const float* in, float* out, const float* Mx, int n, int inner,
                             int total)
{
    for (int e = threadIdx.x; e < total; e += kFilterThreads) {
        const int a = (e / inner) % n;
        const int base = e - a * inner;
        const float* mrow = Mx + a * n;
        float s = 0.f;
        for (int t = 0; t < n; ++t) s = __builtin_fmaf(mrow[t], in[base + t * inner], s);
        out[e] = s;
    }
}

struct GroupShape {
    int n[5];      // K, j0..j3
    int inner[5];  // product of the later extents
    int total;
};

__device__ GroupShape group_shape(const Geo& g, int K)
{
    GroupShape s;
    s.n[0] = K;
    for (int d = 0; d < kAx; ++d) s.n[d + 1] = g.j[d];
    int acc = 1;
    for (int a = 4; a >= 0; --a) {
        s.inner[a] = acc;
        acc *= s.n[a];
    }
    s.total = acc;
    return s;
}

// Apply the separable operator (haar or its variants along the member axis,
// per-axis spatial matrices along the patch axes); returns the buffer that
// holds the result (either x or tmp).
__device__ float* apply_separable(float* x, float* tmp, const GroupShape& s, const float* haar,
                                  const float* const* sp)
{
    float* in = x;
    float* out = tmp;
    for (int a = 0; a < 5; ++a) {
        if (s.n[a] == 1) continue;
        const float* Mx = a == 0 ? haar : sp[a - 1];
        mode_product(in, out, Mx, s.n[a], s.inner[a], s.total);
        __syncthreads();
        float* t = in;
        in = out;
        out = t;
    }
    return in;
}

__device__ double block_sum2(double* red, double v0, double v1, double* r1)
{
    red[threadIdx.x] = v0;
    red[kFilterThreads + threadIdx.x] = v1;
    __syncthreads();
    for (int w = kFilterThreads / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            red[kFilterThreads + threadIdx.x] += red[kFilterThreads + threadIdx.x + w];
        }
        __syncthreads();
    }
    const double a = red[0];
    *r1 = red[kFilterThreads];
    __syncthreads();
    return a;
}

// Decompose a patch sample index i into per-axis indices.
__device__ __forceinline__ void patch_coords(const Geo& g, int i, int* c)
{
    for (int d = kAx - 1; d >= 0; --d) {
        c[d] = i % g.j[d];
        i /= g.j[d];
    }
}

// FP64 recomputation of one transform coefficient and its noise variance
// (hard-threshold decisions within the FP32 error band of lambda sigma).
template <bool EXACT>
__device__ bool rescue_keep(const FilterArgs& a, const float* yb, const float* mvsrc, int K,
                            const int* org, const int* off, int l, int qidx, double* red)
{
    const bool exact = EXACT && l < a.kex;  // exact shared-source plane
    const Geo& g = a.g;
    int q[kAx];
    patch_coords(g, qidx, q);
    const double* H = a.t.f64 + a.t.haar64 + 0;  // 32x32 block for K, see table layout
    // Haar for K is stored at haar64 + K*K offset rows (see device_tables): rows of K.
    int hoff = 0;
    for (int k = 1; k < K; k <<= 1) hoff += k * k;
    H += hoff;
    double sy = 0.0, sv = 0.0, sm = 0.0;
    const int n = K * g.P;
    for (int e = threadIdx.x; e < n; e += kFilterThreads) {
        const int j = e / g.P, i = e - j * g.P;
        int c[kAx];
        patch_coords(g, i, c);
        double w = H[l * K + j];
        for (int d = 0; d < kAx; ++d)
            if (g.j[d] > 1) w *= a.t.f64[a.t.T64[d] + q[d] * g.j[d] + c[d]];
        const int u = org[j] + off[i];
        sy += w * double(yb[u]);
        sm += fabs(w * double(yb[u]));
        double mv;
        if (a.noise == BMND_NOISE_POISSON) mv = a.s_p64 * fmax(double(mvsrc[u]), 0.0);
        else mv = a.sigma2_64;
        if (!exact && !a.cdtab) sv += w * w * mv;
    }
    if (a.cdtab)
        sv = corr_var_part(a, org, K, l, qidx, [&](int r, int j) { return H[r * K + j]; },
                           threadIdx.x, kFilterThreads);
    if constexpr (EXACT) {
        if (exact) sv = exact_partial(a, mvsrc, org, K, l, qidx, threadIdx.x, kFilterThreads);
    }
    double v, unused;
    const double Y = block_sum2(red, sy, sv, &v);
    const double M = block_sum2(red, sm, 0.0, &unused);
    // zero variance: coefficients up to 1e-9 of the magnitude of their terms
    // are rounding residues of exact zeros
    return v > 0.0 ? fabs(Y) > a.lambda64 * sqrt(v) * (1.0 + kTieRel) : fabs(Y) > kTieRel * M;
}

template <bool EXACT>
__global__ __launch_bounds__(kFilterThreads) void k_filter(FilterArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const Geo& g = a.g;
    const FilterLds L(g, a.gmax);
    double* red = reinterpret_cast<double*>(lds + L.off_red);
    float* A = reinterpret_cast<float*>(lds + L.off_A);
    float* B = reinterpret_cast<float*>(lds + L.off_B);
    float* Vb = reinterpret_cast<float*>(lds + L.off_V);
    float* Tb = reinterpret_cast<float*>(lds + L.off_T);
    float* tab = reinterpret_cast<float*>(lds + L.off_tab);
    float* H = reinterpret_cast<float*>(lds + L.off_H);
    float* H2 = reinterpret_cast<float*>(lds + L.off_H2);
    float* win = reinterpret_cast<float*>(lds + L.off_win);
    float* rpl = reinterpret_cast<float*>(lds + L.off_r);
    float* wj = reinterpret_cast<float*>(lds + L.off_w);
    int* off = reinterpret_cast<int*>(lds + L.off_off);
    int* org = reinterpret_cast<int*>(lds + L.off_org);
    int* misc = reinterpret_cast<int*>(lds + L.off_misc);

    const long grp = blockIdx.x;
    const int b = int(grp / a.n_refs);
    const int K = safe_count(a.count[grp], a.gmax);
    const int P = g.P;
    const int n = K * P;
    const float* yb = a.y + long(b) * g.V;
    const float* pb = a.pilot ? a.pilot + long(b) * g.V : nullptr;

    // ---- tables, offsets, window, origins
    const float* spT[kAx];
    const float* spU[kAx];
    const float* spT2[kAx];
    {
        size_t o = 0;
        for (int d = 0; d < kAx; ++d) {
            const int jj = g.j[d] * g.j[d];
            float* dT = tab + o;
            float* dU = tab + o + jj;
            float* dT2 = tab + o + 2 * jj;
            for (int e = threadIdx.x; e < jj; e += kFilterThreads) {
                dT[e] = a.t.f32[a.t.T[d] + e];
                dU[e] = a.t.f32[a.t.U[d] + e];
                dT2[e] = a.t.f32[a.t.T2[d] + e];
            }
            spT[d] = dT;
            spU[d] = dU;
            spT2[d] = dT2;
            o += 3 * jj;
        }
        int hoff = 0;
        for (int k = 1; k < K; k <<= 1) hoff += k * k;
        for (int e = threadIdx.x; e < K * K; e += kFilterThreads) {
            const float h = a.t.f32[a.t.haar + hoff + e];
            H[e] = h;
            H2[e] = h * h;
        }
        for (int i = threadIdx.x; i < P; i += kFilterThreads) {
            int c[kAx];
            patch_coords(g, i, c);
            int o2 = 0;
            float w = 1.f;
            for (int d = 0; d < kAx; ++d) {
                o2 += c[d] * g.st[d];
                w *= a.t.f32[a.t.win[d] + c[d]];
            }
            off[i] = o2;
            win[i] = w;
        }
        for (int j = threadIdx.x; j < K; j += kFilterThreads)
            org[j] = safe_origin(a.match[grp * a.gmax + j], last_origin(g));
        for (int l = threadIdx.x; l < K; l += kFilterThreads) rpl[l] = 0.f;
        if (threadIdx.x == 0) misc[0] = 0;
    }
    __syncthreads();

    const GroupShape gs = group_shape(g, K);
    float* res = A;    // synthesized patches end up here

    if (a.out_mode >= 0 && a.patches_in == nullptr) {
        // ---- gather: y group, pilot group, variance map m_v
        const float* mvsrc = a.stage == BMND_STAGE_WIENER ? pb : yb;
        for (int e = threadIdx.x; e < n; e += kFilterThreads) {
            const int j = e / P, i = e - j * P;
            const int u = org[j] + off[i];
            A[e] = yb[u];
            if (a.stage == BMND_STAGE_WIENER) B[e] = pb[u];
            Vb[e] = a.noise == BMND_NOISE_POISSON ? a.s_p * fmaxf(mvsrc[u], 0.f) : a.sigma2;
        }
        // group norm for the hard-threshold error band
        double gn = 0.0;
        if (a.shrink == BMND_SHRINK_HARD) {
            double part = 0.0;
            for (int e = threadIdx.x; e < n; e += kFilterThreads) part += double(A[e]) * A[e];
            double dummy;
            __syncthreads();
            gn = sqrt(block_sum2(red, part, 0.0, &dummy));
        }
        __syncthreads();

        // ---- forward transforms
        float* Yc = apply_separable(A, Tb, gs, H, spT);
        if (Yc != A) {
            for (int e = threadIdx.x; e < n; e += kFilterThreads) A[e] = Yc[e];
            __syncthreads();
        }
        if (a.cdtab) {
            // correlated noise: sigma^2 from the variance table
            unsigned* keys = reinterpret_cast<unsigned*>(lds + L.off_key);
            int* pix = reinterpret_cast<int*>(lds + L.off_pix);
            for (int j = threadIdx.x; j < K; j += kFilterThreads) keys[j] = corr_member_key(a, org[j]);
            __syncthreads();
            corr_pair_rows(a, keys, K, pix, threadIdx.x, kFilterThreads);
            __syncthreads();
            corr_group_variances<kMaxGroup>(a, pix, K, Vb, threadIdx.x, kFilterThreads);
            __syncthreads();
        } else {
            float* Vc = apply_separable(Vb, Tb, gs, H2, spT2);
            if (Vc != Vb) {
                for (int e = threadIdx.x; e < n; e += kFilterThreads) Vb[e] = Vc[e];
                __syncthreads();
            }
        }
        // exact shared-source variances of the leading planes
        if constexpr (EXACT) {
            const int kex = min(a.kex, K);
            exact_plane_variances(a, mvsrc, org, K, kex, Vb, threadIdx.x, kFilterThreads);
            __syncthreads();
        }
        if (a.stage == BMND_STAGE_WIENER) {
            float* Gc = apply_separable(B, Tb, gs, H, spT);
            if (Gc != B) {
                for (int e = threadIdx.x; e < n; e += kFilterThreads) B[e] = Gc[e];
                __syncthreads();
            }
        }

        // ---- shrinkage; per-plane risk surrogates r_l
        int* rescue = reinterpret_cast<int*>(B);  // B is free in the HT stage
        for (int e = threadIdx.x; e < n; e += kFilterThreads) {
            const int l = e / P;
            const float Y = A[e];
            const float v = fmaxf(Vb[e], 0.f);
            float att, C, shat = 0.f;
            if (a.shrink == BMND_SHRINK_HARD) {
                // strict inequality; exact ties |Y| = lambda sigma (common with
                // integral counts) fall inside the band and are dropped by the
                // FP64 decision, which applies a 1e-9 relative tie margin
                const float thr = a.lambda * sqrtf(v);
                const bool keep = fabsf(Y) > thr;
                // error band of the FP32 decision: transform round-off is
                // bounded by the row norm of T times the group norm
                int q[kAx];
                patch_coords(g, e - l * P, q);
                float rn = 1.f;
                for (int d = 0; d < kAx; ++d) rn *= a.t.f32[a.t.rn[d] + q[d]];
                const float band = 1e-5f * (rn * float(gn) + thr);
                // v == 0 (every source sample of the coefficient has zero
                // variance): the FP64 decision tells rounding residues of
                // exact zeros from kept coefficients
                if (fabsf(fabsf(Y) - thr) <= band) {
                    const int slot = atomicAdd(&misc[0], 1);
                    rescue[slot] = e;
                }
                att = keep ? 1.f : 0.f;
                C = Y;  // masked after the FP64 decisions
            } else if (a.shrink == BMND_SHRINK_SOFT) {
                const float m = fmaxf(fabsf(Y) - a.lambda * sqrtf(v), 0.f);
                C = copysignf(m, Y);
                if (Y == 0.f) C = 0.f;
                att = Y != 0.f ? m / fabsf(Y) : 0.f;
            } else {
                const float gam = B[e];
                shat = fmaxf(gam * gam - a.power_a * v, 0.f);
                const float den = shat + a.s_v * v;
                att = den > 0.f ? shat / den : 0.f;
                C = att * Y;
            }
            A[e] = C;
            Tb[e] = att;  // keep the attenuation for the weights
            Vb[e] = v;
            if (a.shrink == BMND_SHRINK_WIENER) B[e] = shat;
        }
        __syncthreads();
        if (a.shrink == BMND_SHRINK_HARD) {
            const int nres = misc[0];
            for (int k = 0; k < nres; ++k) {
                const int e = rescue[k];
                const int l = e / P;
                const bool keep = rescue_keep<EXACT>(a, yb, yb, K, org, off, l, e - l * P, red);
                if (threadIdx.x == 0) Tb[e] = keep ? 1.f : 0.f;
                __syncthreads();
            }
            for (int e = threadIdx.x; e < n; e += kFilterThreads)
                if (Tb[e] == 0.f) A[e] = 0.f;
        }
        __syncthreads();
        // risk surrogates per plane
        for (int e = threadIdx.x; e < n; e += kFilterThreads) {
            const int l = e / P;
            const float at = Tb[e];
            const float v = Vb[e];
            float r;
            if (a.wmodel == BMND_WEIGHT_CLASSIC) r = at * at;
            else if (a.wmodel == BMND_WEIGHT_VARIANCE) r = at * at * v;
            else r = at * at * v + (1.f - at) * (1.f - at) * B[e];
            if (a.wdomain == BMND_WDOMAIN_WINDOWED) r *= window_metric(a, e - l * P);
            atomicAdd(&rpl[l], r);
        }
        __syncthreads();
        if (a.wscope == BMND_SCOPE_GROUP) {
            float R = 0.f;
            for (int l = 0; l < K; ++l) R += rpl[l];
            const float w = R > 0.f ? 1.f / R : 1.f;
            for (int j = threadIdx.x; j < K; j += kFilterThreads) wj[j] = w;
        } else {
            for (int j = threadIdx.x; j < K; j += kFilterThreads) {
                float R = 0.f;
                for (int l = 0; l < K; ++l) R += H2[l * K + j] * rpl[l];
                wj[j] = R > 0.f ? 1.f / R : 1.f;
            }
        }
        __syncthreads();

        // ---- synthesis p = U C  (U = H^T (x) U_0 (x) ...)
        // transpose H in place into H2 (H2 no longer needed)
        for (int e = threadIdx.x; e < K * K; e += kFilterThreads) {
            const int r0 = e / K, c0 = e - r0 * K;
            H2[e] = H[c0 * K + r0];
        }
        __syncthreads();
        res = apply_separable(A, Tb, gs, H2, spU);
    } else {
        // aggregate-only launch: patches and weights are given
        const float* pin = a.patches_in + grp * long(a.gmax) * P;
        for (int e = threadIdx.x; e < n; e += kFilterThreads) A[e] = pin[e];
        for (int j = threadIdx.x; j < K; j += kFilterThreads) wj[j] = a.weights_in[grp * a.gmax + j];
        __syncthreads();
        res = A;
    }

    // ---- outputs
    if (a.out_mode == 0) {
        float* pout = a.patches + grp * long(a.gmax) * P;
        for (int e = threadIdx.x; e < a.gmax * P; e += kFilterThreads) pout[e] = e < n ? res[e] : 0.f;
        if (threadIdx.x < unsigned(a.gmax))
            a.weights[grp * a.gmax + threadIdx.x] = int(threadIdx.x) < K ? wj[threadIdx.x] : 0.f;
        return;
    }
    const long vb = long(b) * g.V;
    if (a.out_mode == 1) {
        for (int e = threadIdx.x; e < n; e += kFilterThreads) {
            const int j = e / P, i = e - j * P;
            const long u = vb + org[j] + off[i];
            const float ww = wj[j] * win[i];
            // FP64 sums: the float result does not depend on the order
            unsafeAtomicAdd(&a.numd[u], double(ww * res[e]));
            unsafeAtomicAdd(&a.dend[u], double(ww));
        }
    } else if (a.out_mode == 2) {
        for (int e = threadIdx.x; e < n; e += kFilterThreads) {
            const int j = e / P, i = e - j * P;
            const long u = vb + org[j] + off[i];
            unsafeAtomicAdd(&a.dend[u], double(wj[j]) * double(win[i]));
        }
    } else {
        // alpha_g = zeta^T (y_g - p_g) / zeta^T 1,  zeta = w omega / eta
        double zs = 0.0, zr = 0.0;
        for (int e = threadIdx.x; e < n; e += kFilterThreads) {
            const int j = e / P, i = e - j * P;
            const long u = vb + org[j] + off[i];
            const double zeta = double(wj[j]) * double(win[i]) / a.dend[u];
            zs += zeta;
            zr += zeta * (double(a.y[u]) - double(res[e]));
        }
        double zr_tot;
        const double zs_tot = block_sum2(red, zs, zr, &zr_tot);
        const double alpha = zs_tot > 0.0 ? zr_tot / zs_tot : 0.0;
        for (int e = threadIdx.x; e < n; e += kFilterThreads) {
            const int j = e / P, i = e - j * P;
            const long u = vb + org[j] + off[i];
            unsafeAtomicAdd(&a.numd[u], double(wj[j]) * double(win[i]) * (double(res[e]) + alpha));
        }
    }
}

template <typename T>
__global__ void k_normalize(long n, const T* __restrict__ num, const T* __restrict__ den,
                            float* __restrict__ out, float* __restrict__ out2)
{
    for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += long(gridDim.x) * blockDim.x) {
        const T d = den[i];
        const float v = d > T(0) ? float(num[i] / d) : 0.f;
        out[i] = v;
        if (out2) out2[i] = v;
    }
}

__global__ void k_zero(uint4* __restrict__ p, long n16, unsigned char* tail, int ntail)
{
    for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n16;
         i += long(gridDim.x) * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && int(threadIdx.x) < ntail) tail[threadIdx.x] = 0;
}

int grid_for(long n, int threads)
{
    long g = (n + threads - 1) / threads;
    if (g > 65536L * 4) g = 65536L * 4;
    return int(g < 1 ? 1 : g);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const long n16 = long(bytes / 16);
    const int ntail = int(bytes - size_t(n16) * 16);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n16 > 0 ? n16 : 1, 256)), dim3(256), 0, s,
                       static_cast<uint4*>(p), n16,
                       static_cast<unsigned char*>(p) + size_t(n16) * 16, ntail);
    return hipGetLastError();
}

static int* range_flag_ptr()
{
    static int* p = nullptr;
    if (!p) (void)hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(g_range_flag));
    return p;
}

// counts up to which the int32 count-domain score is exact:
// P kmax^2 < 2^31 and gamma 2 P kmax < 2^31
static int count_limit(const StageCfg& c)
{
    double kmax = std::sqrt(2147483647.0 / double(c.g.P));
    const double kg = 2147483647.0 / (2.0 * double(c.g.P) * std::max(1.0, c.gamma));
    if (kg < kmax) kmax = kg;
    return int(kmax) - 1;
}

hipError_t launch_counts(const StageCfg& c, const float* y, int* kappa, int* psum, hipStream_t s)
{
    const long n = long(c.g.batch) * c.g.V;
    hipLaunchKernelGGL(k_counts, dim3(grid_for(n, 256)), dim3(256), 0, s, c.g, y,
                       float(1.0 / c.s_p), count_limit(c), kappa, range_flag_ptr());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_patch_sums, dim3(grid_for(n, 256)), dim3(256), 0, s, c.g, kappa, psum);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_match_mode(const MatchArgs& a, hipStream_t s)
{
    const long n = long(a.g.batch) * a.n_refs;
    const dim3 grid(unsigned((n + kMatchThreads - 1) / kMatchThreads));
    switch (a.gmax) {
    case 1: hipLaunchKernelGGL((k_match<MODE, 1>), grid, dim3(kMatchThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_match<MODE, 2>), grid, dim3(kMatchThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_match<MODE, 4>), grid, dim3(kMatchThreads), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_match<MODE, 8>), grid, dim3(kMatchThreads), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_match<MODE, 16>), grid, dim3(kMatchThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((k_match<MODE, 32>), grid, dim3(kMatchThreads), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_match(const StageCfg& c, const float* src, int* kappa, int* psum,
                        const int64_t* refs, int n_refs, int* match, int* count, hipStream_t s,
                        const MomentTables* mom, const NdBlocks* blk)
{
    if (c.metric != BMND_METRIC_SSD) {
        // Poisson-likelihood metrics (HT stage, Poisson noise)
        if (!mom) return hipErrorInvalidValue;
        MatchArgs a{};
        a.g = c.g;
        a.src = src;
        a.refs = refs;
        a.n_refs = n_refs;
        a.match = match;
        a.count = count;
        a.gmin = c.gmin;
        a.gmax = c.gmax;
        a.inv_sp = float(1.0 / c.s_p);
        a.range_flag = range_flag_ptr();
        a.policy = c.policy;
        a.integral = c.counts_integral ? 1 : 0;
        a.s_p_d = c.s_p;
        a.t_d = c.match_t;
        a.sbeta_d = c.sbeta;
        a.skappa_d = c.skappa;
        a.mu_f = mom->mu;
        a.v_f = mom->v;
        a.mu_d = mom->mu64;
        a.v_d = mom->v64;
        a.nmom = mom->nmax;
        // fixed: the high-count calibration 1 + t sqrt(2 / P); standardized: t;
        // reference: per reference in the kernel
        a.tau_d = c.policy == BMND_POLICY_FIXED ? 1.0 + c.match_t * std::sqrt(2.0 / c.g.P)
                                                 : c.match_t;
        a.tau_f = float(a.tau_d);
        return launch_match_pois(a, c.metric, 1 << 23, s);
    }
    MatchArgs a{};
    a.g = c.g;
    a.src = src;
    a.kappa = kappa;
    a.psum = psum;
    a.refs = refs;
    a.n_refs = n_refs;
    a.match = match;
    a.count = count;
    a.gmin = c.gmin;
    a.gmax = c.gmax;
    a.inv_sp = float(1.0 / c.s_p);
    a.range_flag = range_flag_ptr();
    int mode;
    if (c.stage == BMND_STAGE_WIENER) {
        mode = kPlain;
        a.tau_f = float(c.tau);
        a.tau_d = c.tau;
    } else if (c.integral) {
        mode = kCount;
        a.gamma_i = int(c.gamma);
        // accept iff score < tau / s_P^2 (integer score): score < ceil(.)
        const double t = c.tau / (c.s_p * c.s_p);
        double ct = std::ceil(t);
        if (ct > 2147483647.0) ct = 2147483647.0;
        if (ct < -2147483647.0) ct = -2147483647.0;
        a.tau_i = int(ct);
    } else if (c.noise == BMND_NOISE_POISSON) {
        mode = kPoissonF;
        a.gamma_sp = float(c.gamma * c.s_p);
        a.gamma_sp_d = c.gamma * c.s_p;
        a.tau_f = float(c.tau);
        a.tau_d = c.tau;
    } else {
        mode = kGauss;
        if (c.noise == BMND_NOISE_CORRELATED) {
            // the bias depends on the candidate's window offset
            a.bias_t = c.corr.bias32;
            a.bias_td = c.corr.bias;
            a.bias_bound = c.corr.bias_bound;
        } else {
            a.bias_d = c.gamma * 2.0 * c.g.P * c.sigma * c.sigma;
            a.bias = float(a.bias_d);
        }
        a.tau_f = float(c.tau);
        a.tau_d = c.tau;
    }
    if (!a.bias_t && match_1d_supported(c.g, mode))
        return launch_match_1d(a, mode, c.step_last, count_limit(c), s);
    if (match_nd_supported(c.g)) return launch_match_nd(a, mode, count_limit(c), blk, s);
    if (mode == kCount) {
        if (!kappa || !psum) return hipErrorInvalidValue;
        hipError_t e = launch_counts(c, src, kappa, psum, s);
        if (e != hipSuccess) return e;
    }
    switch (mode) {
    case kPlain: return launch_match_mode<kPlain>(a, s);
    case kCount: return launch_match_mode<kCount>(a, s);
    case kPoissonF: return launch_match_mode<kPoissonF>(a, s);
    default: return launch_match_mode<kGauss>(a, s);
    }
}

static FilterArgs filter_args(const StageCfg& c, const DevTables& t, int out_mode)
{
    FilterArgs a{};
    a.g = c.g;
    a.stage = c.stage;
    a.shrink = c.shrink;
    a.spatial = c.spatial;
    a.noise = c.noise;
    a.s_p = float(c.s_p);
    a.sigma2 = float(c.sigma * c.sigma);
    a.lambda = float(c.lambda);
    a.s_v = float(c.s_v);
    a.power_a = float(c.power_a);
    a.s_p64 = c.s_p;
    a.sigma2_64 = c.sigma * c.sigma;
    a.lambda64 = c.lambda;
    a.wmodel = c.wmodel;
    a.wscope = c.wscope;
    a.wdomain = c.wdomain;
    a.kex = c.k_exact;
    a.gmax = c.gmax;
    a.out_mode = out_mode;
    a.t = t;
    if (c.noise == BMND_NOISE_CORRELATED) {
        a.cdtab = c.corr.dtab;
        for (int d = 0; d < kAx; ++d) a.cbw[d] = c.corr.bw[d];
        a.kex = 0;
    }
    return a;
}

size_t filter_lds_bytes(const Geo& g, int gmax) { return FilterLds(g, gmax).bytes; }

static hipError_t launch_generic_filter(const FilterArgs& a, size_t lds, long groups, hipStream_t s)
{
    const void* fn = a.kex > 0 ? reinterpret_cast<const void*>(&k_filter<true>)
                               : reinterpret_cast<const void*>(&k_filter<false>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    if (a.kex > 0)
        hipLaunchKernelGGL(k_filter<true>, dim3(unsigned(groups)), dim3(kFilterThreads), lds, s, a);
    else
        hipLaunchKernelGGL(k_filter<false>, dim3(unsigned(groups)), dim3(kFilterThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_filter(const StageCfg& c, const DevTables& t, int out_mode, const float* y,
                         const float* pilot, int n_refs, const int* match, const int* count,
                         float* patches, float* weights, void* num, void* den, hipStream_t s)
{
    FilterArgs a = filter_args(c, t, out_mode);
    a.n_refs = n_refs;
    a.y = y;
    a.pilot = pilot;
    a.match = match;
    a.count = count;
    a.patches = patches;
    a.weights = weights;
    a.numd = static_cast<double*>(num);
    a.dend = static_cast<double*>(den);
    const long groups = long(c.g.batch) * n_refs;
    if (!a.cdtab && filter_1d_supported(c.g, c.gmax, false, c.k_exact))
        return launch_filter_1d(a, c.step_last, s);
    // per-sample denominators are needed here (out modes 1-3 of this entry
    // point); the N-D filter serves the patch output
    if (out_mode == 0 &&
        nd_filter_supported(c.g, c.gmax, a.kex, a.cdtab != nullptr, c.noise, c.shrink))
        return launch_filter_nd(a, nullptr, s);
    if (cube_filter_supported(c.g, c.gmax)) return launch_filter_cube(a, c.step_last, s);
    return launch_generic_filter(a, FilterLds(c.g, c.gmax).bytes, groups, s);
}

hipError_t launch_filter_blocked(const StageCfg& c, const DevTables& t, int out_mode,
                                 const float* y, const float* pilot, int n_refs, const int* match,
                                 const int* count, void* num, void* den, double* wfield,
                                 const NdBlocks* blk, void* sweep_state, hipStream_t s)
{
    FilterArgs a = filter_args(c, t, out_mode);
    if (c.stage == BMND_STAGE_HT && c.shrink == BMND_SHRINK_HARD &&
        (out_mode == 2 || out_mode == 3)) {
        // the decisions and weights passed from sweep 1 to sweep 2
        if (!sweep_state) return hipErrorInvalidValue;
        const size_t members = size_t(c.g.batch) * size_t(n_refs) * size_t(c.gmax);
        a.hmask = static_cast<unsigned*>(sweep_state);
        a.hwt = reinterpret_cast<float*>(static_cast<char*>(sweep_state) + members * 16);
    }
    a.n_refs = n_refs;
    a.y = y;
    a.pilot = pilot;
    a.match = match;
    a.count = count;
    a.numd = static_cast<double*>(num);
    a.dend = static_cast<double*>(den);
    a.wfield = wfield;
    return launch_filter_nd(a, blk, s);
}

hipError_t launch_aggregate(const StageCfg& c, const DevTables& t, int out_mode, const float* y,
                            int n_refs, const int* match, const int* count, const float* patches,
                            const float* weights, void* num, void* den, hipStream_t s)
{
    FilterArgs a = filter_args(c, t, out_mode);
    a.n_refs = n_refs;
    a.y = y;
    a.match = match;
    a.count = count;
    a.patches_in = patches;
    a.weights_in = weights;
    a.numd = static_cast<double*>(num);
    a.dend = static_cast<double*>(den);
    const long groups = long(c.g.batch) * n_refs;
    if (cube_filter_supported(c.g, c.gmax)) return launch_filter_cube(a, c.step_last, s);
    return launch_generic_filter(a, FilterLds(c.g, c.gmax).bytes, groups, s);
}

hipError_t launch_normalize(const StageCfg& c, const void* num, const void* den, float* out,
                            float* out2, hipStream_t s)
{
    // numerator and denominator are FP64 sums in every mode
    (void)c.mc;
    const long n = long(c.g.batch) * c.g.V;
    hipLaunchKernelGGL(k_normalize<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                       static_cast<const double*>(num), static_cast<const double*>(den), out,
                       out2);
    return hipGetLastError();
}

hipError_t read_and_clear_range_flag(int* flag)
{
    hipError_t e = hipMemcpyFromSymbol(flag, HIP_SYMBOL(g_range_flag), sizeof(int));
    if (e != hipSuccess) return e;
    const int zero = 0;
    return hipMemcpyToSymbol(HIP_SYMBOL(g_range_flag), &zero, sizeof(int));
}

}  // namespace bmnd
