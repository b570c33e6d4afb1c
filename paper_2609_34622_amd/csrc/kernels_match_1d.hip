// Block matching for 1-D arrays with 32-sample patches (section Block
// Matching): one wavefront scores the windows of 64 consecutive
// references.  The samples covering their windows are staged once in LDS
// (raw counts for exact count-domain HT scores, the pilot for the Wiener
// stage); each lane keeps its reference patch in registers and walks the
// window offsets 32 at a time over a 64-sample register block, so every
// squared difference is computed from registers.  The Poisson bias uses a
// sliding patch sum of the candidate.
//
// Selection is the two-pass scheme of the generic kernel: pass 1 counts the
// accepted candidates and keeps the M smallest score values (median-of-three
// insertion network); every candidate whose score does not exceed the
// running M-th value is recorded (offset index, in lin order).  The group's
// members are exactly the recorded candidates below the (K-1)-th value and
// the first ties at it, so pass 2 rescans only the record.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <type_traits>

#include "bmnd_internal.h"
#include "match_common.h"

namespace bmnd {

namespace {

constexpr int kWave = 64;
constexpr int kJ = 32;      // patch length
constexpr int kRec = 96;    // recorded offsets per lane before falling back

template <int MODE>
struct Sc { using T = float; };
template <>
struct Sc<kCount> { using T = int; };

__device__ __forceinline__ int smin(int a, int b) { return min(a, b); }
__device__ __forceinline__ int smax(int a, int b) { return max(a, b); }
__device__ __forceinline__ float smin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ float smax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ int as_bits(int v) { return v; }
__device__ __forceinline__ int as_bits(float v) { return __float_as_int(v); }
template <typename S> __device__ __forceinline__ S from_bits(int v);
template <> __device__ __forceinline__ int from_bits<int>(int v) { return v; }
template <> __device__ __forceinline__ float from_bits<float>(int v) { return __int_as_float(v); }
template <typename S> __device__ __forceinline__ S big();
template <> __device__ __forceinline__ int big<int>() { return INT_MAX; }
template <> __device__ __forceinline__ float big<float>() { return FLT_MAX; }

// median of three (one VALU instruction)
__device__ __forceinline__ float med3(float a, float b, float c) { return __builtin_amdgcn_fmed3f(a, b, c); }
__device__ __forceinline__ int med3(int a, int b, int c)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ int p2floor(int x) { return x <= 1 ? 1 : (1 << (31 - __clz(x))); }

// squared distance of the reference patch rp and the candidate starting
// at c (LDS), always in the same order (pass 1 and pass 2 agree bitwise)
template <int MODE>
__device__ __forceinline__ typename Sc<MODE>::T ssd_lds(const typename Sc<MODE>::T* rp,
                                                        const int* sx, int c)
{
    using S = typename Sc<MODE>::T;
    S s = 0;
#pragma unroll
    for (int i = 0; i < kJ; ++i) {
        const S q = from_bits<S>(sx[c + i]);
        const S d = q - rp[i];
        if constexpr (MODE == kCount) s += __mul24(d, d);
        else s = __builtin_fmaf(d, d, s);
    }
    return s;
}

// FP64 score of a float-mode candidate (re-scored near-ties), summed in the
// same order
template <int MODE>
__device__ __forceinline__ double score64_lds(const MatchArgs& a, const float* rp, const int* sx,
                                              int c)
{
    // separately rounded products and sums (no contraction), so the value
    // is the plain FP64 sum in patch order
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kJ; ++i) {
        const double d = __dsub_rn(double(__int_as_float(sx[c + i])), double(rp[i]));
        s = __dadd_rn(s, __dmul_rn(d, d));
    }
    if constexpr (MODE == kGauss) s = __dsub_rn(s, a.bias_d);
    return s;
}

template <int MODE, int GM>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3)))
void k_match_1d(MatchArgs a, int cap_span, int kmax)
{
    using S = typename Sc<MODE>::T;
    constexpr bool kF = MODE != kCount;  // float scores, FP64 near-tie re-scoring
    using Key = typename std::conditional<kF, double, int>::type;
    constexpr int M = GM > 1 ? GM - 1 : 1;
    extern __shared__ __align__(16) int sx[];   // staged samples
    __shared__ Key sel_s[M][kWave];
    __shared__ int sel_l[M][kWave];
    __shared__ unsigned char rec[kRec][kWave];

    const Geo& g = a.g;
    const int L = g.L[kAx - 1];
    const int W = g.W[kAx - 1];
    const int ell = L - kJ;
    const int wlo = -(W / 2), whi = W - 1 - W / 2;
    const int nchunk = (a.n_refs + kWave - 1) / kWave;
    const int b = blockIdx.x / nchunk;
    const int chunk = blockIdx.x - b * nchunk;
    const int lane = threadIdx.x;
    const int gi = chunk * kWave + lane;
    const bool have = gi < a.n_refs;
    const int r = have ? safe_origin(int(a.refs[gi]), last_origin(g)) : 0;
    const float* src = a.src + long(b) * g.V;
    const long t = long(b) * a.n_refs + gi;
    const float inv_sp = a.inv_sp;

    bool pending = have;
    while (__any(pending)) {
        // ---- stage the window of the first pending reference onward
        const int r0 = __shfl(r, __ffsll(__ballot(pending)) - 1);
        // references below r0 (unsorted lists) wait for a later round
        const bool mine = pending && r >= r0 && (r - r0) <= cap_span;
        const int base = r0 + wlo;
        const int len = cap_span + W + 2 * kJ;  // covers the last 64-sample block
        for (int i = lane; i < len; i += kWave) {
            const int pos = base + i;
            int v = 0;
            if (pos >= 0 && pos < L) {
                const float x = src[pos];
                if constexpr (MODE == kCount) {
                    // non-finite or out-of-range counts are flagged (and
                    // scored as 0)
                    const float rk = rintf(x * inv_sp);
                    const bool ok = rk >= 0.f && rk <= float(kmax);
                    if (!ok) atomicOr(a.range_flag, 1);
                    v = ok ? int(rk) : 0;
                } else {
                    v = __float_as_int(x);
                }
            }
            sx[i] = v;
        }
        __syncthreads();

        if (mine) {
            const int rl = r - base;  // reference start in the stage
            S rp[kJ];
            S sr = 0;
#pragma unroll
            for (int i = 0; i < kJ; ++i) {
                rp[i] = from_bits<S>(sx[rl + i]);
                sr += rp[i];
            }
            const int dlo = max(wlo, -r), dhi = min(whi, ell - r);
            const int ncand = dhi - dlo;  // window size minus the reference
            // the M smallest values, and in float modes one more (the value
            // after the K-th tells whether the K-th boundary is a near-tie)
            constexpr int NS = kF ? M + 1 : M;
            S s[NS];
#pragma unroll
            for (int m = 0; m < NS; ++m) s[m] = big<S>();
            int acc = 0, nrec = 0, namb = 0;
            // float modes: band of FP32 round-off around a value (relative
            // to the score's terms; the Gaussian bias is one of them)
            const float bmag = MODE == kGauss ? fabsf(a.bias) : 0.f;
            const float tau_band = float(kTieBand) * (fabsf(a.tau_f) + bmag);
            // count mode: the SSD of integer counts is evaluated exactly as
            // sum p^2 + sum q^2 - 2 sum pq (wrapping uint32 arithmetic; the
            // result is below 2^31), with sliding sums over the candidate
            unsigned sp2 = 0;
            if constexpr (MODE == kCount) {
#pragma unroll
                for (int i = 0; i < kJ; ++i) sp2 += unsigned(__mul24(rp[i], rp[i]));
            }
            for (int d0 = wlo; d0 <= whi; d0 += kJ) {
                S buf[2 * kJ];
#pragma unroll
                for (int i = 0; i < 2 * kJ; ++i) buf[i] = from_bits<S>(sx[rl + d0 + i]);
                S sc = 0;
                unsigned sq2 = 0;
                if constexpr (MODE == kCount) {
#pragma unroll
                    for (int i = 0; i < kJ; ++i) {
                        sc += buf[i];
                        sq2 += unsigned(__mul24(buf[i], buf[i]));
                    }
                }
#pragma unroll
                for (int u = 0; u < kJ; ++u) {
                    const int d = d0 + u;
                    S x = 0;
                    if constexpr (MODE == kCount) {
                        unsigned spq = 0;
#pragma unroll
                        for (int i = 0; i < kJ; ++i) spq += unsigned(__mul24(buf[u + i], rp[i]));
                        x = int(sp2 + sq2 - 2u * spq) - a.gamma_i * (sr + sc);
                        sq2 += unsigned(__mul24(buf[u + kJ], buf[u + kJ]) - __mul24(buf[u], buf[u]));
                        sc += buf[u + kJ] - buf[u];
                    } else {
#pragma unroll
                        for (int i = 0; i < kJ; ++i) {
                            const S df = buf[u + i] - rp[i];
                            x = __builtin_fmaf(df, df, x);
                        }
                        if constexpr (MODE == kGauss) x -= a.bias;
                        x = x == x ? x : big<S>();  // non-finite scores are never selected
                    }
                    // offsets outside the clipped window and the reference
                    // itself score as the largest value (never counted, never
                    // selected)
                    const bool valid = d >= dlo && d <= dhi && d != 0;
                    x = valid ? x : big<S>();
                    if constexpr (MODE == kCount) {
                        acc += x < a.tau_i;
                    } else {
                        acc += x < a.tau_f;
                        namb += fabsf(x - a.tau_f) <= tau_band;
                    }
                    bool rec_it;
                    if constexpr (MODE == kCount) rec_it = valid && x <= s[M - 1];
                    else rec_it = valid && x <= s[M - 1] + float(kTieBand) * (fabsf(s[M - 1]) + bmag);
                    if (rec_it) {
                        if (nrec < kRec) rec[nrec][lane] = (unsigned char)(d - wlo);
                        ++nrec;
                    }
                    // insertion into the sorted M smallest: slot m takes the
                    // median of (s[m-1], x, s[m]) since s[m-1] <= s[m]
#pragma unroll
                    for (int m = NS - 1; m >= 1; --m) s[m] = med3(s[m - 1], x, s[m]);
                    s[0] = smin(s[0], x);
                }
            }

            auto group_size = [&](int acc_) {
                int k = p2floor(min(1 + acc_, a.gmax));
                k = max(k, a.gmin);
                return min(k, p2floor(1 + ncand));
            };
            int K = group_size(acc);
            if constexpr (kF) {
                // scores within the band of tau are accepted or not in FP64,
                // when that can change the group size
                if (namb > 0 && group_size(acc + namb) != K) {
                    acc = 0;
                    for (int d = dlo; d <= dhi; ++d) {
                        if (d == 0) continue;
                        S x = ssd_lds<MODE>(rp, sx, rl + d);
                        if constexpr (MODE == kGauss) x -= a.bias;
                        if (fabsf(x - a.tau_f) <= tau_band)
                            acc += score64_lds<MODE>(a, rp, sx, rl + d) < a.tau_d;
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
            if (need == 0) a.count[t] = K;
            if (need > 0) {
                S theta = s[0], next = s[0];
#pragma unroll
                for (int m = 0; m < NS; ++m) {
                    if (m == need - 1) theta = s[m];
                    if (m == need) next = s[m];
                }
                int got = 0;
                // FP32 (exact in count mode) selection: the members below
                // theta and the first ties at theta, in lin order; then sorted
                // by (score, lin)
                {
                    int n_less = 0;
#pragma unroll
                    for (int m = 0; m < M; ++m) n_less += (m < need && s[m] < theta) ? 1 : 0;
                    int eq_left = need - n_less;
                    auto consider = [&](int d) {
                        S x = ssd_lds<MODE>(rp, sx, rl + d);
                        if constexpr (MODE == kCount) {
                            int sc2 = 0;
                            for (int i = 0; i < kJ; ++i) sc2 += sx[rl + d + i];
                            x -= a.gamma_i * (sr + sc2);
                        } else {
                            if constexpr (MODE == kGauss) x -= a.bias;
                            x = x == x ? x : big<S>();
                        }
                        bool take = x < theta;
                        if (!take && x == theta && eq_left > 0) {
                            take = true;
                            --eq_left;
                        }
                        if (take) {
                            sel_s[got][lane] = Key(x);
                            sel_l[got][lane] = r + d;
                            ++got;
                        }
                    };
                    if (nrec <= kRec) {
                        for (int k = 0; k < nrec && got < need; ++k) consider(int(rec[k][lane]) + wlo);
                    } else {
                        for (int d = dlo; d <= dhi && got < need; ++d)
                            if (d != 0) consider(d);
                    }
                    for (int m = 1; m < got; ++m) {
                        const Key ks = sel_s[m][lane];
                        const int kl = sel_l[m][lane];
                        int p = m - 1;
                        while (p >= 0 && sel_s[p][lane] > ks) {
                            sel_s[p + 1][lane] = sel_s[p][lane];
                            sel_l[p + 1][lane] = sel_l[p][lane];
                            --p;
                        }
                        sel_s[p + 1][lane] = ks;
                        sel_l[p + 1][lane] = kl;
                    }
                }
                if constexpr (kF) {
                    // The FP32 ranking equals the FP64 one unless the value
                    // after the K-th, or two neighbours in the list, lie
                    // within the round-off band (equal zeros are exact).
                    auto near = [&](float lo, float hi) {
                        return hi - lo <= float(kTieBand) * (fabsf(hi) + bmag) &&
                               !(lo == 0.f && hi == 0.f);
                    };
                    bool amb = got == need && near(float(theta), float(next));
                    for (int m = 1; m < got; ++m)
                        amb = amb || near(float(sel_s[m - 1][lane]), float(sel_s[m][lane]));
                    if (amb) {
                        // every candidate up to theta plus the band is
                        // re-scored in FP64; the best `need` are kept by (FP64
                        // score, lin) (candidates arrive in lin order, a strict
                        // comparison keeps the lower lin first on equal scores)
                        got = 0;
                        const float thr = theta + float(kTieBand) * (fabsf(theta) + bmag);
                        auto consider = [&](int d) {
                            S x = ssd_lds<MODE>(rp, sx, rl + d);
                            if constexpr (MODE == kGauss) x -= a.bias;
                            if (!(x <= thr)) return;
                            const double xd = score64_lds<MODE>(a, rp, sx, rl + d);
                            if (!(xd == xd)) return;
                            if (got == need && !(xd < sel_s[need - 1][lane])) return;
                            int p = got < need ? got : need - 1;
                            while (p > 0 && sel_s[p - 1][lane] > xd) {
                                sel_s[p][lane] = sel_s[p - 1][lane];
                                sel_l[p][lane] = sel_l[p - 1][lane];
                                --p;
                            }
                            sel_s[p][lane] = xd;
                            sel_l[p][lane] = r + d;
                            if (got < need) ++got;
                        };
                        if (nrec <= kRec) {
                            for (int k = 0; k < nrec; ++k) consider(int(rec[k][lane]) + wlo);
                        } else {
                            for (int d = dlo; d <= dhi; ++d)
                                if (d != 0) consider(d);
                        }
                    }
                }
                // non-finite scores select fewer members than asked: the
                // group is cut to the largest power of two they fill
                if (got < need) K = p2floor(1 + got);
                a.count[t] = K;
                for (int m = 0; m < K - 1; ++m) out[1 + m] = sel_l[m][lane];
            }
        }
        pending = pending && !mine;
        __syncthreads();
    }
}

template <int MODE>
hipError_t launch_1d_mode(const MatchArgs& a, int cap_span, int kmax, hipStream_t s)
{
    const int nchunk = (a.n_refs + kWave - 1) / kWave;
    const dim3 grid(unsigned(long(nchunk) * a.g.batch));
    const size_t lds = sizeof(int) * size_t(cap_span + a.g.W[kAx - 1] + 2 * kJ);
    switch (a.gmax) {
    case 1: hipLaunchKernelGGL((k_match_1d<MODE, 1>), grid, dim3(kWave), lds, s, a, cap_span, kmax); break;
    case 2: hipLaunchKernelGGL((k_match_1d<MODE, 2>), grid, dim3(kWave), lds, s, a, cap_span, kmax); break;
    case 4: hipLaunchKernelGGL((k_match_1d<MODE, 4>), grid, dim3(kWave), lds, s, a, cap_span, kmax); break;
    case 8: hipLaunchKernelGGL((k_match_1d<MODE, 8>), grid, dim3(kWave), lds, s, a, cap_span, kmax); break;
    case 16: hipLaunchKernelGGL((k_match_1d<MODE, 16>), grid, dim3(kWave), lds, s, a, cap_span, kmax); break;
    default: hipLaunchKernelGGL((k_match_1d<MODE, 32>), grid, dim3(kWave), lds, s, a, cap_span, kmax); break;
    }
    return hipGetLastError();
}

}  // namespace

bool match_1d_supported(const Geo& g, int mode)
{
    for (int d = 0; d < kAx - 1; ++d)
        if (g.L[d] != 1) return false;
    return g.j[kAx - 1] == kJ && g.W[kAx - 1] <= 256 && g.W[kAx - 1] >= 1 &&
           (mode == kCount || mode == kPlain || mode == kGauss);
}

hipError_t launch_match_1d(const MatchArgs& a, int mode, int step, int kmax, hipStream_t s)
{
    const int cap_span = kWave * max(step, 1);
    if (mode == kCount) return launch_1d_mode<kCount>(a, cap_span, kmax, s);
    if (mode == kGauss) return launch_1d_mode<kGauss>(a, cap_span, kmax, s);
    return launch_1d_mode<kPlain>(a, cap_span, kmax, s);
}

}  // namespace bmnd
