// Block matching for N-D arrays (section Block Matching): one wavefront
// scores every candidate of one reference.
//
// The clipped search region of the reference (window origins plus a patch)
// is staged once in LDS: raw counts for exact count-domain HT scores, the
// observation or the pilot otherwise.  The reference patch sits in
// registers, one row (run along the last axis) per register array.  Lanes
// take runs of RB consecutive candidates along the last axis: for every
// patch row a segment of J + RB - 1 staged samples is read once and gives
// the row terms of all RB candidates.  Every candidate's score is kept in
// LDS, in C order over the window.
//
// Selection (Def. matched group): the count of accepted scores gives K; the
// K-1 smallest (score, lin) follow from the (K-1)-th smallest value of
// order-preserving 32-bit keys (a histogram of 256 equal bins over the
// keys' range, then the keys of the rank's bin ranked exactly), and the
// first ties at it in lin order (prefix counts across lanes); the members
// are ranked by (score, lin).  Float scores within the round-off band of the K-th
// value (or of tau, when that changes K) are re-scored in FP64, which then
// decides membership and order.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <algorithm>
#include <type_traits>

#include "bmnd_internal.h"
#include "match_common.h"
#include "filter_nd.h"

namespace bmnd {

namespace {

constexpr int kWave = 64;
constexpr int kRB = 8;          // candidates per run along the last axis (one reference per workgroup)
constexpr int kPad = 32;        // samples staged past a region or box (runs read beyond a row)
constexpr int kMaxRegion = 4096;
constexpr int kMaxCand = 4096;
constexpr int kBandCap = 128;   // FP64 re-scored candidates per chunk

template <int MODE>
struct ScT { using T = float; };
template <>
struct ScT<kCount> { using T = int; };

__device__ __forceinline__ unsigned okey(int v) { return unsigned(v) ^ 0x80000000u; }
__device__ __forceinline__ unsigned okey(float v)
{
    const unsigned b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
// inverse of okey for float scores
__device__ __forceinline__ float key_float(unsigned k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// the score of a key (inverse of okey)
template <typename S> __device__ __forceinline__ S key_value(unsigned k);
template <> __device__ __forceinline__ int key_value<int>(unsigned k) { return int(k ^ 0x80000000u); }
template <> __device__ __forceinline__ float key_value<float>(unsigned k) { return key_float(k); }

template <typename S> __device__ __forceinline__ S bigv();
template <> __device__ __forceinline__ int bigv<int>() { return INT_MAX; }
template <> __device__ __forceinline__ float bigv<float>() { return FLT_MAX; }
__device__ __forceinline__ int as_int(int v) { return v; }
__device__ __forceinline__ int as_int(float v) { return __float_as_int(v); }
template <typename S> __device__ __forceinline__ S from_int(int v);
template <> __device__ __forceinline__ int from_int<int>(int v) { return v; }
template <> __device__ __forceinline__ float from_int<float>(int v) { return __int_as_float(v); }

__device__ __forceinline__ int p2fl(int x) { return x <= 1 ? 1 : (1 << (31 - __clz(x))); }

__device__ __forceinline__ int wsum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ unsigned wmin_u(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, unsigned(__shfl_xor(int(v), o)));
    return v;
}

__device__ __forceinline__ unsigned wmax_u(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, unsigned(__shfl_xor(int(v), o)));
    return v;
}

// Offsets of the patch rows (runs along the last axis) of a patch in a
// staged region of strides sst, rows in C order over the other axes.
template <int MR>
__device__ __forceinline__ void row_offsets(const Geo& g, const int* sst, int (&roff)[MR])
{
    const int rows = g.P / g.j[kAx - 1];
#pragma unroll
    for (int q = 0; q < MR; ++q) {
        int rem = q < rows ? q : 0, o = 0;
#pragma unroll
        for (int d = kAx - 2; d >= 0; --d) {
            const int i = rem % g.j[d];
            rem /= g.j[d];
            o += i * sst[d];
        }
        roff[q] = o;
    }
}

// exclusive prefix sum over the lanes of the wave
__device__ __forceinline__ int wscan_ex(int v)
{
    const int lane = threadIdx.x & (kWave - 1);
    int s = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(s, o);
        if (lane >= o) s += t;
    }
    return s - v;
}

// Orders the LDS accesses of one wavefront.
__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Per-wavefront shared scratch of the selection.
template <int GM>
struct WaveSel {
    static constexpr int M = GM > 1 ? GM - 1 : 1;
    // 16-byte aligned in every element of an array of these: the bin scan
    // reads it four bins at a time
    alignas(16) unsigned hist[256];
    // candidates are named by window index (C order over the clipped
    // window, which is their lin order; lin is formed only for the output)
    int sel_ci[M];    // members in window order
    int sel_key[M];
    int srt_ci[M];    // ranked by (key, window index)
    int srt_key[M];
    double band_x[kBandCap];
    int band_l[kBandCap];   // window indices
    double best_x[M];
    int best_l[M];          // window indices
    int misc[4];
};

// Matching of reference gi of array b by one wavefront.  The samples of its
// clipped search region (window origins plus a patch) are in sx (raw counts
// or float bit patterns), sample (c_0, ..., c_3) of the array at
// sum_d (c_d - sorg[d]) sst[d]; xs holds ncand ints of scratch.
// sb (count mode, nullable): four byte copies of the staged counts, copy c
// (at sb + c cst) holding staged sample k + c at byte k, so the 4 samples
// from any sample index b form the aligned word b / 4 of copy b % 4; scores
// then come from v_dot4_u32_u8 products (exact, counts up to 255).
template <int MODE, int GM, int J3, int RB>
__device__ __forceinline__ void match_one(const MatchArgs& a, int b, int gi, const int* sx,
                                          const int* sorg, const int* sst,
                                          const int (&roff)[64 / J3], int* xs,
                                          WaveSel<GM>& ws, const unsigned char* sb, int cst)
{
    using S = typename ScT<MODE>::T;
    constexpr bool kF = MODE != kCount;
    constexpr int MR = 64 / J3;              // most patch rows (P <= 64)
    constexpr int kRB = RB;                  // candidates per run along the last axis
    constexpr int SEG = J3 + kRB - 1;
    constexpr int M = WaveSel<GM>::M;
    unsigned* hist = ws.hist;
    int* sel_ci = ws.sel_ci;
    int* sel_key = ws.sel_key;
    int* srt_ci = ws.srt_ci;
    int* srt_key = ws.srt_key;
    double* band_x = ws.band_x;
    int* band_l = ws.band_l;
    double* best_x = ws.best_x;
    int* best_l = ws.best_l;
    int* misc = ws.misc;
    (void)M;

    const Geo& g = a.g;
    const int lane = threadIdx.x % kWave;
    const long t = long(b) * a.n_refs + gi;
    const int r = safe_origin(int(a.refs[gi]), last_origin(g));

    // ---- window origins (clipped)
    int lo[kAx], n[kAx], rc[kAx];
    int ncand = 1;
#pragma unroll
    for (int d = 0; d < kAx; ++d) {
        rc[d] = (r / g.st[d]) % g.L[d];
        lo[d] = max(rc[d] - g.W[d] / 2, 0);
        const int hi = min(rc[d] + g.W[d] - 1 - g.W[d] / 2, g.ell[d]);
        n[d] = hi - lo[d] + 1;
        ncand *= n[d];
    }
    // offset in sx of the region's first sample
    int rbase = 0;
#pragma unroll
    for (int d = 0; d < kAx; ++d) rbase += (lo[d] - sorg[d]) * sst[d];

    // ---- reference patch (rows along the last axis, at offsets roff)
    const int rows = g.P / g.j[kAx - 1];
    int rb = 0;  // the reference's own origin in sx
#pragma unroll
    for (int d = 0; d < kAx; ++d) rb += (rc[d] - sorg[d]) * sst[d];
    const bool bytes = MODE == kCount && sb != nullptr;
    S rp[MR][J3];
    S sr = 0;
    if (!bytes) {
#pragma unroll
        for (int q = 0; q < MR; ++q)
#pragma unroll
            for (int i = 0; i < J3; ++i) {
                rp[q][i] = q < rows ? from_int<S>(sx[rb + roff[q] + i]) : S(0);
                sr += rp[q][i];
            }
    }
    int rci = 0;  // the reference's candidate index
    {
        int stride = 1;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            rci += (rc[d] - lo[d]) * stride;
            stride *= n[d];
        }
    }

    // window-offset index of a candidate (correlated noise: the bias of the
    // displacement from the reference), C-order over the W_d offsets
    int wst[kAx];
    {
        int st = 1;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            wst[d] = st;
            st *= g.W[d];
        }
    }
    auto woff = [&](int ci) {
        int rem = ci, o = 0;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            o += (lo[d] + rem % n[d] - rc[d] + g.W[d] / 2) * wst[d];
            rem /= n[d];
        }
        return o;
    };

    // ---- scores of every candidate, and the range of the finite keys
    unsigned kmn = 0xFFFFFFFFu, kmx = 0u;
    const float bmag = MODE == kGauss ? (a.bias_t ? float(*a.bias_bound) : fabsf(a.bias)) : 0.f;
    const int n3 = n[kAx - 1];
    const int rpr = (n3 + kRB - 1) / kRB;  // runs per line
    const int nruns = (ncand / n3) * rpr;
    if constexpr (MODE == kCount) {
        if (bytes) {
            // count mode on bytes: SSD = sum p^2 + sum q^2 - 2 sum pq, bias
            // gamma (sum p + sum q), every sum a v_dot4_u32_u8 chain
            constexpr int NW = J3 / 4;     // words per patch row
            constexpr unsigned kOnes = 0x01010101u;
            unsigned rw[MR][NW];
            unsigned sp2 = 0, sp1 = 0;
            {
                const unsigned* cr =
                    reinterpret_cast<const unsigned*>(sb + (rb & 3) * cst) + (rb >> 2);
#pragma unroll
                for (int q = 0; q < MR; ++q)
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        rw[q][w] = q < rows ? cr[(roff[q] >> 2) + w] : 0u;
                        sp2 = __builtin_amdgcn_udot4(rw[q][w], rw[q][w], sp2, false);
                        sp1 = __builtin_amdgcn_udot4(rw[q][w], kOnes, sp1, false);
                    }
            }
            // words spanning a run's row segment (kRB + J3 - 1 samples)
            constexpr int NWR = (kRB + J3 - 1 + 3) / 4;
            for (int run = lane; run < nruns; run += kWave) {
                const int line = run / rpr;
                const int c3 = (run - line * rpr) * kRB;
                int cb = rbase + c3, rem = line;
#pragma unroll
                for (int d = kAx - 2; d >= 0; --d) {
                    cb += (rem % n[d]) * sst[d];
                    rem /= n[d];
                }
                // the copy in which sample cb starts a word: word k of a
                // row holds the row's samples 4k .. 4k + 3 from the run's
                // start, and the 4 samples from any offset o are a byte
                // alignment of words o / 4 and o / 4 + 1
                const unsigned* cw =
                    reinterpret_cast<const unsigned*>(sb + (cb & 3) * cst) + (cb >> 2);
                unsigned pq[kRB], q2[kRB], q1[kRB];
#pragma unroll
                for (int u = 0; u < kRB; ++u) pq[u] = q2[u] = q1[u] = 0u;
#pragma unroll
                for (int q = 0; q < MR; ++q) {
                    if (q < rows) {
                        unsigned wv[NWR];
#pragma unroll
                        for (int k = 0; k < NWR; ++k) wv[k] = cw[(roff[q] >> 2) + k];
#pragma unroll
                        for (int u = 0; u < kRB; ++u)
#pragma unroll
                            for (int w = 0; w < NW; ++w) {
                                const int o = u + 4 * w;
                                const unsigned qw =
                                    (o & 3) == 0 ? wv[o >> 2]
                                                 : __builtin_amdgcn_alignbyte(wv[(o >> 2) + 1],
                                                                              wv[o >> 2], o & 3);
                                pq[u] = __builtin_amdgcn_udot4(rw[q][w], qw, pq[u], false);
                                q2[u] = __builtin_amdgcn_udot4(qw, qw, q2[u], false);
                                q1[u] = __builtin_amdgcn_udot4(qw, kOnes, q1[u], false);
                            }
                    }
                }
#pragma unroll
                for (int u = 0; u < kRB; ++u) {
                    const int ci = line * n3 + c3 + u;
                    if (c3 + u < n3) {
                        int x = int(sp2 + q2[u] - 2u * pq[u]) - a.gamma_i * int(sp1 + q1[u]);
                        if (ci == rci) x = INT_MAX;
                        xs[ci] = x;
                        if (ci != rci) {
                            kmn = min(kmn, okey(x));
                            kmx = max(kmx, okey(x));
                        }
                    }
                }
            }
        }
    }
    for (int run = lane; run < (bytes ? 0 : nruns); run += kWave) {
        const int line = run / rpr;
        const int c3 = (run - line * rpr) * kRB;
        int cb = rbase + c3, rem = line;
#pragma unroll
        for (int d = kAx - 2; d >= 0; --d) {
            cb += (rem % n[d]) * sst[d];
            rem /= n[d];
        }
        // window offset of the run's first candidate
        int wb = (lo[kAx - 1] + c3 - rc[kAx - 1] + g.W[kAx - 1] / 2);
        {
            int rem2 = line;
#pragma unroll
            for (int d = kAx - 2; d >= 0; --d) {
                wb += (lo[d] + rem2 % n[d] - rc[d] + g.W[d] / 2) * wst[d];
                rem2 /= n[d];
            }
        }
        S acc[kRB], sq[kRB], bq[kRB];
#pragma unroll
        for (int u = 0; u < kRB; ++u) acc[u] = sq[u] = bq[u] = S(0);
#pragma unroll
        for (int q = 0; q < MR; ++q) {
            if (q < rows) {
                S seg[SEG];
#pragma unroll
                for (int k = 0; k < SEG; ++k) seg[k] = from_int<S>(sx[cb + roff[q] + k]);
#pragma unroll
                for (int u = 0; u < kRB; ++u) {
#pragma unroll
                    for (int i = 0; i < J3; ++i) {
                        const S df = seg[u + i] - rp[q][i];
                        if constexpr (MODE == kCount) acc[u] += __mul24(df, df);
                        else acc[u] = __builtin_fmaf(df, df, acc[u]);
                        if constexpr (MODE == kCount) sq[u] += seg[u + i];
                        if constexpr (MODE == kPoissonF) bq[u] += fmaxf(seg[u + i] + rp[q][i], 0.f);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kRB; ++u) {
            const int ci = line * n3 + c3 + u;
            if (c3 + u < n3) {
                S x = acc[u];
                if constexpr (MODE == kCount) x -= a.gamma_i * (sr + sq[u]);
                if constexpr (MODE == kGauss) x -= a.bias_t ? a.bias_t[wb + u] : a.bias;
                if constexpr (MODE == kPoissonF) x = __builtin_fmaf(-a.gamma_sp, bq[u], x);
                if constexpr (kF) x = x == x ? x : bigv<S>();
                if (ci == rci) x = bigv<S>();
                xs[ci] = as_int(x);
                if (okey(x) != okey(bigv<S>())) {
                    kmn = min(kmn, okey(x));
                    kmx = max(kmx, okey(x));
                }
            }
        }
    }
    wsync();

    // ---- accepted count -> group size
    float tau_band = 0.f;
    if constexpr (kF) tau_band = float(kTieBand) * (fabsf(a.tau_f) + bmag);
    const unsigned kbig = okey(bigv<S>());  // excluded: the reference, non-finite scores
    // the histogram of 256 equal bins over the keys' range is built in the
    // same pass (level 1 of the selection below)
    kmn = wmin_u(kmn);
    kmx = wmax_u(kmx);
    const unsigned span = kmx > kmn ? kmx - kmn : 0u;
    const int sh = span < 256u ? 0 : (32 - __clz(span)) - 8;   // span >> sh < 256
    for (int h = lane; h < 256; h += kWave) hist[h] = 0u;
    wsync();
    // The passes over the scores read four per lane before using them (four
    // LDS reads in flight); the reference's own score is the excluded key.
    auto load4 = [&](int c0, unsigned (&kk)[4]) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int ci = c0 + h * kWave + lane;
            kk[h] = ci < ncand ? okey(from_int<S>(xs[ci])) : kbig;
        }
    };
    int acc = 0, namb = 0, nfin = 0;
    for (int c0 = 0; c0 < ncand; c0 += 4 * kWave) {
        unsigned kk[4];
        load4(c0, kk);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const unsigned kx = kk[h];
            if (kx == kbig) continue;
            const S x = key_value<S>(kx);
            ++nfin;
            if (span != 0u) atomicAdd(&hist[(kx - kmn) >> sh], 1u);
            if constexpr (MODE == kCount) {
                acc += x < a.tau_i;
            } else {
                // acc: certain acceptances; namb: the band around tau
                const bool amb = fabsf(x - a.tau_f) <= tau_band;
                acc += x < a.tau_f && !amb;
                namb += amb;
            }
        }
    }
    acc = wsum(acc);
    nfin = wsum(nfin);
    const int ncand_nr = ncand - 1;  // without the reference
    auto group_size = [&](int acc_) {
        int k = p2fl(min(1 + acc_, a.gmax));
        k = max(k, a.gmin);
        return min(k, p2fl(1 + ncand_nr));
    };
    int K = group_size(acc);
    if constexpr (kF) {
        namb = wsum(namb);
        if (namb > 0 && group_size(acc + namb) != K) {
            // scores within the band of tau are accepted or not in FP64
            int acc2 = 0;
            for (int ci = lane; ci < ncand; ci += kWave) {
                if (ci == rci) continue;
                const float x = __int_as_float(xs[ci]);
                if (fabsf(x - a.tau_f) <= tau_band) {
                    // FP64 score of candidate ci (lin order = C order)
                    int rem = ci, cbo = rbase;
#pragma unroll
                    for (int d = kAx - 1; d >= 0; --d) {
                        cbo += (rem % n[d]) * sst[d];
                        rem /= n[d];
                    }
                    double s = 0.0, bb = 0.0;
                    for (int q = 0; q < rows; ++q)
                        for (int i = 0; i < g.j[kAx - 1]; ++i) {
                            const double pv = __int_as_float(sx[rb + roff[q] + i]);
                            const double qv = __int_as_float(sx[cbo + roff[q] + i]);
                            const double df = __dsub_rn(qv, pv);
                            s = __dadd_rn(s, __dmul_rn(df, df));
                            if constexpr (MODE == kPoissonF) bb = __dadd_rn(bb, fmax(__dadd_rn(pv, qv), 0.0));
                        }
                    if constexpr (MODE == kGauss) s = __dsub_rn(s, a.bias_td ? a.bias_td[woff(ci)] : a.bias_d);
                    if constexpr (MODE == kPoissonF) s = __dsub_rn(s, __dmul_rn(a.gamma_sp_d, bb));
                    acc2 += s < a.tau_d;
                } else {
                    acc2 += x < a.tau_f;
                }
            }
            K = group_size(wsum(acc2));
        }
    }
    // non-finite scores are never selected: fewer finite candidates than
    // asked cut the group to the largest power of two they fill
    if (GM > 1 && nfin < K - 1) K = p2fl(1 + nfin);
    const int need = GM > 1 ? K - 1 : 0;
    int* out = a.match + t * a.gmax;
    if (need == 0) {
        for (int m = lane; m < a.gmax; m += kWave) out[m] = m == 0 ? r : -1;
        if (lane == 0) a.count[t] = K;
        return;
    }

    // ---- the need-th smallest finite key.  Level 1: a histogram of 256
    // equal bins over the keys' range [kmn, kmx] gives the bin that holds
    // the rank; level 2: the keys of that bin, at most one per lane, are
    // ranked exactly.  A fuller bin falls back to a radix select, 8 bits at
    // a time, among its keys.
    unsigned theta_key = kmn;   // all finite keys equal: that key is the need-th
    int less_total = 0;         // finite keys below theta (-1: not known yet)
    bool members_done = false;  // the members already in sel_* (and, float modes, nb)
    int nb = 0;                 // float modes: candidates up to theta plus the band
    // histogram of f(k) over the finite keys with in(k), then the bin of the
    // rank-th smallest (1-based) and the rank within it: misc[0], misc[1]
    auto bin_of_rank = [&](auto f, auto in, int rank_, bool built) {
        if (!built) {
            for (int h = lane; h < 256; h += kWave) hist[h] = 0u;
            wsync();
            for (int ci = lane; ci < ncand; ci += kWave) {
                if (ci == rci) continue;
                const unsigned k = okey(from_int<S>(xs[ci]));
                if (k != kbig && in(k)) atomicAdd(&hist[f(k)], 1u);
            }
        }
        wsync();
        // each lane owns 4 consecutive bins; a wave prefix sum gives the
        // keys below each lane's bins, and the lane whose range holds the
        // rank writes the bin
        const uint4 h4 = *reinterpret_cast<const uint4*>(&hist[4 * lane]);
        const int c0 = int(h4.x), c1 = int(h4.y), c2 = int(h4.z), c3 = int(h4.w);
        const int tot = c0 + c1 + c2 + c3;
        const int below = wscan_ex(tot);
        if (below < rank_ && below + tot >= rank_) {
            int c = below, bin = 4 * lane;
            if (c + c0 < rank_) {
                c += c0;
                ++bin;
                if (c + c1 < rank_) {
                    c += c1;
                    ++bin;
                    if (c + c2 < rank_) {
                        c += c2;
                        ++bin;
                    }
                }
            }
            misc[0] = bin;
            misc[1] = rank_ - c;
        }
        wsync();
    };
    if (span != 0u) {
        auto lvl = [&](unsigned k) { return (k - kmn) >> sh; };
        bin_of_rank(lvl, [](unsigned) { return true; }, need, true);
        const unsigned B = unsigned(misc[0]);
        const int rank = misc[1];
        const int cB = int(hist[B]);
        const unsigned blo = kmn + (B << sh);
        wsync();
        const unsigned long long top = (unsigned long long)blo + ((1ull << sh) - 1ull);
        const unsigned bhi = unsigned(top < kmx ? top : kmx);   // the bin's key range
        if (sh == 0 || bhi == blo) {
            theta_key = blo;   // a bin of one key value
            less_total = need - rank;
        } else if (cB <= kWave) {
            // One pass takes the keys of the bins below B as members (slots in
            // window order) and compacts the keys of bin B with their window
            // indices into hist[0 .. cB) and hist[64 .. 64 + cB); the rank
            // smallest of those by (key, window index) complete the members.
            const unsigned long long below = (1ull << lane) - 1ull;
            int mbase = 0, cbase = 0, nz_low = 0;
            for (int c0 = 0; c0 < ncand; c0 += 4 * kWave) {
                unsigned kk[4];
                load4(c0, kk);
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int ci = c0 + h * kWave + lane;
                    const unsigned k = kk[h];
                    const unsigned lv = k != kbig ? lvl(k) : 0xFFFFFFFFu;
                    const bool low = lv < B, inb = lv == B;
                    if constexpr (kF) nz_low += low && key_float(k) == 0.f;
                    const unsigned long long bl = __ballot(low);
                    if (low) {
                        const int slot = mbase + int(__popcll(bl & below));
                        sel_ci[slot] = ci;
                        sel_key[slot] = int(k ^ 0x80000000u);  // signed order = key order
                    }
                    mbase += int(__popcll(bl));
                    const unsigned long long bb = __ballot(inb);
                    if (inb) {
                        const int at = cbase + int(__popcll(bb & below));
                        hist[at] = k;
                        hist[64 + at] = unsigned(ci);
                    }
                    cbase += int(__popcll(bb));
                }
            }
            wsync();
            // each lane's entry against every other, read across lanes
            const unsigned kj = lane < cB ? hist[lane] : 0u;
            const int cj = lane < cB ? int(hist[64 + lane]) : 0;
            int rk = 0;
            const int cBu = __builtin_amdgcn_readfirstlane(cB);   // uniform
            for (int o = 0; o < cBu; ++o) {
                const unsigned ko = unsigned(__builtin_amdgcn_readlane(int(kj), o));
                const int co = __builtin_amdgcn_readlane(cj, o);
                rk += ko < kj || (ko == kj && co < cj);
            }
            const int low_n = need - rank;   // members below bin B (= mbase)
            if (lane < cB && rk < rank) {
                sel_ci[low_n + rk] = cj;
                sel_key[low_n + rk] = int(kj ^ 0x80000000u);
            }
            if (lane < cB && rk == rank - 1) misc[2] = int(kj);
            wsync();
            theta_key = unsigned(misc[2]);
            if constexpr (kF) {
                // candidates up to theta plus the band: the bins below B
                // (less the -0 scores when theta is 0), bin B's entries up to
                // the band, and past bin B only when the band reaches beyond it
                const float th_ = key_float(theta_key);
                const float thr_ = th_ + float(kTieBand) * (fabsf(th_) + bmag);
                const float xj = key_float(kj);
                const bool inband = lane < cB && xj <= thr_ && !(xj == 0.f && th_ == 0.f);
                int tot = low_n - (th_ == 0.f ? wsum(nz_low) : 0) + int(__popcll(__ballot(inband)));
                if (!(okey(thr_) <= bhi)) {
                    int nx = 0;
                    for (int ci = lane; ci < ncand; ci += kWave) {
                        if (ci == rci) continue;
                        const unsigned k = okey(from_int<S>(xs[ci]));
                        const float x = key_float(k);
                        nx += k > bhi && x <= thr_;
                    }
                    tot += wsum(nx);
                }
                nb = lane == 0 ? tot : 0;   // summed over the wavefront below
            }
            members_done = true;
            wsync();
        } else {
            // radix select among the bin's keys, from the highest byte in
            // which the bin's key range [blo, bhi] varies
            const unsigned kd = blo ^ bhi;
            int shift = ((31 - __clz(kd)) >> 3) << 3;
            unsigned pmask = shift >= 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
            unsigned prefix = blo & pmask;
            int r2 = rank;
            for (; shift >= 0; shift -= 8) {
                const int s_ = shift;
                const unsigned pm = pmask, pf = prefix;
                bin_of_rank([s_](unsigned k) { return (k >> s_) & 255u; },
                            [&](unsigned k) { return lvl(k) == B && (k & pm) == pf; }, r2,
                            false);
                prefix |= unsigned(misc[0]) << shift;
                pmask |= 255u << shift;
                r2 = misc[1];
                wsync();
            }
            theta_key = prefix;
            less_total = -1;
        }
    }
    // members: keys below theta, then the first ties at theta in lin order
    // (candidate order is lin order), in one pass of rounds over the
    // candidates with slots from ballots
    if (!members_done && less_total < 0) {
        int nl = 0;
        for (int ci = lane; ci < ncand; ci += kWave) {
            if (ci == rci) continue;
            nl += okey(from_int<S>(xs[ci])) < theta_key;   // kbig is never below theta
        }
        less_total = wsum(nl);
    }
    // float modes: the same pass counts the candidates up to theta plus the
    // FP32 band above it (nb, for the near-tie check below)
    const float th = kF ? key_float(theta_key) : 0.f;
    const float thr = kF ? th + float(kTieBand) * (fabsf(th) + bmag) : 0.f;
    if (!members_done) {
        const unsigned long long below = (1ull << lane) - 1ull;
        int ties_left = need - less_total;
        int base = 0;
        for (int c0 = 0; c0 < ncand; c0 += 4 * kWave) {
            unsigned kk[4];
            load4(c0, kk);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int ci = c0 + h * kWave + lane;
                const unsigned k = kk[h];
                if constexpr (kF) {
                    const float x = key_float(k);
                    nb += ci < ncand && ci != rci && x <= thr && !(x == 0.f && th == 0.f);
                }
                const bool eq = k == theta_key && k != kbig;
                const unsigned long long beq = __ballot(eq);
                // (the population counts are unsigned: kept out of signed arithmetic)
                const int eq_rank = int(__popcll(beq & below)), n_eq = int(__popcll(beq));
                const bool take = k < theta_key || (eq && eq_rank < ties_left);
                ties_left = ties_left > n_eq ? ties_left - n_eq : 0;
                const unsigned long long bt = __ballot(take);
                if (take) {
                    const int slot = base + int(__popcll(bt & below));
                    sel_ci[slot] = ci;
                    sel_key[slot] = int(k ^ 0x80000000u);  // signed order = key order
                }
                base += int(__popcll(bt));
            }
        }
    }
    wsync();
    // ranked by (key, window index), the members read across lanes (need
    // <= 31 < kWave)
    {
        const int km = lane < need ? sel_key[lane] : 0, lm = lane < need ? sel_ci[lane] : 0;
        int rk = 0;
        const int nu = __builtin_amdgcn_readfirstlane(need);   // uniform
        for (int o = 0; o < nu; ++o) {
            const int ko = __builtin_amdgcn_readlane(km, o);
            const int lo_ = __builtin_amdgcn_readlane(lm, o);
            rk += ko < km || (ko == km && lo_ < lm);
        }
        if (lane < need) {
            srt_key[rk] = km;
            srt_ci[rk] = lm;
        }
    }
    wsync();
    int got = need;

    bool fp64 = false;
    if constexpr (kF) {
        // FP32 ranking = FP64 ranking unless a non-member lies within the
        // band above theta, or two members lie within the band of each other
        // (equal zeros are exact)
        nb = wsum(nb);
        // members within the band above theta; two members within the band
        // of each other (the band of the larger): if any pair is, so is a
        // pair adjacent in the ranking with the same larger member
        int members_in_band = 0, close = 0;
        for (int m = lane; m < need; m += kWave) {
            const float xm = key_float(unsigned(srt_key[m]) ^ 0x80000000u);
            members_in_band += xm <= thr && !(xm == 0.f && th == 0.f);
            if (m + 1 < need) {
                const float hi_ = key_float(unsigned(srt_key[m + 1]) ^ 0x80000000u);
                close += hi_ - xm <= float(kTieBand) * (fabsf(hi_) + bmag) &&
                         !(hi_ == 0.f && xm == 0.f);
            }
        }
        const bool amb = nb > wsum(members_in_band) || wsum(close) > 0;
        fp64 = amb;
        // FP64 score of candidate ci (its window index ci is the order key)
        auto score64 = [&](int ci, int& lin) {
            int rem = ci, cbo = rbase;
            lin = ci;
#pragma unroll
            for (int d = kAx - 1; d >= 0; --d) {
                cbo += (rem % n[d]) * sst[d];
                rem /= n[d];
            }
            double s = 0.0, bb = 0.0;
            for (int q = 0; q < rows; ++q)
                for (int i = 0; i < g.j[kAx - 1]; ++i) {
                    const double pv = __int_as_float(sx[rb + roff[q] + i]);
                    const double qv = __int_as_float(sx[cbo + roff[q] + i]);
                    const double df = __dsub_rn(qv, pv);
                    s = __dadd_rn(s, __dmul_rn(df, df));
                    if constexpr (MODE == kPoissonF) bb = __dadd_rn(bb, fmax(__dadd_rn(pv, qv), 0.0));
                }
            if constexpr (MODE == kGauss) s = __dsub_rn(s, a.bias_td ? a.bias_td[woff(ci)] : a.bias_d);
            if constexpr (MODE == kPoissonF) s = __dsub_rn(s, __dmul_rn(a.gamma_sp_d, bb));
            return s;
        };
        // the candidates up to theta plus the band, in lin order (C order
        // over the window), when they fit one per lane
        int nbc = 0;
        if (fp64) {
            for (int c0 = 0; c0 < ncand; c0 += kWave) {
                const int ci = c0 + lane;
                const bool in = ci < ncand && ci != rci && __int_as_float(xs[ci]) <= thr;
                const unsigned long long bal = __ballot(in);
                const int at = nbc + int(__popcll(bal & ((1ull << lane) - 1ull)));
                if (in && at < kWave) band_l[at] = ci;
                nbc += int(__popcll(bal));
            }
            wsync();
        }
        if (fp64 && nbc <= kWave) {
            // each re-scored by one lane, then ranked by (FP64 score, lin)
            double x64 = 0.0;
            int lin = 0;
            bool ok = false;
            if (lane < nbc) {
                x64 = score64(band_l[lane], lin);
                ok = x64 == x64;
            }
            wsync();
            if (lane < nbc) {
                band_x[lane] = ok ? x64 : __longlong_as_double(0x7FF8000000000000LL);
                band_l[lane] = lin;
            }
            wsync();
            int rk = 0;
            if (ok) {
                for (int o = 0; o < nbc; ++o) {
                    const double xo = band_x[o];
                    const int lo_ = band_l[o];
                    rk += xo < x64 || (xo == x64 && lo_ < lin);   // NaN compares false
                }
            }
            if (ok && rk < need) {
                best_x[rk] = x64;
                best_l[rk] = lin;
            }
            got = min(wsum(ok ? 1 : 0), need);
            wsync();
        } else if (fp64) {
            // every candidate up to theta plus the band, re-scored in FP64 in
            // lin order, chunk by chunk; the best `need` by (FP64 score, lin)
            if (lane == 0) misc[2] = 0;  // entries in best_x
            wsync();
            for (int c0 = 0; c0 < ncand; c0 += kBandCap) {
                if (lane == 0) misc[3] = 0;
                wsync();
                for (int ci = c0 + lane; ci < min(ncand, c0 + kBandCap); ci += kWave) {
                    if (ci == rci) continue;
                    const float x = __int_as_float(xs[ci]);
                    if (!(x <= thr)) continue;
                    int lin = 0;
                    const double s = score64(ci, lin);
                    if (!(s == s)) continue;
                    const int slot = atomicAdd(&misc[3], 1);
                    band_x[slot] = s;
                    band_l[slot] = lin;
                }
                wsync();
                // merge the chunk into the running best list: rank counting
                const int nb_c = misc[3], nbest = misc[2];
                const int tot = nb_c + nbest;
                double my_x[4];
                int my_l[4], my_r[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int e = lane + k * kWave;
                    my_r[k] = INT_MAX;
                    if (e < tot) {
                        my_x[k] = e < nbest ? best_x[e] : band_x[e - nbest];
                        my_l[k] = e < nbest ? best_l[e] : band_l[e - nbest];
                        int rk = 0;
                        for (int o = 0; o < tot; ++o) {
                            const double xo = o < nbest ? best_x[o] : band_x[o - nbest];
                            const int lo_ = o < nbest ? best_l[o] : band_l[o - nbest];
                            rk += xo < my_x[k] || (xo == my_x[k] && lo_ < my_l[k]);
                        }
                        my_r[k] = rk;
                    }
                }
                wsync();
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (my_r[k] < need) {
                        best_x[my_r[k]] = my_x[k];
                        best_l[my_r[k]] = my_l[k];
                    }
                }
                if (lane == 0) misc[2] = min(tot, need);
                wsync();
            }
            got = misc[2];
            wsync();
        }
    }

    // ---- output: members ranked by (score, lin)
    if (got < need) K = p2fl(1 + got);
    if (lane == 0) {
        a.count[t] = K;
        out[0] = r;
    }
    for (int m = K + lane; m < a.gmax; m += kWave) out[m] = -1;
    for (int m = lane; m < K - 1; m += kWave) {
        // lin of the member's window index (C order over the window)
        int rem = fp64 ? best_l[m] : srt_ci[m], lin = 0;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            lin += (lo[d] + rem % n[d]) * g.st[d];
            rem /= n[d];
        }
        out[1 + m] = lin;
    }
}

// Stages the box of `ext` samples per axis from array coordinates `org`
// (thread tid of nthreads) into sx, sample (c_0, ..., c_3) of the box at
// sum_d c_d sst[d]: raw counts for count-domain scoring, float bit patterns
// otherwise; positions outside the array are 0 (no candidate reads them).
// Coordinates advance by the thread stride with carries, without a
// division per sample.
template <int MODE>
__device__ __forceinline__ void stage_box(const MatchArgs& a, int kmax, const float* src,
                                          const int* org, const int* ext, int total,
                                          const int* sst, int* sx, int tid, int nthreads)
{
    const Geo& g = a.g;
    int c[kAx], dc[kAx];
    {
        int rem = tid, st = nthreads;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            c[d] = rem % ext[d];
            rem /= ext[d];
            dc[d] = st % ext[d];
            st /= ext[d];
        }
    }
    for (int e = tid; e < total; e += nthreads) {
        bool in = true;
        int u = 0;
#pragma unroll
        for (int d = 0; d < kAx; ++d) {
            const int x = org[d] + c[d];
            in = in && x >= 0 && x < g.L[d];
            u += x * g.st[d];
        }
        int v = 0, p = 0;
#pragma unroll
        for (int d = 0; d < kAx; ++d) p += c[d] * sst[d];
        if (in) {
            const float x = src[u];
            if constexpr (MODE == kCount) {
                // non-finite or out-of-range counts are flagged (scored as 0)
                const float rk = rintf(x * a.inv_sp);
                const bool ok = rk >= 0.f && rk <= float(kmax);
                if (!ok) atomicOr(a.range_flag, 1);
                v = ok ? int(rk) : 0;
            } else {
                v = __float_as_int(x);
            }
        }
        sx[p] = v;
        // advance by nthreads: add the per-axis digits with carries
        int carry = 0;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            c[d] += dc[d] + carry;
            carry = 0;
            while (c[d] >= ext[d]) {
                c[d] -= ext[d];
                ++carry;
            }
        }
    }
}

// One wavefront per reference (any reference list): the reference's own
// clipped region staged alone.
template <int MODE, int GM, int J3>
__global__ __launch_bounds__(kWave) void k_match_nd(MatchArgs a, int kmax)
{
    extern __shared__ __align__(16) int smem[];
    __shared__ WaveSel<GM> ws;
    const Geo& g = a.g;
    const int lane = threadIdx.x;
    const int b = blockIdx.x / a.n_refs;
    const int gi = blockIdx.x - b * a.n_refs;
    const int r = safe_origin(int(a.refs[gi]), last_origin(g));
    int lo[kAx], R[kAx], sst[kAx];
    int nreg = 1;
#pragma unroll
    for (int d = 0; d < kAx; ++d) {
        const int rc = (r / g.st[d]) % g.L[d];
        lo[d] = max(rc - g.W[d] / 2, 0);
        const int hi = min(rc + g.W[d] - 1 - g.W[d] / 2, g.ell[d]);
        R[d] = hi - lo[d] + g.j[d];
        nreg *= R[d];
    }
    {
        int st = 1;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            sst[d] = st;
            st *= R[d];
        }
    }
    int* sx = smem;                   // [nreg + kPad] staged samples
    int* xs = smem + nreg + kPad;     // [ncand] scores (bit patterns)
    stage_box<MODE>(a, kmax, a.src + long(b) * g.V, lo, R, nreg, sst, sx, lane, kWave);
    for (int e = nreg + lane; e < nreg + kPad; e += kWave) sx[e] = 0;
    wsync();
    int roff[64 / J3];
    row_offsets(g, sst, roff);
    match_one<MODE, GM, J3, kRB>(a, b, gi, sx, lo, sst, roff, xs, ws, nullptr, 0);
}

// Candidates per run along the last axis in the block kernel: runs fill
// the 11-candidate lines of 4-sample patches and the 39-candidate lines of
// 8-sample patches.
constexpr int blk_rb(int j3) { return j3 == 4 ? 11 : 13; }

// LDS words of a block's staged box: the 32-bit copy with its pad; in
// count mode also the four byte copies (the same memory), whichever is
// larger.
__host__ __device__ inline int blk_box_words(const NdBlocks& blk, bool count)
{
    return !count || blk.mbox + kPad > blk.mcst ? blk.mbox + kPad : blk.mcst;
}

// One workgroup per spatial block of references (the list in block order,
// inside bmnd_denoise): the block's box (the block, the search window and a
// patch per axis) is staged once and serves every reference of the block,
// one wavefront per reference at a time.
constexpr int kMWaves = 4;

template <int MODE, int GM, int J3>
__global__ __launch_bounds__(kMWaves * kWave) void k_match_blk(MatchArgs a, int kmax,
                                                               NdBlocks blk, int ncand_max)
{
    extern __shared__ __align__(16) int smem[];
    __shared__ WaveSel<GM> ws[kMWaves];
    const Geo& g = a.g;
    const int wave = threadIdx.x / kWave;
    // (workgroups in block order: a contiguous run of blocks per XCD was
    // slower here, unlike in the filter)
    const int blkid = blockIdx.x % blk.nblocks;
    const int b = blockIdx.x / blk.nblocks;
    const int r0 = blk.start[blkid], r1 = blk.start[blkid + 1];
    if (r0 >= r1) return;   // an empty block (uniform over the workgroup)
    int blo[kAx];
    {
        int rem = blkid;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            const int bc = rem % blk.nb[d];
            rem /= blk.nb[d];
            blo[d] = bc * blk.B[d] - g.W[d] / 2;
        }
    }
    constexpr int RB = blk_rb(J3);
    int* sx = smem;                                        // [box words]
    int* xs = smem + blk_box_words(blk, MODE == kCount) + wave * ncand_max;   // [ncand] per wavefront
    const float* src = a.src + long(b) * g.V;
    const unsigned char* sb = nullptr;
    int cst = 0;
    if constexpr (MODE == kCount) {
        // counts of the box as four byte-shifted copies in the same LDS (each
        // copy box + kPad bytes, zero past the box and in the row and plane
        // padding) when every count fits a byte; otherwise staged again as
        // integers below.  Copy 0 is written a word (4 samples of a row) per
        // thread and item; word w of copy c is then bytes 4 w + c .. 4 w + c
        // + 3 of copy 0, a byte alignment of its words w and w + 1.
        __shared__ int big;
        if (threadIdx.x == 0) big = 0;
        cst = blk.mcst;
        unsigned char* cb = reinterpret_cast<unsigned char*>(smem);
        unsigned* w0 = reinterpret_cast<unsigned*>(smem);
        const int nw0 = cst >> 2;   // words of a copy
        __syncthreads();
        {
            // kSw words per thread at a time: the samples of all of them are
            // loaded before the first is used (one memory round trip)
            constexpr int kSw = 4;
            constexpr int kTh = kMWaves * kWave;
            bool over = false;
            for (int wb = threadIdx.x; wb < nw0; wb += kSw * kTh) {
                float xv[kSw][4];
                bool ld[kSw][4];
#pragma unroll
                for (int q = 0; q < kSw; ++q) {
                    int rem = 4 * (wb + q * kTh);
                    // box coordinates of the word's first sample (the rows
                    // start on word boundaries)
                    bool in = wb + q * kTh < nw0 && rem < blk.mbox_b;
                    int base = 0;
#pragma unroll
                    for (int d = 0; d < kAx - 1; ++d) {
                        const int c = rem / blk.MSb[d];
                        rem -= c * blk.MSb[d];
                        const int x = blo[d] + c;
                        in = in && c < blk.E[d] && x >= 0 && x < g.L[d];
                        base += x * g.st[d];
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int c3 = rem + k, x3 = blo[kAx - 1] + c3;
                        ld[q][k] = in && c3 < blk.E[kAx - 1] && x3 >= 0 && x3 < g.L[kAx - 1];
                        xv[q][k] = ld[q][k] ? src[base + x3 * g.st[kAx - 1]] : 0.f;
                    }
                }
#pragma unroll
                for (int q = 0; q < kSw; ++q) {
                    const int w = wb + q * kTh;
                    if (w >= nw0) break;
                    unsigned word = 0u;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        int v = 0;
                        if (ld[q][k]) {
                            const float rk = rintf(xv[q][k] * a.inv_sp);
                            const bool ok = rk >= 0.f && rk <= float(kmax);
                            if (!ok) atomicOr(a.range_flag, 1);
                            v = ok ? int(rk) : 0;
                        }
                        over = over || v > 255;
                        word |= unsigned(v & 255) << (8 * k);
                    }
                    w0[w] = word;
                }
            }
            if (over) atomicOr(&big, 1);
        }
        __syncthreads();
        for (int w = threadIdx.x; w < nw0; w += kMWaves * kWave) {
            const unsigned lw = w0[w], hw = w + 1 < nw0 ? w0[w + 1] : 0u;
#pragma unroll
            for (int c = 1; c < 4; ++c) w0[c * nw0 + w] = __builtin_amdgcn_alignbyte(hw, lw, c);
        }
        __syncthreads();
        if (big == 0) sb = cb;
    }
    if (sb == nullptr) {
        if constexpr (MODE == kCount) __syncthreads();   // the byte copies are done with
        // four consecutive samples of a box row per thread and item (the
        // row's coordinates from one division chain per item)
        const int cpr = (blk.E[kAx - 1] + 3) >> 2;   // items a row
        const int nitems = (blk.box_size / blk.E[kAx - 1]) * cpr;
        // kSi items per thread at a time, all loaded before the first is used
        constexpr int kSi = 4;
        constexpr int kTh = kMWaves * kWave;
        for (int ib = threadIdx.x; ib < nitems; ib += kSi * kTh) {
            float xv[kSi][4];
            bool ld[kSi][4];
            int pp[kSi];
#pragma unroll
            for (int q = 0; q < kSi; ++q) {
                const int it = ib + q * kTh;
                int row = it / cpr;
                const int c3 = 4 * (it - row * cpr);
                bool in = it < nitems;
                int base = 0, p = c3;
#pragma unroll
                for (int d = kAx - 2; d >= 0; --d) {
                    const int c = row % blk.E[d];
                    row /= blk.E[d];
                    const int x = blo[d] + c;
                    in = in && x >= 0 && x < g.L[d];
                    base += x * g.st[d];
                    p += c * blk.MS[d];
                }
                pp[q] = p;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int x3 = blo[kAx - 1] + c3 + k;
                    ld[q][k] = in && c3 + k < blk.E[kAx - 1] && x3 >= 0 && x3 < g.L[kAx - 1];
                    xv[q][k] = ld[q][k] ? src[base + x3 * g.st[kAx - 1]] : 0.f;
                }
            }
#pragma unroll
            for (int q = 0; q < kSi; ++q) {
                const int it = ib + q * kTh;
                if (it >= nitems) break;
                const int c3 = 4 * (it % cpr);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (c3 + k >= blk.E[kAx - 1]) break;
                    int v = 0;
                    if (ld[q][k]) {
                        if constexpr (MODE == kCount) {
                            // non-finite or out-of-range counts are flagged (scored as 0)
                            const float rk = rintf(xv[q][k] * a.inv_sp);
                            const bool ok = rk >= 0.f && rk <= float(kmax);
                            if (!ok) atomicOr(a.range_flag, 1);
                            v = ok ? int(rk) : 0;
                        } else {
                            v = __float_as_int(xv[q][k]);
                        }
                    }
                    sx[pp[q] + k] = v;
                }
            }
        }
        for (int e = blk.mbox + int(threadIdx.x); e < blk.mbox + kPad; e += kMWaves * kWave)
            sx[e] = 0;
    }
    __syncthreads();
    int sst[kAx];
#pragma unroll
    for (int d = 0; d < kAx; ++d) sst[d] = sb != nullptr ? blk.MSb[d] : blk.MS[d];
    int roff[64 / J3];
    row_offsets(g, sst, roff);
    // references taken from a shared counter: a wavefront that finishes
    // early (no FP64 re-ranking, a single-key bin) takes the next one
    __shared__ int next_ref;
    if (threadIdx.x == 0) next_ref = r0 + kMWaves;
    __syncthreads();
    for (int gi = r0 + wave; gi < r1;) {
        match_one<MODE, GM, J3, RB>(a, b, gi, sx, blo, sst, roff, xs, ws[wave], sb, cst);
        int nx = 0;
        if (threadIdx.x % kWave == 0) nx = atomicAdd(&next_ref, 1);
        gi = __builtin_amdgcn_readfirstlane(nx);
    }
}

}  // namespace

namespace {

template <int MODE, int J3>
hipError_t launch_nd_mode(const MatchArgs& a, int kmax, size_t lds, hipStream_t s)
{
    const dim3 grid(unsigned(long(a.n_refs) * a.g.batch));
    switch (a.gmax) {
    case 1: hipLaunchKernelGGL((k_match_nd<MODE, 1, J3>), grid, dim3(kWave), lds, s, a, kmax); break;
    case 2: hipLaunchKernelGGL((k_match_nd<MODE, 2, J3>), grid, dim3(kWave), lds, s, a, kmax); break;
    case 4: hipLaunchKernelGGL((k_match_nd<MODE, 4, J3>), grid, dim3(kWave), lds, s, a, kmax); break;
    case 8: hipLaunchKernelGGL((k_match_nd<MODE, 8, J3>), grid, dim3(kWave), lds, s, a, kmax); break;
    case 16: hipLaunchKernelGGL((k_match_nd<MODE, 16, J3>), grid, dim3(kWave), lds, s, a, kmax); break;
    default: hipLaunchKernelGGL((k_match_nd<MODE, 32, J3>), grid, dim3(kWave), lds, s, a, kmax); break;
    }
    return hipGetLastError();
}

template <int MODE, int GM, int J3>
hipError_t launch_blk3(const MatchArgs& a, int kmax, const NdBlocks& blk, int ncand_max,
                       size_t lds, hipStream_t s)
{
    const void* fn = reinterpret_cast<const void*>(&k_match_blk<MODE, GM, J3>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    const dim3 grid(unsigned(long(blk.nblocks) * a.g.batch));
    hipLaunchKernelGGL((k_match_blk<MODE, GM, J3>), grid, dim3(kMWaves * kWave), lds, s, a, kmax,
                       blk, ncand_max);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_blk(const MatchArgs& a, int kmax, const NdBlocks& blk, int ncand_max, size_t lds,
                      hipStream_t s)
{
    const bool three = a.g.j[kAx - 1] == 4;
    if (a.gmax == 16)
        return three ? launch_blk3<MODE, 16, 4>(a, kmax, blk, ncand_max, lds, s)
                     : launch_blk3<MODE, 16, 8>(a, kmax, blk, ncand_max, lds, s);
    return three ? launch_blk3<MODE, 32, 4>(a, kmax, blk, ncand_max, lds, s)
                 : launch_blk3<MODE, 32, 8>(a, kmax, blk, ncand_max, lds, s);
}

template <int MODE>
hipError_t launch_nd_j(const MatchArgs& a, int kmax, size_t lds, hipStream_t s)
{
    const int j3 = a.g.j[kAx - 1];
    if (j3 == 4) return launch_nd_mode<MODE, 4>(a, kmax, lds, s);
    if (j3 == 8) return launch_nd_mode<MODE, 8>(a, kmax, lds, s);
    return launch_nd_mode<MODE, 16>(a, kmax, lds, s);
}

}  // namespace

// window region (window origins plus a patch) and candidate counts of the
// largest window, for the LDS size
static void nd_sizes(const Geo& g, int* region, int* cand)
{
    int rg = 1, cd = 1;
    for (int d = 0; d < kAx; ++d) {
        const int nw = std::min(g.W[d], g.ell[d] + 1);
        rg *= nw + g.j[d] - 1;
        cd *= nw;
    }
    *region = rg;
    *cand = cd;
}

namespace {

// Bank collisions of a wavefront's reads in a staged box: lanes take runs of
// rb candidates in order, run = r + rpr * line with the line in C order over
// the window's other axes (positions n[0..2]), and read at the same offset
// from their run's first sample.  32-bit samples sit at strides S (words);
// byte copies (bytes true) at strides S in bytes, copy c at word offset
// c * x, a lane reading the word of its run's first sample in the copy of
// its byte phase.  Summed over the first run groups (and the four byte
// phases): the largest number of lanes on one bank, with 32 banks for each
// half of a wavefront plus with 64 banks for the whole of it.
int bank_cost(const int* n, const int* S, int rb, int rpr, bool bytes, int x)
{
    const int nruns = n[0] * n[1] * n[2] * rpr;
    int cost = 0;
    for (int g0 = 0; g0 < std::min(nruns, 4 * kWave); g0 += kWave)
        for (int v = 0; v < (bytes ? 4 : 1); ++v) {
            int c32[2][32] = {}, c64[64] = {};
            int w32 = 0, w64 = 0;
            for (int run = g0; run < std::min(nruns, g0 + kWave); ++run) {
                const int line = run / rpr, r = run - line * rpr;
                long p = long(rb) * r + v;
                int rem = line;
                for (int d = kAx - 2; d >= 0; --d) {
                    p += long(rem % n[d]) * S[d];
                    rem /= n[d];
                }
                const long w = bytes ? (p >> 2) + (p & 3) * long(x) : p;
                const int half = (run - g0) >> 5;
                w32 = std::max(w32, ++c32[half][w & 31]);
                w64 = std::max(w64, ++c64[w & 63]);
            }
            cost += w32 + w64;
        }
    return cost;
}

}  // namespace

// The matcher's LDS layouts of a block's box: row and plane strides padded
// so that the lanes of a wavefront, one run of candidates each, read from
// distinct banks where the padding allows it.  Candidates: row strides up
// to 32 samples past the row (multiples of 4 bytes for the byte copies),
// plane strides up to 32 words past the plane, and for byte copies whose
// lanes differ in byte phase (several runs a line) the copies' word offset
// mod 64.  The fewest collisions win, then the smallest box; a layout only
// counts while the workgroup's LDS stays within what the unpadded box
// needs or half a compute unit's LDS, whichever is larger, so that as many
// workgroups stay resident.  Outer strides of 4-D boxes are left unpadded.
void nd_match_layout(const Geo& g, NdBlocks& blk)
{
    const int rb = blk_rb(g.j[kAx - 1]);
    int n[kAx];
    for (int d = 0; d < kAx; ++d) n[d] = std::min(g.W[d], g.ell[d] + 1);
    const int rpr = (n[kAx - 1] + rb - 1) / rb;
    int region = 0, cand = 0;
    nd_sizes(g, &region, &cand);
    const long fixed = long(sizeof(int)) * kMWaves * cand + kMWaves * long(sizeof(WaveSel<32>));
    const long plain_words = blk.box_size + kPad;
    const long budget_words =
        std::max(plain_words, (80L * 1024L - fixed) / long(sizeof(int)));
    const bool plane = n[kAx - 3] > 1;   // lines span a second axis

    auto outer = [&](int* S) {
        for (int d = kAx - 4; d >= 0; --d) S[d] = blk.E[d + 1] * S[d + 1];
    };
    // 32-bit copy
    {
        int best = INT_MAX;
        long best_size = 0;
        int S[kAx];
        S[kAx - 1] = 1;
        for (int s2 = blk.E[kAx - 1]; s2 < blk.E[kAx - 1] + 32; ++s2)
            for (int s1 = blk.E[kAx - 2] * s2; s1 < blk.E[kAx - 2] * s2 + (plane ? 32 : 1); ++s1) {
                S[kAx - 2] = s2;
                S[kAx - 3] = s1;
                outer(S);
                const long size = long(blk.E[0]) * S[0];
                if (size + kPad > budget_words) continue;
                const int k = bank_cost(n, S, rb, rpr, false, 0);
                if (k < best || (k == best && size < best_size)) {
                    best = k;
                    best_size = size;
                    std::copy(S, S + kAx, blk.MS);
                }
            }
        if (best == INT_MAX) std::copy(blk.S, blk.S + kAx, blk.MS);
        blk.mbox = blk.E[0] * blk.MS[0];
    }
    // byte copies
    {
        int best = INT_MAX;
        long best_size = 0;
        int bx = 0;
        int S[kAx];
        S[kAx - 1] = 1;
        const int e3 = (blk.E[kAx - 1] + 3) & ~3;
        const int nx = rpr > 1 ? 64 : 1, xstep = plane ? 4 : 1;
        for (int s2 = e3; s2 < e3 + 32; s2 += 4)
            for (int s1 = blk.E[kAx - 2] * s2; s1 < blk.E[kAx - 2] * s2 + (plane ? 128 : 1);
                 s1 += 4)
                for (int x = 0; x < nx; x += xstep) {
                    S[kAx - 2] = s2;
                    S[kAx - 3] = s1;
                    outer(S);
                    const long bytes = long(blk.E[0]) * S[0];
                    long cst = (bytes + kPad + 3) & ~3L;
                    if (rpr > 1) cst += ((4L * x - cst) % 256 + 256) % 256;
                    if (cst > budget_words) continue;   // four copies: cst words
                    const int k = bank_cost(n, S, rb, rpr, true, x);
                    if (k < best || (k == best && cst < best_size)) {
                        best = k;
                        best_size = cst;
                        bx = x;
                        std::copy(S, S + kAx, blk.MSb);
                    }
                }
        if (best == INT_MAX) {
            std::copy(blk.S, blk.S + kAx, blk.MSb);
            blk.mbox_b = blk.box_size;
            blk.mcst = (blk.box_size + kPad + 3) & ~3;
        } else {
            blk.mbox_b = blk.E[0] * blk.MSb[0];
            long cst = (long(blk.mbox_b) + kPad + 3) & ~3L;
            if (rpr > 1) cst += ((4L * bx - cst) % 256 + 256) % 256;
            blk.mcst = int(cst);
        }
    }
}

bool match_nd_supported(const Geo& g)
{
    const int j3 = g.j[kAx - 1];
    // the row loops run over exactly the last-axis extent
    if (g.P > 64 || (j3 != 4 && j3 != 8 && j3 != 16)) return false;
    int region = 0, cand = 0;
    nd_sizes(g, &region, &cand);
    return region <= kMaxRegion && cand <= kMaxCand;
}

hipError_t launch_match_nd(const MatchArgs& a, int mode, int kmax, const NdBlocks* blk,
                           hipStream_t s)
{
    int region = 0, cand = 0;
    nd_sizes(a.g, &region, &cand);
    if (blk && (a.gmax == 16 || a.gmax == 32) &&
        (a.g.j[kAx - 1] == 4 || a.g.j[kAx - 1] == 8)) {
        // the block's box staged once per workgroup, beside one score array
        // per wavefront; within a compute unit's LDS with the static scratch
        const size_t lds =
            sizeof(int) * size_t(blk_box_words(*blk, mode == kCount) + kMWaves * cand);
        if (lds + kMWaves * sizeof(WaveSel<32>) <= 160u * 1024u) {
            switch (mode) {
            case kCount: return launch_blk<kCount>(a, kmax, *blk, cand, lds, s);
            case kPoissonF: return launch_blk<kPoissonF>(a, kmax, *blk, cand, lds, s);
            case kGauss: return launch_blk<kGauss>(a, kmax, *blk, cand, lds, s);
            default: return launch_blk<kPlain>(a, kmax, *blk, cand, lds, s);
            }
        }
    }
    const size_t lds = sizeof(int) * size_t(region + kPad + cand);
    switch (mode) {
    case kCount: return launch_nd_j<kCount>(a, kmax, lds, s);
    case kPoissonF: return launch_nd_j<kPoissonF>(a, kmax, lds, s);
    case kGauss: return launch_nd_j<kGauss>(a, kmax, lds, s);
    default: return launch_nd_j<kPlain>(a, kmax, lds, s);
    }
}

}  // namespace bmnd
