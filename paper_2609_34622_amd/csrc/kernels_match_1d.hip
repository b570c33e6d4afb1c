// Block matching for 1-D arrays with 32-sample patches (section Block
// Matching): one wavefront scores the windows of 64 consecutive
// references.  The samples covering their windows are staged once in LDS
// (raw counts for exact count-domain HT scores, the pilot for the Wiener
// stage); each lane keeps its reference patch in registers and walks the
// window offsets 32 at a time over a 64-sample register block, so every
// squared difference is computed from registers.
//
// Selection keeps the M = group_max - 1 smallest keys of a median-of-three
// insertion network, where a key is a candidate's score in the high bits and
// its window offset (0..255, increasing with lin) in the low 8 bits:
//  * count mode with counts <= 255 (k_match_1d_u8): the score is exact and
//    below 2^23 in magnitude, so key = score * 256 + offset orders by
//    (score, lin) exactly and the network's first K-1 keys are the members
//    in output order.  Patch products use byte dot products (4 counts per
//    instruction) on the staged counts.
//  * float modes (k_match_1d_f): key = the score's order-preserving bits with
//    the low 8 mantissa bits replaced by the offset, which orders by the
//    score truncated to 15 mantissa bits, then lin.  The K-1 members and the
//    next candidate are re-scored in FP32 and sorted by (score, lin); a
//    truncation tie at the group boundary or an FP32 near-tie sends the
//    reference to FP64 re-scoring of the recorded candidates.
//  * count mode with larger counts (k_match_1d_rec): the two-pass scheme
//    (values in the network, candidates up to the running M-th value
//    recorded, members rescanned from the record).
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

__device__ __forceinline__ int p2floor(int x) { return x <= 1 ? 1 : (1 << (31 - __clz(x))); }

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// group size from the accepted count (power of two in [gmin, gmax], at most
// the candidates plus the reference)
__device__ __forceinline__ int group_size_of(const MatchArgs& a, int acc, int ncand)
{
    int k = p2floor(min(1 + acc, a.gmax));
    k = max(k, a.gmin);
    return min(k, p2floor(1 + ncand));
}

// median of three (one VALU instruction)
__device__ __forceinline__ int med3(int a, int b, int c)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// FP64 score of a float-mode candidate (re-scored near-ties): separately
// rounded products and sums (no contraction), so the value is the plain
// FP64 sum in patch order
template <int MODE>
__device__ __forceinline__ double score64_lds(const MatchArgs& a, const float* rp, const int* sx,
                                              int c)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kJ; ++i) {
        const double d = __dsub_rn(double(__int_as_float(sx[c + i])), double(rp[i]));
        s = __dadd_rn(s, __dmul_rn(d, d));
    }
    if constexpr (MODE == kGauss) s = __dsub_rn(s, a.bias_d);
    return s;
}

// Count mode, any counts: two passes.  Pass 1 counts the accepted candidates
// and keeps the M smallest exact scores; every candidate whose score does
// not exceed the running M-th value is recorded (offset index, in lin
// order).  The members are exactly the recorded candidates below the K-1-th
// value and the first ties at it, so pass 2 rescans only the record.
// only_marked: just the references that k_match_1d_u8 left (count 0).
template <int GM>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2)))
void k_match_1d_rec(MatchArgs a, int cap_span, int kmax, int only_marked)
{
    constexpr int M = GM > 1 ? GM - 1 : 1;
    extern __shared__ __align__(16) int sx[];   // staged counts
    __shared__ int sel_s[M][kWave];
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

    bool pending = have && (!only_marked || a.count[t] == 0);
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
                // non-finite or out-of-range counts are flagged (and scored as 0)
                const float rk = rintf(src[pos] * inv_sp);
                const bool ok = rk >= 0.f && rk <= float(kmax);
                if (!ok) atomicOr(a.range_flag, 1);
                v = ok ? int(rk) : 0;
            }
            sx[i] = v;
        }
        __syncthreads();

        if (mine) {
            const int rl = r - base;  // reference start in the stage
            int rp[kJ];
            int sr = 0;
#pragma unroll
            for (int i = 0; i < kJ; ++i) {
                rp[i] = sx[rl + i];
                sr += rp[i];
            }
            const int dlo = max(wlo, -r), dhi = min(whi, ell - r);
            const int ncand = dhi - dlo;  // window size minus the reference
            int s[M];
#pragma unroll
            for (int m = 0; m < M; ++m) s[m] = INT_MAX;
            int acc = 0, nrec = 0;
            // the SSD of integer counts is evaluated exactly as sum p^2 +
            // sum q^2 - 2 sum pq (wrapping uint32 arithmetic; the result is
            // below 2^31), with sliding sums over the candidate
            unsigned sp2 = 0;
#pragma unroll
            for (int i = 0; i < kJ; ++i) sp2 += unsigned(__mul24(rp[i], rp[i]));
            for (int d0 = wlo; d0 <= whi; d0 += kJ) {
                int buf[2 * kJ];
#pragma unroll
                for (int i = 0; i < 2 * kJ; ++i) buf[i] = sx[rl + d0 + i];
                int sc = 0;
                unsigned sq2 = 0;
#pragma unroll
                for (int i = 0; i < kJ; ++i) {
                    sc += buf[i];
                    sq2 += unsigned(__mul24(buf[i], buf[i]));
                }
#pragma unroll
                for (int u = 0; u < kJ; ++u) {
                    const int d = d0 + u;
                    unsigned spq = 0;
#pragma unroll
                    for (int i = 0; i < kJ; ++i) spq += unsigned(__mul24(buf[u + i], rp[i]));
                    int x = int(sp2 + sq2 - 2u * spq) - a.gamma_i * (sr + sc);
                    sq2 += unsigned(__mul24(buf[u + kJ], buf[u + kJ]) - __mul24(buf[u], buf[u]));
                    sc += buf[u + kJ] - buf[u];
                    // offsets outside the clipped window and the reference
                    // itself score as the largest value (never counted, never
                    // selected)
                    const bool valid = d >= dlo && d <= dhi && d != 0;
                    x = valid ? x : INT_MAX;
                    acc += x < a.tau_i;
                    if (valid && x <= s[M - 1]) {
                        if (nrec < kRec) rec[nrec][lane] = (unsigned char)(d - wlo);
                        ++nrec;
                    }
                    // insertion into the sorted M smallest: slot m takes the
                    // median of (s[m-1], x, s[m]) since s[m-1] <= s[m]
#pragma unroll
                    for (int m = M - 1; m >= 1; --m) s[m] = med3(s[m - 1], x, s[m]);
                    s[0] = min(s[0], x);
                }
            }

            int K = group_size_of(a, acc, ncand);
            const int need = GM > 1 ? K - 1 : 0;
            int* out = a.match + t * a.gmax;
            out[0] = r;
            for (int m = 1; m < a.gmax; ++m) out[m] = -1;
            if (need == 0) a.count[t] = K;
            if (need > 0) {
                int theta = s[0];
#pragma unroll
                for (int m = 0; m < M; ++m)
                    if (m == need - 1) theta = s[m];
                // the members below theta and the first ties at theta, in lin
                // order; then sorted by (score, lin)
                int n_less = 0;
#pragma unroll
                for (int m = 0; m < M; ++m) n_less += (m < need && s[m] < theta) ? 1 : 0;
                int eq_left = need - n_less;
                int got = 0;
                auto consider = [&](int d) {
                    int x = 0, sc2 = 0;
#pragma unroll
                    for (int i = 0; i < kJ; ++i) {
                        const int q = sx[rl + d + i];
                        x += __mul24(q - rp[i], q - rp[i]);
                        sc2 += q;
                    }
                    x -= a.gamma_i * (sr + sc2);
                    bool take = x < theta;
                    if (!take && x == theta && eq_left > 0) {
                        take = true;
                        --eq_left;
                    }
                    if (take) {
                        sel_s[got][lane] = x;
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
                    const int ks = sel_s[m][lane];
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
                if (got < need) K = p2floor(1 + got);
                a.count[t] = K;
                for (int m = 0; m < K - 1; ++m) out[1 + m] = sel_l[m][lane];
            }
        }
        pending = pending && !mine;
        __syncthreads();
    }
}

// Count mode, counts <= 255: one lane per reference, exact integer scores
//   SSD - gamma (sum p + sum q) = sum p^2 - gamma sum p + sum q^2 - gamma sum q - 2 sum pq
// with sum pq from byte dot products and the candidate terms slid along the
// window.  Waves whose staged counts exceed 255 mark their references with
// count 0 for k_match_1d_rec.
template <int GM>
__global__ __launch_bounds__(kWave) void k_match_1d_u8(MatchArgs a, int cap_span, int kmax)
{
    constexpr int M = GM > 1 ? GM - 1 : 1;
    extern __shared__ __align__(16) unsigned sw[];  // staged counts, 4 per word

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
    const int gam = a.gamma_i;
    // words staged: the last block reads 18 words from its first sample
    const int nw = (cap_span + W + 2 * kJ + 8 + 3) / 4;

    bool pending = have;
    while (__any(pending)) {
        const int r0 = __shfl(r, __ffsll(__ballot(pending)) - 1);
        const bool mine = pending && r >= r0 && (r - r0) <= cap_span;
        const int base = r0 + wlo;
        int vmax = 0;
        for (int k = lane; k < nw; k += kWave) {
            unsigned word = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int pos = base + 4 * k + e;
                int v = 0;
                if (pos >= 0 && pos < L) {
                    const float rk = rintf(src[pos] * inv_sp);
                    const bool ok = rk >= 0.f && rk <= float(kmax);
                    if (!ok) atomicOr(a.range_flag, 1);
                    v = ok ? int(rk) : 0;
                }
                vmax = max(vmax, v);
                word |= unsigned(min(v, 255)) << (8 * e);
            }
            sw[k] = word;
        }
        vmax = wave_max_i(vmax);
        __syncthreads();

        if (vmax > 255) {
            if (mine) a.count[t] = 0;
        } else if (mine) {
            const int rl = r - base;  // reference start in the stage (>= -wlo)
            unsigned rw[8];           // reference counts, 4 per word
            {
                const int w0 = rl >> 2, sh = rl & 3;
                unsigned A[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) A[k] = sw[w0 + k];
#pragma unroll
                for (int j = 0; j < 8; ++j) rw[j] = __builtin_amdgcn_alignbyte(A[j + 1], A[j], sh);
            }
            unsigned sp2 = 0, sr = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sp2 = __builtin_amdgcn_udot4(rw[j], rw[j], sp2, false);
                sr = __builtin_amdgcn_udot4(rw[j], 0x01010101u, sr, false);
            }
            const int c0 = int(sp2) - gam * int(sr);
            const int dlo = max(wlo, -r), dhi = min(whi, ell - r);
            const int ncand = dhi - dlo;

            int s[M];
#pragma unroll
            for (int m = 0; m < M; ++m) s[m] = INT_MAX;

            for (int d0 = wlo; d0 <= whi; d0 += kJ) {
                // bytes st .. st + 71 of the stage; B[s][k] holds the four
                // counts from st + s + 4k
                const int st = rl + d0;
                unsigned B[4][16];
                unsigned b16;
                {
                    const int w0 = st >> 2, sh = st & 3;
                    unsigned A[18];
#pragma unroll
                    for (int k = 0; k < 18; ++k) A[k] = sw[w0 + k];
#pragma unroll
                    for (int k = 0; k < 16; ++k) B[0][k] = __builtin_amdgcn_alignbyte(A[k + 1], A[k], sh);
                    b16 = __builtin_amdgcn_alignbyte(A[17], A[16], sh);
                }
#pragma unroll
                for (int sft = 1; sft < 4; ++sft) {
#pragma unroll
                    for (int k = 0; k < 15; ++k)
                        B[sft][k] = __builtin_amdgcn_alignbyte(B[0][k + 1], B[0][k], sft);
                    B[sft][15] = __builtin_amdgcn_alignbyte(b16, B[0][15], sft);
                }
                // candidate terms of offset d0: sum q^2 - gamma sum q
                int q;
                {
                    unsigned sq2 = 0, sq = 0;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        sq2 = __builtin_amdgcn_udot4(B[0][j], B[0][j], sq2, false);
                        sq = __builtin_amdgcn_udot4(B[0][j], 0x01010101u, sq, false);
                    }
                    q = int(sq2) - gam * int(sq);
                }
                // valid offsets of this block: inside the clipped window, not
                // the reference itself
                const int lo = max(dlo - d0, 0), hi = min(dhi - d0, kJ - 1);
                unsigned vm = lo > hi ? 0u : ((0xFFFFFFFFu >> (kJ - 1 - hi)) & (0xFFFFFFFFu << lo));
                if (d0 <= 0 && 0 < d0 + kJ) vm &= ~(1u << (-d0));
                const bool full = __ballot(vm != 0xFFFFFFFFu) == 0;
                const int idx0 = d0 - wlo;
                auto block = [&](auto check) {
#pragma unroll
                    for (int u = 0; u < kJ; ++u) {
                        const int sft = u & 3, a4 = u >> 2;
                        // two independent dot-product chains
                        unsigned p0 = 0, p1 = 0;
#pragma unroll
                        for (int j = 0; j < 8; j += 2) {
                            p0 = __builtin_amdgcn_udot4(B[sft][a4 + j], rw[j], p0, false);
                            p1 = __builtin_amdgcn_udot4(B[sft][a4 + j + 1], rw[j + 1], p1, false);
                        }
                        const int x = c0 + q - 2 * int(p0 + p1);
                        // slide to offset d0 + u + 1: drop count u, add count u + 32
                        const int e0 = int(B[sft][a4] & 255u), e1 = int(B[sft][a4 + 8] & 255u);
                        q += __mul24(e1 - e0, e1 + e0 - gam);
                        int key = __mul24(x, 256) + (idx0 + u);
                        if constexpr (decltype(check)::value) key = (vm >> u) & 1u ? key : INT_MAX;
#pragma unroll
                        for (int m = M - 1; m >= 1; --m) s[m] = med3(s[m - 1], key, s[m]);
                        s[0] = min(s[0], key);
                    }
                };
                if (full) block(std::false_type{});
                else block(std::true_type{});
            }

            // accepted candidates among the M smallest keys (the group size
            // saturates at group_max = M + 1): key < tau * 256 iff score < tau
            int acc = 0;
            const long long tk = (long long)a.tau_i * 256;
#pragma unroll
            for (int m = 0; m < M; ++m) acc += (s[m] != INT_MAX && (long long)s[m] < tk) ? 1 : 0;
            int K = group_size_of(a, acc, ncand);
            if (GM == 1) K = 1;
            int got = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) got += (m < K - 1 && s[m] != INT_MAX) ? 1 : 0;
            if (got < K - 1) K = p2floor(1 + got);
            int* out = a.match + t * a.gmax;
            out[0] = r;
#pragma unroll
            for (int m = 1; m < GM; ++m) out[m] = m < K ? r + wlo + (s[m - 1] & 255) : -1;
            a.count[t] = K;
        }
        pending = pending && !mine;
        __syncthreads();
    }
}

// order-preserving int image of a float and back
__device__ __forceinline__ int ord_of(float x)
{
    const int b = __float_as_int(x);
    return b >= 0 ? b : b ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float float_of_ord(int m) { return __int_as_float(m >= 0 ? m : m ^ 0x7FFFFFFF); }

// Float modes (plain SSD of the pilot, Gaussian bias): one lane per
// reference, keys of truncated scores, FP32 re-scoring of the K-1 members and
// the next candidate, FP64 re-scoring of near-ties.
//
// SHARE (references 4 samples apart): a window of 32 samples is 8 blocks of
// 4, and block k of the reference of lane l is block 0 of lane l + k.  Each
// lane squares the differences of its first block only, and the window sum
// b0 + (b1 + (b2 + ... + (b6 + b7))) is folded from the next lanes by seven
// adds of the value one lane up (DPP wave shift); the per-lane re-scoring
// nests its sum the same way, so a member's re-scored value equals its key's
// value bit for bit.  The last 7 lanes of a wavefront only supply blocks (57
// references per wavefront).  A wavefront whose references are not 4 apart
// scores them one lane each.
constexpr int kShareBlk = 4;
constexpr int kShareRefs = kWave - kJ / kShareBlk + 1;

// the value of lane + 1 (0 in the last lane): DPP wave shift left by one
__device__ __forceinline__ float from_next_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

template <int MODE, int GM, bool SHARE>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3)))
void k_match_1d_f(MatchArgs a, int cap_span)
{
    constexpr int M = GM > 1 ? GM - 1 : 1;
    constexpr int NS = M + 1;  // the M smallest keys and the next one
    extern __shared__ __align__(16) int sx[];  // staged samples (float bits)
    __shared__ unsigned char rec[kRec][kWave];

    const Geo& g = a.g;
    const int L = g.L[kAx - 1];
    const int W = g.W[kAx - 1];
    const int ell = L - kJ;
    const int wlo = -(W / 2), whi = W - 1 - W / 2;
    constexpr int rpw = SHARE ? kShareRefs : kWave;  // references per wavefront
    const int nchunk = (a.n_refs + rpw - 1) / rpw;
    const int b = blockIdx.x / nchunk;
    const int chunk = blockIdx.x - b * nchunk;
    const int lane = threadIdx.x;
    const int gi = chunk * rpw + lane;
    const bool have = lane < rpw && gi < a.n_refs;
    int r = have ? safe_origin(int(a.refs[gi]), last_origin(g)) : 0;
    const float* src = a.src + long(b) * g.V;
    const long t = long(b) * a.n_refs + gi;
    // shared blocks: every reference of the wavefront 4 after the previous;
    // lanes without one take the next positions of that run (their samples
    // lie inside the staged span, which covers 64 lanes)
    bool share = false;
    if constexpr (SHARE) {
        const int rf = __shfl(r, 0);
        share = __all(!have || r == rf + kShareBlk * lane);
        if (share) r = rf + kShareBlk * lane;
    }

    bool pending = have || share;
    while (__any(pending)) {
        const int r0 = __shfl(r, __ffsll(__ballot(pending)) - 1);
        const bool mine = pending && r >= r0 && (r - r0) <= cap_span;
        const int base = r0 + wlo;
        const int len = cap_span + W + 2 * kJ;
        // positions outside the array are staged as NaN: a candidate reaching
        // them scores NaN and fails the finiteness test, so the shared paths
        // need no window bounds per candidate (a reference's sum only reads
        // its candidate's samples)
        for (int i = lane; i < len; i += kWave) {
            const int pos = base + i;
            sx[i] = (pos >= 0 && pos < L) ? __float_as_int(src[pos]) : 0x7FC00000;
        }
        __syncthreads();

        if (mine) {
            const int rl = r - base;
            float rp[kJ];
#pragma unroll
            for (int i = 0; i < kJ; ++i) rp[i] = __int_as_float(sx[rl + i]);
            const int dlo = max(wlo, -r), dhi = min(whi, ell - r);
            const int ncand = dhi - dlo;
            int s[NS];
#pragma unroll
            for (int m = 0; m < NS; ++m) s[m] = INT_MAX;
            // INT_MAX held in a scalar register: the key select takes it as
            // an operand instead of building the constant per candidate
            int kEmpty;
            asm volatile("s_mov_b32 %0, 0x7fffffff" : "=s"(kEmpty));
            int acc = 0, nrec = 0, namb = 0;
            // FP32 round-off band around a value (relative to the score's
            // terms; the Gaussian bias is one of them)
            const float bmag = MODE == kGauss ? fabsf(a.bias) : 0.f;
            const float band = float(kTieBand);
            const float tau_band = band * (fabsf(a.tau_f) + bmag);
            // the band around tau is [tau_lo, tau_hi]: below it a score is
            // accepted, above it rejected, inside it decided in FP64
            const float tau_lo = a.tau_f - tau_band, tau_hi = a.tau_f + tau_band;
            auto score = [&](int c) {
                float x = 0.f;
                if (SHARE && share) {
                    float bs[kJ / kShareBlk];
#pragma unroll
                    for (int k = 0; k < kJ / kShareBlk; ++k) {
                        float bk = 0.f;
#pragma unroll
                        for (int i = 0; i < kShareBlk; ++i) {
                            const float df = __int_as_float(sx[c + kShareBlk * k + i]) - rp[kShareBlk * k + i];
                            bk = __builtin_fmaf(df, df, bk);
                        }
                        bs[k] = bk;
                    }
                    x = bs[kJ / kShareBlk - 1];
#pragma unroll
                    for (int k = kJ / kShareBlk - 2; k >= 0; --k) x = bs[k] + x;
                } else {
#pragma unroll
                    for (int i = 0; i < kJ; ++i) {
                        const float df = __int_as_float(sx[c + i]) - rp[i];
                        x = __builtin_fmaf(df, df, x);
                    }
                }
                if constexpr (MODE == kGauss) x -= a.bias;
                return x;
            };
            // one candidate: counts, record, insertion network
            auto take = [&](int d, float x, int rec_key) __attribute__((always_inline)) {
                const bool valid = d != 0 && fabsf(x) <= FLT_MAX;
                // plain SSD scores are never negative: their order is that of
                // their bit patterns (the same key, fewer instructions)
                const int ord = MODE == kPlain ? __float_as_int(x) : ord_of(x);
                // acc: certain acceptances; namb (less acc at the end): up to
                // the band's top
                acc += (valid && x < tau_lo) ? 1 : 0;
                namb += (valid && x <= tau_hi) ? 1 : 0;
                const int key = valid ? ((ord & ~255) | (d - wlo)) : kEmpty;
                if (key <= rec_key) {
                    if (nrec < kRec) rec[nrec][lane] = (unsigned char)(d - wlo);
                    ++nrec;
                }
#pragma unroll
                for (int m = NS - 1; m >= 1; --m) s[m] = med3(s[m - 1], key, s[m]);
                s[0] = min(s[0], key);
            };
            // candidates within the band of the running M-th value are
            // recorded (the value at the start of a run of offsets bounds
            // the later ones)
            auto record_bound = [&]() __attribute__((always_inline)) {
                int rk = INT_MAX - 1;
                if (s[M - 1] != INT_MAX) {
                    const float ub = float_of_ord(s[M - 1] | 255);
                    const float lim = ub + band * (fabsf(ub) + bmag);
                    if (fabsf(lim) <= FLT_MAX) rk = ord_of(lim) | 255;
                }
                return rk;
            };
            if (SHARE && share) {
                constexpr int kRun = 8;  // offsets per pass (kept short: code size)
                for (int d0 = wlo; d0 <= whi; d0 += kRun) {
                    float buf[kRun + kShareBlk];
#pragma unroll
                    for (int i = 0; i < kRun + kShareBlk; ++i) buf[i] = __int_as_float(sx[rl + d0 + i]);
                    const int rec_key = record_bound();
                    // this lane's block of every offset of the run, then the
                    // window sums over the blocks of the next lanes (the
                    // run's folds interleave, so no fold waits on its own
                    // previous step)
                    float blk[kRun], x[kRun];
#pragma unroll
                    for (int u = 0; u < kRun; ++u) {
                        float b = 0.f;
#pragma unroll
                        for (int i = 0; i < kShareBlk; ++i) {
                            const float df = buf[u + i] - rp[i];
                            b = __builtin_fmaf(df, df, b);
                        }
                        blk[u] = x[u] = b;
                    }
#pragma unroll
                    for (int k = 1; k < kJ / kShareBlk; ++k)
#pragma unroll
                        for (int u = 0; u < kRun; ++u) x[u] = blk[u] + from_next_lane(x[u]);
#pragma unroll
                    for (int u = 0; u < kRun; ++u) {
                        float xu = x[u];
                        if constexpr (MODE == kGauss) xu -= a.bias;
                        take(d0 + u, xu, rec_key);
                    }
                }
            } else if (SHARE) {
                // references not 4 apart: one candidate at a time
                int rec_key = INT_MAX - 1;
                for (int d = wlo; d <= whi; ++d) {
                    if (((d - wlo) & (kJ - 1)) == 0) rec_key = record_bound();
                    take(d, score(rl + d), rec_key);
                }
            } else
            for (int d0 = wlo; d0 <= whi; d0 += kJ) {
                float buf[2 * kJ];
#pragma unroll
                for (int i = 0; i < 2 * kJ; ++i) buf[i] = __int_as_float(sx[rl + d0 + i]);
                // candidates within the band of the running M-th value are
                // recorded (the block-start value bounds the later ones)
                int rec_key = INT_MAX - 1;
                if (s[M - 1] != INT_MAX) {
                    const float ub = float_of_ord(s[M - 1] | 255);
                    const float lim = ub + band * (fabsf(ub) + bmag);
                    if (fabsf(lim) <= FLT_MAX) rec_key = ord_of(lim) | 255;
                }
#pragma unroll
                for (int u = 0; u < kJ; ++u) {
                    const int d = d0 + u;
                    float x = 0.f;
#pragma unroll
                    for (int i = 0; i < kJ; ++i) {
                        const float df = buf[u + i] - rp[i];
                        x = __builtin_fmaf(df, df, x);
                    }
                    if constexpr (MODE == kGauss) x -= a.bias;
                    // offsets outside the clipped window, the reference itself
                    // and non-finite scores are never counted or selected
                    const bool valid = d >= dlo && d <= dhi && d != 0 && fabsf(x) <= FLT_MAX;
                    acc += (valid && x < tau_lo) ? 1 : 0;
                    namb += (valid && x <= tau_hi) ? 1 : 0;
                    const int key = valid ? ((ord_of(x) & ~255) | (d - wlo)) : INT_MAX;
                    if (key <= rec_key) {
                        if (nrec < kRec) rec[nrec][lane] = (unsigned char)(d - wlo);
                        ++nrec;
                    }
#pragma unroll
                    for (int m = NS - 1; m >= 1; --m) s[m] = med3(s[m - 1], key, s[m]);
                    s[0] = min(s[0], key);
                }
            }

            // lanes that only supplied blocks stop here (their window sums
            // are partial, and a wavefront pays for any lane's fallback work)
            if (have) {
            int K = group_size_of(a, acc, ncand);
            // scores within the band of tau are accepted or not in FP64, when
            // that can change the group size
            namb -= acc;
            if (namb > 0 && group_size_of(a, acc + namb, ncand) != K) {
                acc = 0;
                for (int d = dlo; d <= dhi; ++d) {
                    if (d == 0) continue;
                    const float x = score(rl + d);
                    if (!(fabsf(x) <= FLT_MAX)) continue;
                    if (x >= tau_lo && x <= tau_hi)
                        acc += score64_lds<MODE>(a, rp, sx, rl + d) < a.tau_d ? 1 : 0;
                    else
                        acc += x < a.tau_f ? 1 : 0;
                }
                K = group_size_of(a, acc, ncand);
            }
            if (GM == 1) K = 1;
            const int need = K - 1;
            // members: the first `need` keys, re-scored in FP32; the next key
            float ms[M];
            int ml[M];
            int got = 0, kb = INT_MAX, kn = INT_MAX;
            float xb = 0.f;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const bool in = m < need && s[m] != INT_MAX;
                ms[m] = INFINITY;
                ml[m] = 0;
                if (in) {
                    const int d = (s[m] & 255) + wlo;
                    ms[m] = score(rl + d);
                    ml[m] = r + d;
                    ++got;
                }
                if (m == need - 1) {
                    kb = s[m];
                    xb = ms[m];
                }
            }
#pragma unroll
            for (int m = 0; m < NS; ++m)
                if (m == need) kn = s[m];
            bool amb = false;
            float xn = INFINITY;
            if (need > 0 && got == need && kn != INT_MAX) {
                xn = score(rl + (kn & 255) + wlo);
                // the boundary is a truncation tie: the member set is open
                amb = (kn >> 8) == (kb >> 8) && !(xb == 0.f && xn == 0.f && (kb >> 8) == 0);
            }
            // (score, lin) order of the members
#pragma unroll
            for (int i = 1; i < M; ++i)
#pragma unroll
                for (int j = i; j >= 1; --j) {
                    const bool sw_ = ms[j - 1] > ms[j] || (ms[j - 1] == ms[j] && ml[j - 1] > ml[j]);
                    const float tx = ms[j - 1];
                    const int tl = ml[j - 1];
                    ms[j - 1] = sw_ ? ms[j] : tx;
                    ml[j - 1] = sw_ ? ml[j] : tl;
                    ms[j] = sw_ ? tx : ms[j];
                    ml[j] = sw_ ? tl : ml[j];
                }
            // The FP32 ranking equals the FP64 one unless the value after the
            // K-th, or two neighbours in the list, lie within the round-off
            // band (equal zeros are exact).
            auto near = [&](float lo, float hi) {
                return hi - lo <= band * (fabsf(hi) + bmag) && !(lo == 0.f && hi == 0.f);
            };
            float theta = 0.f;
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m == got - 1) theta = ms[m];
            if (need > 0 && got == need && kn != INT_MAX) amb = amb || near(theta, xn);
#pragma unroll
            for (int m = 1; m < M; ++m) amb = amb || (m < got && near(ms[m - 1], ms[m]));
            if (amb) {
                // every candidate up to theta plus the band is re-scored in
                // FP64; the best are kept by (FP64 score, lin): candidates
                // arrive in lin order and a later one passes an equal score
                // only when strictly smaller
                const float thr = theta + band * (fabsf(theta) + bmag);
                double bx[M];
                int bl[M];
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    bx[m] = INFINITY;
                    bl[m] = 0;
                }
                auto consider = [&](int d) {
                    const float x = score(rl + d);
                    if (!(x <= thr)) return;
                    const double xd = score64_lds<MODE>(a, rp, sx, rl + d);
                    if (!(xd == xd)) return;
                    const int ld = r + d;
#pragma unroll
                    for (int m = M - 1; m >= 1; --m) {
                        const bool shift = bx[m - 1] > xd;
                        const bool place = !shift && bx[m] > xd;
                        bx[m] = shift ? bx[m - 1] : (place ? xd : bx[m]);
                        bl[m] = shift ? bl[m - 1] : (place ? ld : bl[m]);
                    }
                    if (bx[0] > xd) {
                        bx[0] = xd;
                        bl[0] = ld;
                    }
                };
                if (nrec <= kRec) {
                    for (int k = 0; k < nrec; ++k) consider(int(rec[k][lane]) + wlo);
                } else {
                    for (int d = dlo; d <= dhi; ++d)
                        if (d != 0) consider(d);
                }
                got = 0;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    got += (m < need && bx[m] < INFINITY) ? 1 : 0;
                    ml[m] = bl[m];
                }
            }
            // non-finite scores select fewer members than asked: the group is
            // cut to the largest power of two they fill
            if (got < need) K = p2floor(1 + got);
            int* out = a.match + t * a.gmax;
            out[0] = r;
#pragma unroll
            for (int m = 1; m < GM; ++m) out[m] = m < K ? ml[m - 1] : -1;
            a.count[t] = K;
            }
        }
        pending = pending && !mine;
        __syncthreads();
    }
}

template <int GM>
hipError_t launch_1d_gm(const MatchArgs& a, int mode, int cap_span, int kmax, int step,
                        hipStream_t s)
{
    const int nchunk = (a.n_refs + kWave - 1) / kWave;
    const dim3 grid(unsigned(long(nchunk) * a.g.batch));
    const int W = a.g.W[kAx - 1];
    const size_t lds = sizeof(int) * size_t(cap_span + W + 2 * kJ);
    if (mode != kCount) {
        // shared blocks when the references are 4 apart (the staged span of
        // 64 steps covers the helper lanes)
        const bool share = step == kShareBlk;
        const int ns = (a.n_refs + kShareRefs - 1) / kShareRefs;
        const dim3 grid_s(unsigned(long(ns) * a.g.batch));
        if (mode == kGauss) {
            if (share)
                hipLaunchKernelGGL((k_match_1d_f<kGauss, GM, true>), grid_s, dim3(kWave), lds, s, a,
                                   cap_span);
            else
                hipLaunchKernelGGL((k_match_1d_f<kGauss, GM, false>), grid, dim3(kWave), lds, s, a,
                                   cap_span);
        } else if (share) {
            hipLaunchKernelGGL((k_match_1d_f<kPlain, GM, true>), grid_s, dim3(kWave), lds, s, a,
                               cap_span);
        } else {
            hipLaunchKernelGGL((k_match_1d_f<kPlain, GM, false>), grid, dim3(kWave), lds, s, a,
                               cap_span);
        }
        return hipGetLastError();
    }
    // byte counts first (scores below 2^23 in magnitude need gamma <= 256);
    // the record kernel takes the references of waves with larger counts
    int only_marked = 0;
    if (a.gamma_i >= 0 && a.gamma_i <= 256) {
        const size_t lds_u8 = sizeof(unsigned) * size_t((cap_span + W + 2 * kJ + 8 + 3) / 4);
        hipLaunchKernelGGL((k_match_1d_u8<GM>), grid, dim3(kWave), lds_u8, s, a, cap_span, kmax);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        only_marked = 1;
    }
    hipLaunchKernelGGL((k_match_1d_rec<GM>), grid, dim3(kWave), lds, s, a, cap_span, kmax,
                       only_marked);
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
    switch (a.gmax) {
    case 1: return launch_1d_gm<1>(a, mode, cap_span, kmax, step, s);
    case 2: return launch_1d_gm<2>(a, mode, cap_span, kmax, step, s);
    case 4: return launch_1d_gm<4>(a, mode, cap_span, kmax, step, s);
    case 8: return launch_1d_gm<8>(a, mode, cap_span, kmax, step, s);
    case 16: return launch_1d_gm<16>(a, mode, cap_span, kmax, step, s);
    default: return launch_1d_gm<32>(a, mode, cap_span, kmax, step, s);
    }
}

}  // namespace bmnd
