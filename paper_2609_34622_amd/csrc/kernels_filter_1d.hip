// Collaborative filtering of 32-sample patches on the matrix cores
// (section Collaborative Filtering, 3-D transform of a group).
//
// A group of K <= 16 members is the 16 x 32 matrix X (rows: members, zero
// rows past K).  Its 3-D transform is
//     Y = H (X T^T)        (spatial transform T per member, Haar H over members)
// and the synthesis is  X^ = (H^T C) U^T.  The variance of every coefficient
// is (H o H) (M (T o T)^T) for the per-sample variance map M.  One wavefront
// filters one group:
//   * The spatial products (X T^T, M (T o T)^T and the synthesis' Z U^T)
//     run as split half-precision products on v_mfma_f32_16x16x32_f16 (see
//     below).  Operand layout: A, lane l: row l%16, depth 8(l/16)..+7;
//     B, lane l: depth 8(l/16)..+7, column l%16; result, lane l, register r:
//     row 4(l/16)+r, column l%16.  The spatial depth (sample index i) is
//     i = 8(l/16) + s, so each lane gathers eight contiguous samples of one
//     member.
//   * A result holds member 4(l/16)+r in register r, so the Haar transform
//     over the members runs in registers: the first two levels inside a
//     lane, the last two between lane groups (permlane swaps).
//   * The synthesis contracts over the members' samples, so H^T C goes
//     through a 16 x 32 LDS buffer once (write by rows, read by rows of the
//     transpose).
// Shrinkage, risk surrogates, weights and the aggregation work on the
// result layout (8 coefficients per lane).  Hard-threshold decisions within
// the FP32 error band of the threshold are recomputed in FP64 from the
// input samples, as in the generic filter.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bmnd_internal.h"
#include "filter_common.h"

namespace bmnd {

namespace {

constexpr int kWave = 64;
constexpr int kJ = 32;        // patch length
constexpr int kWaves = 4;     // wavefronts per workgroup
constexpr int kSubMax = 48;   // references per wavefront with a staged pilot, at most
constexpr int kTargetWaves = 16384;  // enough wavefronts to fill the device
constexpr int kZs = 36;       // row stride (floats) of the transpose buffer
constexpr float kRsqrt2 = 0.70710678118654752440f;

typedef float f4 __attribute__((ext_vector_type(4)));

// Orders the LDS accesses of one wavefront.
__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// 2^(-e/2) rounded once from 1/sqrt(2)
__device__ __forceinline__ float pow_rsqrt2(int e)
{
    const float v = ldexpf(1.f, -(e >> 1));
    return (e & 1) ? v * kRsqrt2 : v;
}

// ---- Haar transform over the members, in registers.  Member m = 4 lg + r
// of a group is register r of lane group lg (lanes 16 lg .. 16 lg + 15), so
// the first two levels pair registers of one lane and the last two pair lane
// groups (v_permlane16_swap, v_permlane32_swap).  Butterflies are
// unnormalised and in place: the sum of a block stays at its first member,
// the detail of a block at the first member of its second half, so the
// detail row of level t (support 2^t) of block b sits at position
// b 2^t + 2^(t - 1) and the scaling row at position 0.  The orthonormal
// coefficient at position p is the butterfly value times 2^(-t/2) (t the
// level of p; lk for position 0), the same factor that H^T needs before the
// inverse butterflies.

// (value at the even lane group, value at the odd one) of the lane-group
// pair (0, 1) or (2, 3) this lane belongs to
// (the swap overwrites both of its operands: an opaque second copy lets the
// value itself be the other one, one register move instead of two)
__device__ __forceinline__ void pair16(float v, float& a, float& b)
{
    float w = v;
    asm("" : "+v"(w));
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(w), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// (value at lane group 0 or 1, value at lane group 2 or 3) of the pair
// (0, 2) or (1, 3) this lane belongs to
__device__ __forceinline__ void pair32(float v, float& a, float& b)
{
    float w = v;
    asm("" : "+v"(w));
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(w), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// One butterfly of the last two levels on register 0: the first block of
// the pair takes a + b, the second a - b (s = +1 or -1 per lane group).
// The forward and inverse transforms both use these levels (the butterfly
// is its own inverse up to the factor 2).
__device__ __forceinline__ float level3(float v, float s3)
{
    float a, b;
    pair16(v, a, b);
    return __builtin_fmaf(s3, b, a);
}

// Level 4 as cA a + sB b: lane groups 0 and 2 take a +- b; 1 and 3 keep
// their own value, which is a in lane group 1 and b in 3 (cA = 1, sB = 0
// and cA = 0, sB = 1), so the value before the swap is not needed after it
__device__ __forceinline__ float level4(float v, float sB, float cA)
{
    float a, b;
    pair32(v, a, b);
    return __builtin_fmaf(sB, b, a * cA);
}

// Forward butterflies over all 16 member slots.  Slots past K hold zeros,
// and a level that pairs a block with an all-zero block leaves the valid
// positions unchanged, so the four levels serve every K = 2^lk; only the
// normalisation of position 0 depends on K.
__device__ __forceinline__ f4 haar_fwd(f4 v, float s3, float sB, float cA)
{
    const float a0 = v[0] + v[1], a1 = v[0] - v[1];
    const float a2 = v[2] + v[3], a3 = v[2] - v[3];
    const float b0 = a0 + a2, b2 = a0 - a2;
    return f4{level4(level3(b0, s3), sB, cA), a1, b2, a3};
}

// the squared Haar rows on non-negative values: every row keeps the sum of
// its support (the detail positions included)
__device__ __forceinline__ f4 haar_fwd_sq(f4 v, float sBq, float cA)
{
    const float a0 = v[0] + v[1], a2 = v[2] + v[3];
    const float b0 = a0 + a2;
    return f4{level4(level3(b0, 1.f), sBq, cA), a0, b0, a2};
}

// inverse butterflies (levels in the reverse order); positions past K must
// hold zeros
__device__ __forceinline__ f4 haar_inv(f4 v, float s3, float sB, float cA)
{
    const float c0 = level3(level4(v[0], sB, cA), s3);
    const float b0 = c0 + v[2], b2 = c0 - v[2];
    return f4{b0 + v[1], b0 - v[1], b2 + v[3], b2 - v[3]};
}

// normalisation 2^(-t/2) of position 4 lg (register 0) for 2^lk members
__device__ __forceinline__ float haar_norm0(int lg, int lk)
{
    return (lg & 1) ? 0.35355339059327376f : (lg == 2 ? 0.25f : pow_rsqrt2(lk));
}

// standard Haar row (scaling, then detail rows with support K, K/2, ..., 2)
// held at position p
__device__ __forceinline__ int haar_row_of(int p, int lk)
{
    if (p == 0) return 0;
    const int t = __ffs(p);  // level: p = b 2^t + 2^(t - 1)
    return (1 << (lk - t)) + (p >> t);
}

__device__ __forceinline__ double haar_d(int lk, int l, int j)
{
    const int K = 1 << lk;
    if (l >= K || j >= K) return 0.0;
    if (l == 0) return 1.0 / sqrt(double(K));
    const int t = 31 - __clz(l);
    const int e = lk - t;
    const int first = (l - (1 << t)) << e;
    if (j < first || j >= first + (1 << e)) return 0.0;
    const double v = 1.0 / sqrt(double(1 << e));
    return (j - first) < (1 << (e - 1)) ? v : -v;
}

// hardware square root and reciprocal (about 1 ulp)
__device__ __forceinline__ float fsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }
// [v]_+ in one instruction (v_med3_f32; +inf becomes the largest float)
__device__ __forceinline__ float relu(float v) { return __builtin_amdgcn_fmed3f(v, 0.f, 3.40282347e38f); }

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// sum over the 16 lanes of a row: pairs, quads, then the quad pairs (0, 1),
// (2, 3) and the two halves, each step adding the same two values in every
// lane, so that all lanes of the row get the same sum
__device__ __forceinline__ float sum16(float v)
{
    v += dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp<0x141>(v);  // row_half_mirror
    v += dpp<0x140>(v);  // row_mirror
    return v;
}

// sum over the wavefront: the row by DPP, then the lane-group pairs (0, 1),
// (2, 3) and (0, 2), (1, 3) by permlane swaps (every lane adds the same two
// values, so all get the same sum)
__device__ __forceinline__ float wave_sum(float v)
{
    float a, b;
    pair16(sum16(v), a, b);
    pair32(a + b, a, b);
    return a + b;
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

// max over the wavefront of non-negative values, which order as their bit
// patterns (integer maxima need no canonicalisation)
__device__ __forceinline__ float wave_max(float v)
{
    int x = __float_as_int(v);
    x = max(x, dpp_i<0xB1>(x));
    x = max(x, dpp_i<0x4E>(x));
    x = max(x, dpp_i<0x141>(x));
    x = max(x, dpp_i<0x140>(x));
    float a, b;
    pair16(__int_as_float(x), a, b);
    pair32(__int_as_float(max(__float_as_int(a), __float_as_int(b))), a, b);
    return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
}

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---- spatial products in split half precision.  An FP32 operand v is
// scaled by a power of two 2^k (so |v 2^k| < 2^14) and written as
// hi + lo, hi = fp16(v 2^k), lo = fp16(v 2^k - hi), both rounded to nearest:
// |v 2^k - hi - lo| <= 2^-22 |v 2^k| (lo below the fp16 normal range loses
// at most 2^-25 absolutely).  A product a . b over 32 depth steps is
// ah.bh + (ah.bl + al.bh) on v_mfma_f32_16x16x32_f16 (fp16 products are
// exact in FP32; the small cross terms accumulate apart from the main
// term), then unscaled exactly.  Its error is within 2^-21 + 32 u (u =
// 2^-24) of sum |a_i| |b_i|, which the hard-threshold error band covers.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma_h(h8 a, h8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// 2^(14 - e) for a bound B = m 2^e (0.5 <= m < 1) of the values to split,
// and its inverse
__device__ __forceinline__ float split_scale(float bound, float* inv)
{
    int e;
    (void)frexpf(bound, &e);
    *inv = ldexpf(1.f, e - 14);
    return ldexpf(1.f, 14 - e);
}

__device__ __forceinline__ void split8(const float* v, float sc, h8& hi, h8& lo)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float t = v[i] * sc;
        const _Float16 h = (_Float16)t;
        hi[i] = h;
        lo[i] = (_Float16)(t - (float)h);
    }
}

// sum over the 32 depth steps of (ah + al)(bh + bl), dropping al.bl
__device__ __forceinline__ f4 mul3(h8 ah, h8 al, h8 bh, h8 bl)
{
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    const f4 d = mfma_h(ah, bh, z);
    f4 x = mfma_h(ah, bl, z);
    x = mfma_h(al, bh, x);
    return d + x;
}

// Operand tables in LDS: matrix m (T, T o T, U), part (hi, lo), column
// block c, lane; lane (m16, lg) holds the eight B operands of block c at
// depth 8lg + s (one 16-byte read).
__device__ __forceinline__ int opnd_index(int m, int part, int c, int lane)
{
    return (((m * 2 + part) * 2 + c) * kWave + lane) * 8;
}

__device__ __forceinline__ h8 opnd_h(const _Float16* ops, int m, int part, int c, int lane)
{
    return *reinterpret_cast<const h8*>(ops + opnd_index(m, part, c, lane));
}

// SH: shrinkage; STAGED: 1-D arrays whose chunk windows are staged in LDS;
// WPLAIN: classic weights in group scope, coefficient domain
template <int SH, bool STAGED, bool WPLAIN>
__global__ __launch_bounds__(kWave * kWaves) __attribute__((amdgpu_waves_per_eu(3)))
void k_filter_1d(FilterArgs a, int sub, int tile_cap, int tile_back, int wcap)
{
    const int chunk = sub * kWaves;  // references per workgroup
    constexpr bool wiener = SH == BMND_SHRINK_WIENER;
    __shared__ __align__(16) _Float16 ops[3 * 2 * 2 * kWave * 8];
    __shared__ unsigned omax_[3];  // bit patterns of max |T|, |T o T|, |U|
    __shared__ unsigned negs_;     // some staged variance-map source is negative
    __shared__ unsigned smax_[2];  // bit patterns of the largest staged |y|, |pilot|
    __shared__ __align__(16) float ztr_[kWaves][16 * kZs];
    __shared__ float rl_[kWaves][16];
    // per wavefront its accumulation tile: two [wcap] numerator copies and
    // [wcap] member weights by origin; then 8 zeros and [tile_cap] staged
    // samples, 8 zeros and [tile_cap] staged pilot
    extern __shared__ __align__(16) float tile[];

    const Geo& g = a.g;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int m16 = lane & 15;
    const int lg = lane >> 4;
    float* ztr = ztr_[wave];
    float* rl = rl_[wave];

    // ---- operands of the spatial products: T[q][i], (T o T)[q][i] and
    // U[i][q] at q (or i) = 16c + m16 and depth i (or q) = 8lg + s, split
    // into halves at a power-of-two scale per matrix
    if (threadIdx.x < 3) omax_[threadIdx.x] = 0u;
    if (threadIdx.x == 0) negs_ = 0u;
    if (threadIdx.x < 2) smax_[threadIdx.x] = 0u;
    __syncthreads();
    {
        float mt = 0.f, mu = 0.f;
        for (int e = threadIdx.x; e < kJ * kJ; e += kWave * kWaves) {
            mt = fmaxf(mt, fabsf(a.t.f32[a.t.T[kAx - 1] + e]));
            mu = fmaxf(mu, fabsf(a.t.f32[a.t.U[kAx - 1] + e]));
        }
        // non-negative floats order as their bit patterns
        atomicMax(&omax_[0], __float_as_uint(mt));
        atomicMax(&omax_[1], __float_as_uint(mt * mt));
        atomicMax(&omax_[2], __float_as_uint(mu));
    }
    __syncthreads();
    float osc[3], oinv[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) osc[m] = split_scale(__uint_as_float(omax_[m]), &oinv[m]);
    for (int e = threadIdx.x; e < 3 * 2 * kWave * 8; e += kWave * kWaves) {
        const int k = e & 7;
        const int ln = (e >> 3) & (kWave - 1);
        const int c = (e >> 9) & 1;
        const int m = e >> 10;
        const int off = m == 2 ? a.t.U[kAx - 1] : a.t.T[kAx - 1];
        float v = a.t.f32[off + (16 * c + (ln & 15)) * kJ + 8 * (ln >> 4) + k];
        if (m == 1) v = v * v;
        const float t = v * (m == 0 ? osc[0] : (m == 1 ? osc[1] : osc[2]));
        const _Float16 h = (_Float16)t;
        ops[opnd_index(m, 0, c, ln) + k] = h;
        ops[opnd_index(m, 1, c, ln) + k] = (_Float16)(t - (float)h);
    }
    float w0 = 1.f, rn0 = 1.f;  // leading axes have one-sample patches
#pragma unroll
    for (int d = 0; d < kAx - 1; ++d) {
        w0 *= a.t.f32[a.t.win[d]];
        rn0 *= a.t.f32[a.t.rn[d]];
    }
    float wq[2], rq[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        wq[c] = w0 * a.t.f32[a.t.win[kAx - 1] + 16 * c + m16];
        rq[c] = rn0 * a.t.f32[a.t.rn[kAx - 1] + 16 * c + m16];
    }
    const double* T64 = a.t.f64 + a.t.T64[kAx - 1];
    // signs of the cross-lane Haar levels and the lane groups that keep
    // their level-3 value at level 4
    const float s3 = (lg & 1) ? -1.f : 1.f;
    // level 4 as cA a + sB b (sBq: the squared rows, all signs +)
    const float sB = lg == 0 ? 1.f : (lg == 1 ? 0.f : (lg == 2 ? -1.f : 1.f));
    const float sBq = lg == 1 ? 0.f : 1.f;
    const float cA = lg == 3 ? 0.f : 1.f;

    const int nchunk = (a.n_refs + chunk - 1) / chunk;
    // workgroups are dealt to the 8 XCDs in turn: give each XCD a contiguous
    // run of chunks, so neighbours (whose windows and tiles overlap) share an
    // L2 (a bijection; the last gridDim.x % 8 workgroups keep their index)
    int bid = int(blockIdx.x);
    {
        const int q = int(gridDim.x) / 8;
        if (bid < 8 * q) bid = (bid % 8) * q + bid / 8;
    }
    const int b = bid / nchunk;
    const int g0 = (bid - b * nchunk) * chunk;
    const int g1 = min(a.n_refs, g0 + chunk);
    const long vb = long(b) * g.V;
    // this wavefront: references [w0g, w1g), accumulated in its own tile
    // [wlo, wlo + wcap); the workgroup stages [tile_lo, tile_lo + tile_cap)
    const int w0g = min(g1, g0 + wave * sub);
    const int w1g = min(g1, w0g + sub);
    const int tile_lo = tile_cap > 0 ? a.match[(long(b) * a.n_refs + g0) * a.gmax] - tile_back : 0;
    const int wlo = (wcap > 0 && w0g < w1g) ? a.match[(long(b) * a.n_refs + w0g) * a.gmax] - tile_back : 0;
    float* tnum = tile + wave * 3 * wcap;  // copies [0, wcap) and [wcap, 2 wcap)
    float* twt = tnum + 2 * wcap;
    // each staged array follows 8 zeros, which lanes past a group's K read
    float* ysm = tile + kWaves * 3 * wcap + 8;
    float* psm = ysm + tile_cap + 8;
    const bool poisson = a.noise == BMND_NOISE_POISSON;
    const int omax = last_origin(g);
    // lanes past a group's K gather (and add zeros) at the wavefront's first
    // reference origin (slot 0 of its first group), which lies inside the
    // chunk's staged range and the wavefront's tile
    const int fall = safe_origin(w0g < w1g ? a.match[(long(b) * a.n_refs + w0g) * a.gmax] : tile_lo, omax);
    const bool acc_tile = wcap > 0 && a.out_mode == 1;
    const float* yb = a.y + vb;
    const float* pb = a.pilot ? a.pilot + vb : nullptr;
    // 1-D arrays: the samples around the chunk's references, staged once
    {
        bool neg = false;
        float my = 0.f, mp = 0.f;
        for (int i = threadIdx.x; i < tile_cap; i += kWave * kWaves) {
            const int u = tile_lo + i;
            const bool inb = u >= 0 && u < g.V;
            const float yv = inb ? yb[u] : 0.f;
            ysm[i] = yv;
            float src = yv;
            if constexpr (wiener) {
                src = inb ? pb[u] : 0.f;
                psm[i] = src;
                my = fmaxf(my, fabsf(yv));
                mp = fmaxf(mp, fabsf(src));
            }
            neg = neg || src < 0.f;
        }
        if (neg) atomicOr(&negs_, 1u);
        if constexpr (wiener) {
            // non-negative floats order as their bit patterns
            atomicMax(&smax_[0], __float_as_uint(my));
            atomicMax(&smax_[1], __float_as_uint(mp));
        }
    }
    for (int i = lane; i < 3 * wcap; i += kWave) tnum[i] = 0.f;
    if (threadIdx.x < 8) {
        ysm[int(threadIdx.x) - 8] = 0.f;
        if constexpr (wiener) psm[int(threadIdx.x) - 8] = 0.f;
    }
    __syncthreads();
    // Poisson: no negative source sample in the staged range, so the groups
    // read from it need no test of their own
    const bool staged_nonneg = poisson && __builtin_amdgcn_readfirstlane(negs_) == 0u;
    // the Wiener stage bounds the split scales of groups read from the staged
    // range by its largest magnitudes instead of the group norms (a split
    // keeps 22 bits of every value above 2^-17 of its bound; the
    // hard-threshold stage keeps the group norm, its error band needs it)
    const float ymax = __uint_as_float(__builtin_amdgcn_readfirstlane(smax_[0]));
    const float pmax = __uint_as_float(__builtin_amdgcn_readfirstlane(smax_[1]));

    // ---- front end of one group: its size and origin, the gather of its
    // samples (and pilot) and the forward products on the matrix cores.
    // The loop below runs the front end of group gi + 1 in the same basic
    // block as the shrinkage of group gi, so the scheduler interleaves the
    // matrix-core chain of one with the vector work of the other.
    struct Front {
        // Wiener stage: butterfly values as they come (see the shrinkage);
        // other stages: orthonormal coefficients and their variances
        f4 Y[2], V[2], G[2];
        float uy, uv, up;  // split unscales (powers of two)
        float rp;          // 1 / up (exact: the product of the forward scales)
        float gn;   // norm of the group's samples
        int K, lk, oa;
        bool ok;    // every lane's samples came from the staged range
    };
    auto front = [&](int kraw, int mraw, bool lds) __attribute__((always_inline)) -> Front {
        Front f;
        f.rp = 1.f;
        f.K = __builtin_amdgcn_readfirstlane(safe_count(kraw, a.gmax));
        f.lk = 31 - __clz(f.K);
        const bool av = m16 < f.K;  // this lane's member in the A layout
        // lanes past K read the samples at the fallback origin and drop them
        f.oa = av ? safe_origin(mraw, omax) : fall;
        float x[8], pv[8], mv[8];
        f.ok = true;
        if (lds) {
            // clamped reads keep the block branch-free; a group reaching
            // outside the staged range is redone from global memory
            // (lanes past K read the zeros before the arrays)
            const int ol = f.oa - tile_lo + 8 * lg;
            f.ok = __all(!av || (ol >= 0 && ol + 8 <= tile_cap));
            const int olc = av ? max(min(ol, tile_cap - 8), 0) : -8;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                x[s] = ysm[olc + s];
                pv[s] = wiener ? psm[olc + s] : 0.f;
            }
        } else {
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                x[s] = av ? yb[f.oa + 8 * lg + s] : 0.f;
                pv[s] = wiener && av ? pb[f.oa + 8 * lg + s] : 0.f;
            }
        }
        // split operands; the group norms (or the staged maxima) bound every
        // entry
        float gp = 0.f;
        if (wiener && lds) {
            f.gn = ymax;
            gp = pmax;
        } else {
            float gn2 = 0.f, gp2 = 0.f;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                gn2 = __builtin_fmaf(x[s], x[s], gn2);
                if constexpr (wiener) gp2 = __builtin_fmaf(pv[s], pv[s], gp2);
            }
            f.gn = fsqrt(wave_sum(gn2));
            if constexpr (wiener) gp = fsqrt(wave_sum(gp2));
        }
        h8 xh, xl, mh, ml, ph, pl;
        float ix, ip = 1.f, im;
        split8(x, split_scale(f.gn, &ix), xh, xl);
        if constexpr (wiener) {
            const float scp = split_scale(gp, &ip);
            split8(pv, scp, ph, pl);
            f.rp = osc[0] * scp;
        }
        // variance map s_P [src]_+ (Poisson) or sigma^2, scaled while formed.
        // Poisson with no negative source sample in the group (always so
        // for counts): the map is s_P src, whose split is the source's own
        // with s_P in the unscale.
        bool nonneg = lds && staged_nonneg;
        if (poisson && !nonneg) {
            float mn = 0.f;
#pragma unroll
            for (int s = 0; s < 8; ++s) mn = fminf(mn, wiener ? pv[s] : x[s]);
            nonneg = __all(mn >= 0.f);
        }
        if (nonneg) {
            mh = wiener ? ph : xh;
            ml = wiener ? pl : xl;
            im = (wiener ? ip : ix) * a.s_p;
        } else {
            const float scm = split_scale(poisson ? a.s_p * (wiener ? gp : f.gn) : a.sigma2, &im);
            const float mp = poisson ? a.s_p * scm : 0.f, mg = poisson ? 0.f : a.sigma2 * scm;
#pragma unroll
            for (int s = 0; s < 8; ++s)
                mv[s] = __builtin_fmaf(relu(wiener ? pv[s] : x[s]), mp, av ? mg : 0.f);
            split8(mv, 1.f, mh, ml);
        }
        // ---- analysis: spatial rows 16c + m16 of every member (split
        // half-precision products), then the Haar transform over the members
        // in registers; the split scales are undone together with the Haar
        // normalisation 2^(-t/2) of each position
        f.uy = oinv[0] * ix;
        f.uv = oinv[1] * im;
        f.up = oinv[0] * ip;
        const float d0 = haar_norm0(lg, f.lk);
        const f4 ny = {f.uy * d0, f.uy * kRsqrt2, f.uy * 0.5f, f.uy * kRsqrt2};
        const f4 nv = {f.uv * d0 * d0, f.uv * 0.5f, f.uv * 0.25f, f.uv * 0.5f};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const h8 th = opnd_h(ops, 0, 0, c, lane), tl = opnd_h(ops, 0, 1, c, lane);
            const f4 y1 = mul3(xh, xl, th, tl);
            const f4 v1 = mul3(mh, ml, opnd_h(ops, 1, 0, c, lane), opnd_h(ops, 1, 1, c, lane));
            f.Y[c] = haar_fwd(y1, s3, sB, cA);
            f.V[c] = haar_fwd_sq(v1, sBq, cA);
            f.G[c] = f4{0.f, 0.f, 0.f, 0.f};
            if constexpr (wiener) {
                f.G[c] = haar_fwd(mul3(ph, pl, th, tl), s3, sB, cA);
            } else {
                f.Y[c] = f.Y[c] * ny;
                f.V[c] = f.V[c] * nv;
            }
        }
        if constexpr (wiener && WPLAIN) {
            // the group weight needs only the gains: they replace G here (the
            // shrinkage below explains the folded scales), and V is not kept
            const float kuv = f.uv * (f.rp * f.rp);
            const float kA = a.power_a * kuv, kS = a.s_v * kuv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float lv = 4 * lg + r < f.K ? 1.f : 0.f;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float v = relu(f.V[c][r]), gam = f.G[c][r];
                    const float shat = relu(__builtin_fmaf(-kA, v, gam * gam)) * lv;
                    const float den = __builtin_fmaf(kS, v, shat);
                    f.G[c][r] = den > 0.f ? shat * frcp(den) : 0.f;
                }
            }
        }
        return f;
    };

    const long grp_base = long(b) * a.n_refs;
    // group gidx's size and this lane's entry of its match list
    auto list = [&](int gidx, int& kr, int& mr) __attribute__((always_inline)) {
        const long grp = grp_base + gidx;
        kr = a.count[grp];
        mr = a.match[grp * a.gmax + min(m16, a.gmax - 1)];
    };
    if (w0g < w1g) {
        int kr0, mr0, kr1, mr1;
        list(w0g, kr0, mr0);
        list(min(w0g + 1, w1g - 1), kr1, mr1);
        Front F = front(kr0, mr0, STAGED);
        if (!F.ok) F = front(kr0, mr0, false);
        for (int gi = w0g; gi < w1g; ++gi) {
            const long grp = grp_base + gi;
            const int K = F.K, lk = F.lk, oa = F.oa;
            // ---- block A: the next group's front end (the last group
            // repeats itself) beside this group's shrinkage; the match-list
            // entries are loaded two groups ahead
            Front N = front(kr1, mr1, STAGED);
            const int krn = kr1, mrn = mr1;
            list(min(gi + 2, w1g - 1), kr1, mr1);

            // shrinkage; coefficient (c, r), bit 4c + r: Haar position
            // 4lg + r, spatial row 16c + m16
            float C[2][4], at_[2][4], v_[2][4], sh_[2][4];
            // Wiener stage on butterfly values: at position p, Gamma = Gb up
            // D and V = Vb uv D^2 (D the Haar normalisation of p), so the gain
            // shat / (shat + s_v V), shat = [Gamma^2 - a V]_+, is that of
            // Gb^2 - kA Vb and kS Vb with kA = a uv / up^2, kS = s_v uv / up^2
            // (up, uv powers of two).  C is kept pre-multiplied by D, as the
            // inverse butterflies need it: C D = at Yb uy D^2.
            const float dq = haar_norm0(lg, lk);
            const float kuv = F.uv * (F.rp * F.rp);  // uv / up^2, no division
            const float kA = a.power_a * kuv;
            const float kS = a.s_v * kuv;
            const f4 d2 = {dq * dq, 0.5f, 0.25f, 0.5f};
            // 1 at Haar positions below K, 0 past it (the Wiener gain is 0
            // there, which zeroes C and the weight terms)
            float lvf[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) lvf[r] = 4 * lg + r < F.K ? 1.f : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float Yv = F.Y[c][r];
                    const float v = relu(F.V[c][r]);
                    float at = 0.f, Cv = 0.f, shat = 0.f;
                    if constexpr (SH == BMND_SHRINK_SOFT) {
                        const float m = fmaxf(fabsf(Yv) - a.lambda * fsqrt(v), 0.f);
                        Cv = Yv > 0.f ? m : (Yv < 0.f ? -m : 0.f);
                        at = Yv != 0.f ? m * frcp(fabsf(Yv)) : 0.f;
                    } else if constexpr (SH == BMND_SHRINK_WIENER && WPLAIN) {
                        at = F.G[c][r];  // the gain, from the front end
                        Cv = at * Yv * (F.uy * d2[r]);
                    } else if constexpr (SH == BMND_SHRINK_WIENER) {
                        const float gam = F.G[c][r];
                        shat = relu(__builtin_fmaf(-kA, v, gam * gam)) * lvf[r];
                        const float den = __builtin_fmaf(kS, v, shat);
                        at = den > 0.f ? shat * frcp(den) : 0.f;
                        Cv = at * Yv * (F.uy * d2[r]);
                        if constexpr (!WPLAIN) {
                            // the weighting models need the true scales
                            shat *= F.up * F.up * d2[r];
                        }
                    }
                    // positions past K carry no coefficient (the inverse
                    // butterflies need zeros there)
                    C[c][r] = SH == BMND_SHRINK_WIENER || 4 * lg + r < F.K ? Cv : 0.f;
                    at_[c][r] = at;
                    v_[c][r] = SH == BMND_SHRINK_WIENER && !WPLAIN ? v * (F.uv * d2[r]) : v;
                    sh_[c][r] = shat;
                }
            }
            // hard threshold on squares: |Y| > lambda sqrt(v) iff Y^2 >
            // lambda^2 v.  The FP32 error band: transform round-off is bounded
            // by the row norm times the group norm (e), so a decision can be
            // wrong only if ||Y| - thr| <= d = 1e-5 (e + thr); then thr <=
            // |Y| + d, d <= d' = 1.0001e-5 (e + |Y|), and |Y^2 - thr^2| =
            // ||Y| - thr| (|Y| + thr) <= d' (2 |Y| + d'), the test below.
            const float l2 = a.lambda * a.lambda;
            bool anynear = false;
            if constexpr (SH == BMND_SHRINK_HARD) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float e = rq[c] * F.gn;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float Yv = F.Y[c][r];
                        const float v = v_[c][r];
                        const float q = __builtin_fmaf(Yv, Yv, -l2 * v);
                        const bool lv = 4 * lg + r < K;
                        const bool kp = lv & (q > 0.f);
                        const float ay = fabsf(Yv);
                        const float d = 1.0001e-5f * (e + ay);
                        anynear |= lv & (fabsf(q) <= d * (2.f * ay + d));
                        at_[c][r] = kp ? 1.f : 0.f;
                        C[c][r] = kp ? Yv : 0.f;
                    }
                }
            }

            if constexpr (SH == BMND_SHRINK_HARD) {
                // FP64 decisions for the coefficients in the error band, one
                // at a time, from the group's samples read again
                if (__any(anynear)) {
                    unsigned keep = 0, near = 0;
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const float e = rq[c] * F.gn;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float Yv = F.Y[c][r];
                            const float v = v_[c][r];
                            const float q = __builtin_fmaf(Yv, Yv, -l2 * v);
                            const bool lv = 4 * lg + r < K;
                            const float ay = fabsf(Yv);
                            const float d = 1.0001e-5f * (e + ay);
                            const bool nr = lv & (fabsf(q) <= d * (2.f * ay + d));
                            keep |= unsigned(at_[c][r] != 0.f) << (4 * c + r);
                            near |= unsigned(nr) << (4 * c + r);
                        }
                    }
                    float x[8];
                    {
                        const bool av = m16 < K;
                        const int ol = oa - tile_lo + 8 * lg;
                        const bool lds = STAGED && __all(ol >= 0 && ol + 8 <= tile_cap);
#pragma unroll
                        for (int s = 0; s < 8; ++s) {
                            const float xs = lds ? ysm[max(min(ol, tile_cap - 8), 0) + s]
                                                 : yb[oa + 8 * lg + s];
                            x[s] = av ? xs : 0.f;
                        }
                    }
                    for (;;) {
                        const unsigned long long mk = __ballot(near != 0);
                        if (mk == 0) break;
                        const int src = __ffsll(mk) - 1;
                        const int bit = __ffs(__shfl(int(near), src)) - 1;
                        // standard Haar row of the coefficient's position
                        const int l = haar_row_of(4 * (src >> 4) + (bit & 3), lk);
                        const int q = 16 * (bit >> 2) + (src & 15);
                        // opaque copies keep the FP64 set-up inside this
                        // rarely taken loop
                        int lkv = lk;
                        asm volatile("" : "+v"(lkv));
                        const double h = haar_d(lkv, l, m16);
                        double sy = 0.0, sv = 0.0, sm = 0.0;
                        if (m16 < K) {
#pragma unroll
                            for (int s = 0; s < 8; ++s) {
                                float xv = x[s];
                                asm volatile("" : "+v"(xv));
                                const double w = h * T64[q * kJ + 8 * lg + s];
                                const double xs = double(xv);
                                sy += w * xs;
                                sm += fabs(w * xs);
                                sv += w * w * (poisson ? a.s_p64 * fmax(xs, 0.0) : a.sigma2_64);
                            }
                        }
                        sy = wave_sum64(sy);
                        sv = wave_sum64(sv);
                        sm = wave_sum64(sm);
                        // strict inequality with the 1e-9 relative tie margin;
                        // with zero variance, coefficients up to 1e-9 of the
                        // magnitude of their terms are rounding residues of
                        // exact zeros
                        const bool kp = sv > 0.0 ? fabs(sy) > a.lambda64 * sqrt(sv) * (1.0 + 1e-9)
                                                 : fabs(sy) > 1e-9 * sm;
                        if (lane == src) {
                            near &= ~(1u << bit);
                            keep = kp ? (keep | (1u << bit)) : (keep & ~(1u << bit));
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const float at = (keep >> (4 * c + r)) & 1u ? 1.f : 0.f;
                            at_[c][r] = at;
                            C[c][r] = at != 0.f ? F.Y[c][r] : 0.f;
                        }
                }
            }

            // ---- block C: risk surrogates and weights beside the synthesis
            // products.  Synthesis: Z = H^T C (A[row m16][depth (lg, s)] =
            // H[4lg + s][m16]) ...
            // (the Wiener stage's C is pre-multiplied by D already)
            const f4 nz = SH == BMND_SHRINK_WIENER ? f4{1.f, 1.f, 1.f, 1.f}
                                                   : f4{dq, kRsqrt2, 0.5f, kRsqrt2};
            f4 Z[2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
                Z[c] = haar_inv(f4{C[c][0], C[c][1], C[c][2], C[c][3]} * nz, s3, sB, cA);
            float wA;  // weight of member m16
            if constexpr (WPLAIN) {
                // classic model, group scope: R = sum of a_t^2 over the group
                float t = 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // (hard-threshold and Wiener gains are 0 past K already)
                    const bool lv = SH != BMND_SHRINK_SOFT || 4 * lg + r < K;
                    t += lv ? at_[0][r] * at_[0][r] + at_[1][r] * at_[1][r] : 0.f;
                }
                const float R = wave_sum(t);
                wA = R > 0.f ? frcp(R) : 1.f;
            } else {
                float tr[2][4];
                if (a.wmodel == BMND_WEIGHT_CLASSIC) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 2; ++c) tr[c][r] = at_[c][r] * at_[c][r];
                } else if (a.wmodel == BMND_WEIGHT_VARIANCE) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 2; ++c) tr[c][r] = at_[c][r] * at_[c][r] * v_[c][r];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const float at = at_[c][r];
                            tr[c][r] = at * at * v_[c][r] + (1.f - at) * (1.f - at) * sh_[c][r];
                        }
                }
                // windowed synthesized domain: each term weighted by the
                // metric's diagonal at its spatial coefficient
                float hq[2] = {1.f, 1.f};
                if (a.wdomain == BMND_WDOMAIN_WINDOWED) {
#pragma unroll
                    for (int c = 0; c < 2; ++c) hq[c] = window_metric(a, 16 * c + m16);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool lv = 4 * lg + r < K;
#pragma unroll
                    for (int c = 0; c < 2; ++c) tr[c][r] = lv ? tr[c][r] * hq[c] : 0.f;
                }
                if (a.wscope == BMND_SCOPE_GROUP) {
                    float t = 0.f;
#pragma unroll
                    for (int r = 0; r < 4; ++r) t += tr[0][r] + tr[1][r];
                    const float R = wave_sum(t);
                    wA = R > 0.f ? frcp(R) : 1.f;
                } else {
                    // per-plane surrogates r_l by Haar position 4lg + r; R_j = sum_l
                    // H[l][j]^2 r_l: the scaling row and one detail row per
                    // level hold member j
                    float rr[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) rr[r] = sum16(tr[0][r] + tr[1][r]);
                    if (m16 == 0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) rl[4 * lg + r] = rr[r];
                    }
                    wsync();
                    // (rl by coefficient position: the detail row of level
                    // e holding member j sits at ((j >> e) << e) + 2^(e-1))
                    float R = ldexpf(rl[0], -lk);
                    for (int e = 1; e <= lk; ++e)
                        R += ldexpf(rl[((m16 >> e) << e) + (1 << (e - 1))], -e);
                    wA = R > 0.f ? frcp(R) : 1.f;
                    wsync();
                }
            }
            // ... through LDS into the A layout, then X^ = Z U^T
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) ztr[(4 * lg + r) * kZs + 16 * c + m16] = Z[c][r];
            wsync();
            float za[8];
            {
                // members past K read the zeros before the staged samples, so
                // their synthesized samples are 0
                const float* zs = m16 < K ? ztr + m16 * kZs + 8 * lg : ysm - 8;
                const float4 u0 = *reinterpret_cast<const float4*>(zs);
                const float4 u1 = *reinterpret_cast<const float4*>(zs + 4);
                za[0] = u0.x; za[1] = u0.y; za[2] = u0.z; za[3] = u0.w;
                za[4] = u1.x; za[5] = u1.y; za[6] = u1.z; za[7] = u1.w;
            }
            wsync();
            // the split bound: the largest |Z| of the group
            float zm = 0.f;
#pragma unroll
            for (int i = 0; i < 8; ++i) zm = fmaxf(zm, fabsf(za[i]));
            float iz;
            const float scz = split_scale(wave_max(zm), &iz);
            h8 zh, zl;
            split8(za, scz, zh, zl);
            const float uz = oinv[2] * iz;
            f4 o[2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
                o[c] = mul3(zh, zl, opnd_h(ops, 2, 0, c, lane), opnd_h(ops, 2, 1, c, lane)) * uz;

            // ---- outputs; o[c][r] is sample 16c + m16 of member 4lg + r
            int od[4];
            float wd[4];
            // group-scope weights are the same for every member
            const bool wuni = WPLAIN || a.wscope == BMND_SCOPE_GROUP;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                od[r] = __shfl(oa, 4 * lg + r);
                wd[r] = wuni ? wA : __shfl(wA, 4 * lg + r);
            }
            // every member of the group inside the accumulation tile (members
            // past K sit at the fallback origin and add zeros)
            bool in_tile = acc_tile;
#pragma unroll
            for (int r = 0; r < 4; ++r) in_tile = in_tile & (unsigned(od[r] - wlo) <= unsigned(wcap - kJ));
            if (a.out_mode == 0) {
                float* pout = a.patches + grp * long(a.gmax) * kJ;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 4 * lg + r;
                    if (k < a.gmax) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) pout[k * kJ + 16 * c + m16] = k < K ? o[c][r] : 0.f;
                    }
                }
                if (lane < a.gmax) a.weights[grp * a.gmax + lane] = lane < K ? wA : 0.f;
            } else if (a.out_mode == 1 && __all(in_tile)) {
                // every member inside this wavefront's tile (members past K add
                // zeros at the fallback origin).  Numerators: lane groups
                // 0 and 2 update the first copy, 1 and 3 the second, and the
                // pairs (0, 1) and (2, 3) take turns, so no instruction updates
                // a sample twice.  LDS requests of a wavefront are served in
                // issue order, so each read sees every earlier write without a
                // wait between them.  Denominators: the weight of each member
                // at its origin (the members of a group have distinct origins);
                // the flush applies the window.
                float add[4][2];
                int tl[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    tl[r] = od[r] - wlo + m16 + ((lg & 1) ? wcap : 0);
#pragma unroll
                    for (int c = 0; c < 2; ++c) add[r][c] = wd[r] * wq[c] * o[c][r];
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if ((lg >> 1) == q) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
#pragma unroll
                            for (int c = 0; c < 2; ++c) tnum[tl[r] + 16 * c] += add[r][c];
                        }
                    }
                }
                if (lane < K) twt[oa - wlo] += wA;
                wsync();
            } else if (a.out_mode == 1) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (4 * lg + r < K) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const int u = od[r] + 16 * c + m16;
                            const float ww = wd[r] * wq[c];
                            unsafeAtomicAdd(&a.numd[vb + u], double(ww * o[c][r]));
                            unsafeAtomicAdd(&a.dend[vb + u], double(ww));
                        }
                    }
                }
            } else if (a.out_mode == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (4 * lg + r < K) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const long u = vb + od[r] + 16 * c + m16;
                            unsafeAtomicAdd(&a.dend[u], double(wd[r]) * double(wq[c]));
                        }
                    }
                }
            } else {
                double zs = 0.0, zr = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (4 * lg + r < K) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const long u = vb + od[r] + 16 * c + m16;
                            const double zeta = double(wd[r]) * double(wq[c]) / a.dend[u];
                            zs += zeta;
                            zr += zeta * (double(a.y[u]) - double(o[c][r]));
                        }
                    }
                }
                zs = wave_sum64(zs);
                zr = wave_sum64(zr);
                const double alpha = zs > 0.0 ? zr / zs : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (4 * lg + r < K) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const long u = vb + od[r] + 16 * c + m16;
                            unsafeAtomicAdd(&a.numd[u], double(wd[r]) * double(wq[c]) *
                                                            (double(o[c][r]) + alpha));
                        }
                    }
                }
            }
            if (!N.ok) N = front(krn, mrn, false);
            F = N;
        }
    }

    // ---- flush this wavefront's tile; the denominator at i is the member
    // weights at origins i - t times the patch window at t
    if (acc_tile) {
        wsync();
        for (int i = lane; i < wcap; i += kWave) {
            float den = 0.f;
#pragma unroll
            for (int t = 0; t < kJ; ++t) {
                const float wt = i >= t ? twt[i - t] : 0.f;
                den = __builtin_fmaf(wt, w0 * a.t.f32[a.t.win[kAx - 1] + t], den);
            }
            const int u = wlo + i;
            if (den != 0.f && u >= 0 && u < g.V) {
                // FP64 sums: the float result does not depend on the order
                unsafeAtomicAdd(&a.numd[vb + u], double(tnum[i] + tnum[wcap + i]));
                unsafeAtomicAdd(&a.dend[vb + u], double(den));
            }
        }
    }
}

}  // namespace

bool filter_1d_supported(const Geo& g, int gmax, bool patches_in, int kex)
{
    return !patches_in && kex == 0 && g.j[0] == 1 && g.j[1] == 1 && g.j[2] == 1 && g.j[kAx - 1] == kJ &&
           gmax <= 16;
}

hipError_t launch_filter_1d(const FilterArgs& a, int step_last, hipStream_t s)
{
    const Geo& g = a.g;
    // 1-D arrays: the windows of a chunk of references fall into a short lin
    // range, staged in LDS; each wavefront accumulates its own run of
    // references in an LDS tile.  Elsewhere both are off.
    constexpr int kDynFloats = 9216;  // dynamic LDS (36 KiB) beside the static arrays
    int tile_cap = 0, tile_back = 0, wcap = 0;
    const bool one_d = g.L[0] == 1 && g.L[1] == 1 && g.L[2] == 1;
    const int nstage = a.shrink == BMND_SHRINK_WIENER ? 2 : 1;  // staged arrays
    // references per wavefront: up to 64 (48 with a staged pilot), the most
    // for which three workgroups share a compute unit's LDS with a 256-offset
    // window; fewer for small arrays so that the launch still fills the device
    const long groups = long(a.n_refs) * g.batch;
    const int sub_max = nstage == 2 ? kSubMax : 4 * kSubMax / 3;
    const int sub = int(std::max(1L, std::min<long>(sub_max, groups / kTargetWaves)));
    const int chunk = sub * kWaves;
    if (one_d) {
        const int st = max(step_last, 1);
        tile_back = g.W[kAx - 1] / 2;
        tile_cap = (chunk - 1) * st + g.W[kAx - 1] + kJ;
        if (a.out_mode == 1) wcap = (sub - 1) * st + g.W[kAx - 1] + kJ;
        if (kWaves * 3 * wcap + nstage * (tile_cap + 8) > kDynFloats) wcap = 0;
        tile_cap = min(tile_cap, kDynFloats / nstage - 8);
    }
    const int nchunk = (a.n_refs + chunk - 1) / chunk;
    const dim3 grid(unsigned(long(nchunk) * g.batch));
    const size_t lds = sizeof(float) * size_t(kWaves * 3 * wcap + nstage * (tile_cap + 8));
    const bool staged = tile_cap >= 8;
    const bool wplain = a.wmodel == BMND_WEIGHT_CLASSIC && a.wscope == BMND_SCOPE_GROUP &&
                        a.wdomain == BMND_WDOMAIN_COEFFICIENT;
#define BMND_F1D(SH, ST, WP)                                                                     \
    hipLaunchKernelGGL((k_filter_1d<SH, ST, WP>), grid, dim3(kWave * kWaves), lds, s, a, sub,   \
                       tile_cap, tile_back, wcap)
#define BMND_F1D_SH(SH)                                                                          \
    do {                                                                                         \
        if (staged && wplain) BMND_F1D(SH, true, true);                                          \
        else if (staged) BMND_F1D(SH, true, false);                                              \
        else if (wplain) BMND_F1D(SH, false, true);                                              \
        else BMND_F1D(SH, false, false);                                                         \
    } while (0)
    if (a.shrink == BMND_SHRINK_HARD) BMND_F1D_SH(BMND_SHRINK_HARD);
    else if (a.shrink == BMND_SHRINK_SOFT) BMND_F1D_SH(BMND_SHRINK_SOFT);
    else BMND_F1D_SH(BMND_SHRINK_WIENER);
#undef BMND_F1D_SH
#undef BMND_F1D
    return hipGetLastError();
}

}  // namespace bmnd
