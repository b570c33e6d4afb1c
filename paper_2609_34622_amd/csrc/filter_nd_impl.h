// Collaborative filtering for 2-D 8x8 and 3-D 4x4x4 patches (P = 64) with
// the diagonal variance model: one lane per group member, its whole patch
// in registers.  Included by the translation units that instantiate it
// (one per patch shape and stage).
//
// Layout.  A wavefront holds 64 / GM groups ("segments" of GM lanes, GM the
// stage's group_max); lane j of a segment owns member j of its group.
//   - The separable spatial transform (T on every patch axis, section Method
//     Overview: T = H_K (x) T_0 (x) ...) runs inside the lane: J-point
//     products along each axis, the matrix entries uniform (scalar
//     registers).  The variance map goes through T o T (Prop. diagonal
//     Poisson variance propagation).
//   - The orthonormal Haar transform over the K members runs across the
//     segment's lanes as unnormalised butterflies (sum on the low lane,
//     difference on the high lane, pair distances 1, 2, ..., K/2), then one
//     scale per lane: lane 0 ends with the scaling coefficient (support K),
//     lane p > 0 with the detail coefficient of support 2 lowbit(p).  The
//     squared Haar of the variances are block sums over the same supports.
//     The synthesis runs the same butterflies in reverse order on the
//     rescaled coefficients (H = F B, B the butterfly network, F the scales,
//     so H^-1 = H^T = B^T F, and every level of B is symmetric).
//   - Lanes past a group's K take no part: the butterflies of a group of K
//     never pair a member below K with one above it.
//   - Wiener stage: the gains G come from the pilot (eq. pilot-power-family,
//     eq. wiener-gain) before the observation is read, so at most two
//     64-sample arrays are live in a lane at any time.
// Shrinkage and the weight surrogates are per coefficient inside the lane;
// group sums are segment reductions.
//
// Overlap-add (Def. weighted overlap-add).  The denominator is not summed
// per sample: every member adds its weight at its origin to a per-origin
// field W, and eta = W convolved with the patch window, which is the same
// sum.  The numerator: inside bmnd_denoise a workgroup owns a spatial block
// of references, so every sample its groups touch lies in one box (the
// block, the search window and a patch); the workgroup accumulates into that
// box in LDS (FP64) and adds it once
// to the FP64 numerator with coalesced atomics.  A member outside the box
// (only for lists that bmnd_match did not produce) adds its samples to the
// numerator directly.
//
// Mass conservation (section Aggregation-Aware Mass Conservation): sweep 1
// only needs the weights (forward transforms, shrinkage, W); sweep 2 filters
// again, forms alpha_g = sum zeta (y - p) / sum zeta with zeta = w omega / eta
// in FP64 and accumulates w omega (p + alpha_g) in an FP64 box.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "bmnd_internal.h"
#include "filter_common.h"
#include "filter_nd.h"

namespace bmnd {
namespace nd {

constexpr int kWave = 64;
constexpr int kWaves = 4;                 // wavefronts per workgroup
constexpr int kThreads = kWave * kWaves;

__device__ __forceinline__ float fsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }

// value of the lane `lane ^ d` (d < 32): DPP quad permutations for 1 and
// 2, a DPP rotation of the 16-lane row by 8 for 8 (every source lane valid,
// so no old value is kept and the move can merge into the instruction that
// uses it), bit-mode swizzles (xor within 32 lanes) for 4 and 16
template <int d>
__device__ __forceinline__ float xlane(float v)
{
    const int x = __float_as_int(v);
    if constexpr (d == 1) return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xf, 0xf, true));
    else if constexpr (d == 2) return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xf, 0xf, true));
    else if constexpr (d == 8) return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x128, 0xf, 0xf, true));
    else return __int_as_float(__builtin_amdgcn_ds_swizzle(x, 0x1F | (d << 10)));
}
template <int d>
__device__ __forceinline__ double xlane64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __float_as_int(xlane<d>(__int_as_float(int(b & 0xffffffffll))));
    const int hi = __float_as_int(xlane<d>(__int_as_float(int(b >> 32))));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// sum over the lanes of a segment of GM lanes
template <int GM>
__device__ __forceinline__ float seg_sum(float v)
{
    if constexpr (GM > 1) v += xlane<1>(v);
    if constexpr (GM > 2) v += xlane<2>(v);
    if constexpr (GM > 4) v += xlane<4>(v);
    if constexpr (GM > 8) v += xlane<8>(v);
    if constexpr (GM > 16) v += xlane<16>(v);
    return v;
}
template <int GM>
__device__ __forceinline__ double seg_sum64(double v)
{
    if constexpr (GM > 1) v += xlane64<1>(v);
    if constexpr (GM > 2) v += xlane64<2>(v);
    if constexpr (GM > 4) v += xlane64<4>(v);
    if constexpr (GM > 8) v += xlane64<8>(v);
    if constexpr (GM > 16) v += xlane64<16>(v);
    return v;
}

// one J-point product along a fibre (samples base + b * stride):
// out[a] = sum_b M[a J + b] in[b]
template <int J, int stride>
__device__ __forceinline__ void fibre(float* x, int base, const float* __restrict__ M)
{
    float t[J];
#pragma unroll
    for (int a = 0; a < J; ++a) {
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < J; ++b) s = __builtin_fmaf(M[a * J + b], x[base + b * stride], s);
        t[a] = s;
    }
#pragma unroll
    for (int a = 0; a < J; ++a) x[base + a * stride] = t[a];
}

// 4-point fibres with the structure of the stage's spatial transform.
// Orthonormal DCT-II (the Wiener stage's transform): KIND 1 the analysis T (even and odd halves,
// C_0,2 = T_00 (a0 +- a1), C_1 = T_10 b0 + T_11 b1, C_3 = T_11 b0 - T_10 b1
// with a = x_n + x_3-n, b = x_n - x_3-n), 2 the synthesis U = T^T (the same
// butterflies reversed), 3 the squared entries T o T of the variance
// propagation (rows 0 and 2 both 1/4, rows 1 and 3 the even sums weighted
// (T_10^2, T_11^2) and (T_11^2, T_10^2)).  bior1.5 (the hard-threshold
// stage's), which on 4 points is the two-level Haar transform: KIND 4 T,
// 5 U, 6 T o T.  The coefficients come from the same tables as the matrix
// products; the results agree with them to FP32 round-off.
template <int KIND, int stride>
__device__ __forceinline__ void fibre_dct4(float* x, int base, const float* __restrict__ M)
{
    const float x0 = x[base], x1 = x[base + stride], x2 = x[base + 2 * stride],
                x3 = x[base + 3 * stride];
    if constexpr (KIND == 1) {
        const float h = M[0], c1 = M[4], c3 = M[5];
        const float a0 = x0 + x3, a1 = x1 + x2, b0 = x0 - x3, b1 = x1 - x2;
        x[base] = h * (a0 + a1);
        x[base + stride] = __builtin_fmaf(c1, b0, c3 * b1);
        x[base + 2 * stride] = h * (a0 - a1);
        x[base + 3 * stride] = __builtin_fmaf(c3, b0, -(c1 * b1));
    } else if constexpr (KIND == 2) {
        const float h = M[0], u1 = M[1], u3 = M[3];
        const float e0 = h * (x0 + x2), e1 = h * (x0 - x2);
        const float o0 = __builtin_fmaf(u1, x1, u3 * x3), o1 = __builtin_fmaf(u3, x1, -(u1 * x3));
        x[base] = e0 + o0;
        x[base + stride] = e1 + o1;
        x[base + 2 * stride] = e1 - o1;
        x[base + 3 * stride] = e0 - o0;
    } else if constexpr (KIND == 3) {
        const float q = M[0], s1 = M[4], s3 = M[5];
        const float e = x0 + x3, f = x1 + x2;
        const float v02 = q * (e + f);
        x[base] = v02;
        x[base + stride] = __builtin_fmaf(s1, e, s3 * f);
        x[base + 2 * stride] = v02;
        x[base + 3 * stride] = __builtin_fmaf(s3, e, s1 * f);
    } else if constexpr (KIND == 4) {
        // bior1.5 on 4 points is the two-level orthonormal Haar transform:
        // rows (1 1 1 1)/2, (1 1 -1 -1)/2, (1 -1 0 0) r, (0 0 1 -1) r
        const float h = M[0], r = M[8];
        const float s0 = x0 + x1, s1 = x2 + x3;
        x[base] = h * (s0 + s1);
        x[base + stride] = h * (s0 - s1);
        x[base + 2 * stride] = r * (x0 - x1);
        x[base + 3 * stride] = r * (x2 - x3);
    } else if constexpr (KIND == 5) {
        const float h = M[0], r = M[2];
        const float e = h * (x0 + x1), f = h * (x0 - x1), g = r * x2, k = r * x3;
        x[base] = e + g;
        x[base + stride] = e - g;
        x[base + 2 * stride] = f + k;
        x[base + 3 * stride] = f - k;
    } else {
        const float q = M[0], w = M[8];
        const float s0 = x0 + x1, s1 = x2 + x3;
        const float v01 = q * (s0 + s1);
        x[base] = v01;
        x[base + stride] = v01;
        x[base + 2 * stride] = w * s0;
        x[base + 3 * stride] = w * s1;
    }
}

// 8-point fibres.  DCT-II: rows k even are symmetric and rows k odd
// antisymmetric about the centre, so T x takes the half sums a_n = x_n +
// x_7-n and differences b_n = x_n - x_7-n (KIND 7), U C the even and odd
// partial sums E_n +- O_n (KIND 8), and T o T the half sums (KIND 9).
// bior1.5 (KIND 10 T, 12 T o T): rows 4-7 are the level-1 Haar details of
// the sample pairs (two nonzero entries each).  Coefficients from the
// tables, as above.
template <int KIND, int stride>
__device__ __forceinline__ void fibre_fast8(float* x, int base, const float* __restrict__ M)
{
    float v[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) v[n] = x[base + n * stride];
    if constexpr (KIND == 7 || KIND == 9) {
        float a[4], b[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            a[n] = v[n] + v[7 - n];
            b[n] = v[n] - v[7 - n];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float* h = (KIND == 9 || (k & 1) == 0) ? a : b;
            float acc = 0.f;
#pragma unroll
            for (int n = 0; n < 4; ++n) acc = __builtin_fmaf(M[k * 8 + n], h[n], acc);
            x[base + k * stride] = acc;
        }
    } else if constexpr (KIND == 8) {
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            float e = 0.f, o = 0.f;
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                e = __builtin_fmaf(M[n * 8 + k], v[k], e);
                o = __builtin_fmaf(M[n * 8 + k + 1], v[k + 1], o);
            }
            x[base + n * stride] = e + o;
            x[base + (7 - n) * stride] = e - o;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int n = 0; n < 8; ++n) acc = __builtin_fmaf(M[k * 8 + n], v[n], acc);
            x[base + k * stride] = acc;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float w = M[(4 + k) * 8 + 2 * k];
            x[base + (4 + k) * stride] =
                w * (KIND == 12 ? v[2 * k] + v[2 * k + 1] : v[2 * k] - v[2 * k + 1]);
        }
    }
}

template <int J, int stride, int KIND>
__device__ __forceinline__ void fibre_k(float* x, int base, const float* __restrict__ M)
{
    if constexpr (KIND != 0 && J == 4) fibre_dct4<KIND, stride>(x, base, M);
    else if constexpr (KIND != 0 && J == 8) fibre_fast8<KIND, stride>(x, base, M);
    else fibre<J, stride>(x, base, M);
}

// separable spatial transform inside a lane: the same J x J matrix along
// every patch axis (samples in C order); KIND (4-point DCT stages only)
// selects the butterfly form of fibre_dct4
template <int D, int J, int KIND = 0>
__device__ __forceinline__ void spatial_reg(float* x, const float* __restrict__ M)
{
    if constexpr (D == 2) {
#pragma unroll
        for (int r = 0; r < J; ++r) fibre_k<J, 1, KIND>(x, r * J, M);
#pragma unroll
        for (int c = 0; c < J; ++c) fibre_k<J, J, KIND>(x, c, M);
    } else {
#pragma unroll
        for (int i0 = 0; i0 < J; ++i0)
#pragma unroll
            for (int i1 = 0; i1 < J; ++i1) fibre_k<J, 1, KIND>(x, (i0 * J + i1) * J, M);
#pragma unroll
        for (int i0 = 0; i0 < J; ++i0)
#pragma unroll
            for (int i2 = 0; i2 < J; ++i2) fibre_k<J, J, KIND>(x, i0 * J * J + i2, M);
#pragma unroll
        for (int i1 = 0; i1 < J; ++i1)
#pragma unroll
            for (int i2 = 0; i2 < J; ++i2) fibre_k<J, J * J, KIND>(x, i1 * J + i2, M);
    }
}

// One butterfly level at pair distance d: lanes aligned to d take part
// (while d < K), the low lane of a pair gets the sum, the high lane the
// difference (low - high).  The lane exchanges run with every lane active;
// the arithmetic is one product and one FMA per value, s x + p m with
// m = 1, s = +-1 on the participating lanes and m = 0, s = 1 on the others
// (which keep x while p is finite: lanes past K hold zeros, and a
// non-finite sample makes its whole group non-finite through the inverse
// transform either way).  MASK: the arithmetic of a
// chunk of kHc values runs under the participating lanes' mask instead
// (fewer registers: taken where the kernel spills anyway).  At most kHc
// exchanges in flight (register pressure).
constexpr int kHc = 8;
template <int d, int N, bool MASK>
__device__ __forceinline__ void bfly(float* x, int jl, int lk)
{
    constexpr int t = d == 1 ? 0 : (d == 2 ? 1 : (d == 4 ? 2 : (d == 8 ? 3 : 4)));
    const bool part = t < lk && (jl & (d - 1)) == 0;
    const float sg = (jl & d) ? -1.f : 1.f;
    const float sm = part ? sg : 1.f;
    const float pm = part ? 1.f : 0.f;
#pragma unroll
    for (int k0 = 0; k0 < N; k0 += kHc) {
        float p[kHc];
#pragma unroll
        for (int k = 0; k < kHc; ++k) p[k] = xlane<d>(x[k0 + k]);
        if constexpr (MASK) {
            if (part) {
#pragma unroll
                for (int k = 0; k < kHc; ++k)
                    x[k0 + k] = __builtin_fmaf(sg, x[k0 + k], p[k]);   // low: x + p; high: p - x
            }
        } else {
#pragma unroll
            for (int k = 0; k < kHc; ++k) x[k0 + k] = __builtin_fmaf(sm, x[k0 + k], p[k] * pm);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}
// block sums: both lanes of a pair get the sum
template <int d, int N, bool MASK>
__device__ __forceinline__ void bsum(float* x, int jl, int lk)
{
    constexpr int t = d == 1 ? 0 : (d == 2 ? 1 : (d == 4 ? 2 : (d == 8 ? 3 : 4)));
    const bool part = t < lk && (jl & (d - 1)) == 0;
    const float pm = part ? 1.f : 0.f;
#pragma unroll
    for (int k0 = 0; k0 < N; k0 += kHc) {
        float p[kHc];
#pragma unroll
        for (int k = 0; k < kHc; ++k) p[k] = xlane<d>(x[k0 + k]);
        if constexpr (MASK) {
            if (part) {
#pragma unroll
                for (int k = 0; k < kHc; ++k) x[k0 + k] += p[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < kHc; ++k) x[k0 + k] = __builtin_fmaf(p[k], pm, x[k0 + k]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}
template <int GM, int N, bool MASK>
__device__ __forceinline__ void haar_fwd(float* x, int jl, int lk)
{
    if constexpr (GM > 1) bfly<1, N, MASK>(x, jl, lk);
    if constexpr (GM > 2) bfly<2, N, MASK>(x, jl, lk);
    if constexpr (GM > 4) bfly<4, N, MASK>(x, jl, lk);
    if constexpr (GM > 8) bfly<8, N, MASK>(x, jl, lk);
    if constexpr (GM > 16) bfly<16, N, MASK>(x, jl, lk);
}
template <int GM, int N, bool MASK>
__device__ __forceinline__ void haar_inv(float* x, int jl, int lk)
{
    if constexpr (GM > 16) bfly<16, N, MASK>(x, jl, lk);
    if constexpr (GM > 8) bfly<8, N, MASK>(x, jl, lk);
    if constexpr (GM > 4) bfly<4, N, MASK>(x, jl, lk);
    if constexpr (GM > 2) bfly<2, N, MASK>(x, jl, lk);
    if constexpr (GM > 1) bfly<1, N, MASK>(x, jl, lk);
}
template <int GM, int N, bool MASK>
__device__ __forceinline__ void haar_sq(float* x, int jl, int lk)
{
    if constexpr (GM > 1) bsum<1, N, MASK>(x, jl, lk);
    if constexpr (GM > 2) bsum<2, N, MASK>(x, jl, lk);
    if constexpr (GM > 4) bsum<4, N, MASK>(x, jl, lk);
    if constexpr (GM > 8) bsum<8, N, MASK>(x, jl, lk);
    if constexpr (GM > 16) bsum<16, N, MASK>(x, jl, lk);
}

// FP64 Haar entry H[row of lane p][member j] for a group of K
__device__ __forceinline__ double haar_entry64(int p, int j, int K)
{
    if (j >= K) return 0.0;
    if (p == 0) return 1.0 / sqrt(double(K));
    const int d = p & -p;
    const double v = 1.0 / sqrt(double(2 * d));
    if (j >= p - d && j < p) return v;
    if (j >= p && j < p + d) return -v;
    return 0.0;
}

template <int D, int J>
__device__ __forceinline__ int patch_off(int i, const Geo& g)
{
    if constexpr (D == 2) return (i / J) * g.st[kAx - 2] + (i % J);
    else return (i / (J * J)) * g.st[kAx - 3] + ((i / J) % J) * g.st[kAx - 2] + (i % J);
}

// Rows of a patch (runs of J samples along the last axis) read four samples
// per load: one address per row and four samples instead of a load per
// sample (a wavefront's lanes read different patches, so each load costs
// one address per lane).  Global memory takes these 4-byte aligned.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double d4u __attribute__((ext_vector_type(4), aligned(8)));

template <int D, int J, int P>
__device__ __forceinline__ void load_patch(const float* __restrict__ p, const Geo& g,
                                           float (&out)[P])
{
    static_assert(J % 4 == 0, "rows of a multiple of 4 samples");
#pragma unroll
    for (int r = 0; r < P / J; ++r) {
        const float* row = p + patch_off<D, J>(r * J, g);
#pragma unroll
        for (int c = 0; c < J; c += 4) {
            const f4u v = *reinterpret_cast<const f4u*>(row + c);
            out[r * J + c] = v.x;
            out[r * J + c + 1] = v.y;
            out[r * J + c + 2] = v.z;
            out[r * J + c + 3] = v.w;
        }
    }
}

// product over the patch axes of a per-axis table entry tab[axis][c_axis]
// for sample (or coefficient) index i, C-order over the D patch axes
template <int D, int J>
__device__ __forceinline__ float axis_prod(const float* __restrict__ tab, const int* off, int i)
{
    float w = 1.f;
#pragma unroll
    for (int d = D - 1; d >= 0; --d) {
        w *= tab[off[kAx - D + d] + i % J];
        i /= J;
    }
    return w;
}

// diagonal of the windowed synthesis metric for coefficient q (the product
// over the patch axes of sum_i (w_i U[i][q_d])^2)
template <int D, int J>
__device__ __forceinline__ float nd_window_metric(const float* __restrict__ tab, const FilterArgs& a,
                                                  int q)
{
    return axis_prod<D, J>(tab, a.t.hw, q);
}

// FP64 decision of one hard-threshold coefficient per segment (the row of
// lane p of the segment, spatial coefficient q): the segment's lanes add
// their members' terms, separably over the patch axes (Y, its variance and
// the magnitude of its terms), then a segment reduction.  `mine`: the lane
// takes part.  Returns the decision and, in cy / cv, the FP64 coefficient and
// its variance.
template <int D, int J, int GM>
__device__ __forceinline__ bool ht_decide64(const FilterArgs& a,
                                            const double* __restrict__ tab64,
                                            const float* __restrict__ yo, bool mine, int p,
                                            int jl, int K, int q, double* cy, double* cv)
{
    const double* __restrict__ T64 = tab64 + a.t.T64[kAx - 1];
    const bool poisson = a.noise == BMND_NOISE_POISSON;
    int qd[3] = {0, 0, 0};   // q's digit per patch axis
    {
        int qq = q;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            qd[d] = qq % J;
            qq /= J;
        }
    }
    double sy = 0.0, sv = 0.0, sm = 0.0;
    const double h = mine ? haar_entry64(p, jl, K) : 0.0;
    if (h != 0.0) {
        if constexpr (D == 2) {
#pragma unroll 1
            for (int i0 = 0; i0 < J; ++i0) {
                double ty = 0.0, tv = 0.0, tm = 0.0;
#pragma unroll
                for (int i1 = 0; i1 < J; ++i1) {
                    const double t = T64[qd[1] * J + i1];
                    const double yv = double(yo[i0 * a.g.st[kAx - 2] + i1]);
                    ty += t * yv;
                    tm += fabs(t * yv);
                    tv += t * t * (poisson ? a.s_p64 * fmax(yv, 0.0) : a.sigma2_64);
                }
                const double t0 = T64[qd[0] * J + i0];
                sy += t0 * ty;
                sm += fabs(t0) * tm;
                sv += t0 * t0 * tv;
            }
        } else {
#pragma unroll 1
            for (int i0 = 0; i0 < J; ++i0) {
                double uy = 0.0, uv = 0.0, um = 0.0;
#pragma unroll
                for (int i1 = 0; i1 < J; ++i1) {
                    double ty = 0.0, tv = 0.0, tm = 0.0;
#pragma unroll
                    for (int i2 = 0; i2 < J; ++i2) {
                        const double t = T64[qd[2] * J + i2];
                        const double yv =
                            double(yo[i0 * a.g.st[kAx - 3] + i1 * a.g.st[kAx - 2] + i2]);
                        ty += t * yv;
                        tm += fabs(t * yv);
                        tv += t * t * (poisson ? a.s_p64 * fmax(yv, 0.0) : a.sigma2_64);
                    }
                    const double t1 = T64[qd[1] * J + i1];
                    uy += t1 * ty;
                    um += fabs(t1) * tm;
                    uv += t1 * t1 * tv;
                }
                const double t0 = T64[qd[0] * J + i0];
                sy += t0 * uy;
                sm += fabs(t0) * um;
                sv += t0 * t0 * uv;
            }
        }
        sy *= h;
        sm *= fabs(h);
        sv *= h * h;
    }
    sy = seg_sum64<GM>(sy);
    sv = seg_sum64<GM>(sv);
    sm = seg_sum64<GM>(sm);
    *cy = sy;
    *cv = sv;
    // strict inequality with the 1e-9 relative tie margin; with zero
    // variance, coefficients up to 1e-9 of the magnitude of their terms are
    // rounding residues of exact zeros
    return sv > 0.0 ? fabs(sy) > a.lambda64 * sqrt(sv) * (1.0 + 1e-9) : fabs(sy) > 1e-9 * sm;
}

// OM: output mode (0 patches and weights, 1 overlap-add, 2 mass-conservation
// sweep 1, 3 mass-conservation sweep 2); SH: shrinkage; BLK: references come
// in spatial blocks (one per workgroup) with an LDS box for the numerator
// The arrays and tables come as separate restrict-qualified arguments:
// loads from them are then known not to be clobbered by the kernel's stores,
// so uniform table entries are read with scalar loads and samples with global
// (not generic) loads.
// SPK: the stage's spatial transform on 4-point fibres by butterflies (1 the
// DCT, 2 bior1.5), 0 matrix products
template <int D, int J, int GM, int SH, int OM, bool BLK, int SPK>
__global__ __launch_bounds__(kThreads, 2) void k_filter_nd(
    FilterArgs a, NdBlocks blk, const float* __restrict__ y_, const float* __restrict__ pilot_,
    const int* __restrict__ match_, const int* __restrict__ count_, const float* __restrict__ tab,
    const double* __restrict__ tab64, const int* __restrict__ bstart, double* __restrict__ numd,
    const double* __restrict__ dend, double* __restrict__ wfield)
{
    constexpr int P = D == 2 ? J * J : J * J * J;
    static_assert(P == 64, "64-sample patches");
    constexpr int NG = kWave / GM;                 // groups per wavefront
    constexpr bool WIE = SH == BMND_SHRINK_WIENER;
    static_assert(SPK == 0 || J == 4 || J == 8, "structured fibres on 4 or 8 points");
    // fibre kinds: 4 points 1-3 (DCT) and 4-6 (bior1.5); 8 points 7-9 (DCT),
    // 10 and 12 (bior1.5; its synthesis by the matrix)
    constexpr int kT = SPK == 1 ? (J == 4 ? 1 : 7) : (SPK == 2 ? (J == 4 ? 4 : 10) : 0);
    constexpr int kU = SPK == 1 ? (J == 4 ? 2 : 8) : (SPK == 2 && J == 4 ? 5 : 0);
    constexpr int kT2 = SPK == 1 ? (J == 4 ? 3 : 9) : (SPK == 2 ? (J == 4 ? 6 : 12) : 0);
    // second sweep of a thresholding stage: the first sweep recorded every
    // member's final decisions and weight (a.hmask, a.hwt), so this sweep
    // neither propagates the variances nor decides again
    constexpr bool kRecHT = !WIE && SH == BMND_SHRINK_HARD && OM == 3;
    // masked Haar arithmetic for the thresholding stages that spill either
    // way; per-lane factors for the Wiener stage and the recorded sweep
    // (which then keep their registers)
    constexpr bool kMask = !WIE && !kRecHT;
    // FP64 box: sums that do not depend on the order of the LDS atomics
    // beyond FP64 round-off, so an array's result is the same in every run
    // and in every batch or serving mix
    using Acc = double;
    extern __shared__ __align__(16) unsigned char nd_smem[];
    Acc* box = reinterpret_cast<Acc*>(nd_smem);

    const Geo& g = a.g;
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int seg = lane / GM;
    const int jl = lane % GM;
    const int omax = last_origin(g);

    // ---- this workgroup's references and (with blocks) its box
    int b = 0, r0 = 0, r1 = 0;
    int blo[kAx] = {0, 0, 0, 0};
    if constexpr (BLK) {
        // workgroups are dealt to the 8 XCDs in turn: each XCD takes a
        // contiguous run of blocks, so neighbours (whose boxes overlap)
        // share an L2 (a bijection; the last gridDim.x % 8 keep their index)
        int bid = int(blockIdx.x);
        {
            const int q = int(gridDim.x) / 8;
            if (bid < 8 * q) bid = (bid % 8) * q + bid / 8;
        }
        const int blkid = bid % blk.nblocks;
        b = bid / blk.nblocks;
        r0 = bstart[blkid];
        r1 = bstart[blkid + 1];
        if (r0 >= r1) return;   // an empty block (uniform over the workgroup)
        int rem = blkid;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            const int bc = rem % blk.nb[d];
            rem /= blk.nb[d];
            blo[d] = bc * blk.B[d] - g.W[d] / 2;
        }
        if constexpr (OM == 1 || OM == 3) {
            for (int e = threadIdx.x; e < blk.fbox; e += kThreads) box[e] = Acc(0);
            __syncthreads();
        }
    } else {
        const long per = long(kWaves) * NG;
        const long nchunk = (a.n_refs + per - 1) / per;
        b = int(blockIdx.x / nchunk);
        r0 = int((blockIdx.x - long(b) * nchunk) * per);
        r1 = min(a.n_refs, int(r0 + per));
    }
    const long vb = long(b) * g.V;
    const float* __restrict__ yb = y_ + vb;
    const float* __restrict__ pb = WIE ? pilot_ + vb : nullptr;
    const float* __restrict__ Tm = tab + a.t.T[kAx - 1];
    const float* __restrict__ T2m = tab + a.t.T2[kAx - 1];
    const float* __restrict__ Um = tab + a.t.U[kAx - 1];
    const bool poisson = a.noise == BMND_NOISE_POISSON;

    // groups handed to the wavefronts NG at a time from a shared counter (a
    // wavefront whose groups need no FP64 re-decision takes the next ones)
    __shared__ int next_grp;
    if (threadIdx.x == 0) next_grp = r0 + kWaves * NG;
    __syncthreads();
    auto take = [&]() {
        int nx = 0;
        if (lane == 0) nx = atomicAdd(&next_grp, NG);
        return __builtin_amdgcn_readfirstlane(nx);
    };
    // Wiener stage: a group's count and list entry are loaded one iteration
    // ahead (the next group base is taken from the counter at the start of
    // an iteration), so its patch loads do not wait behind them.  The
    // thresholding stages load them in their own iteration (the prefetch
    // made them slower).
    constexpr bool kPf = WIE;
    auto fetch = [&](int gb, int& c, int& m) {
        const int gi = gb + seg;
        const long grp = long(b) * a.n_refs + (gi < r1 ? gi : r0);
        c = count_[grp];
        m = jl < a.gmax ? match_[grp * a.gmax + jl] : 0;
    };
    int cnt_n = 0, mt_n = 0, nb = 0;
    if (kPf && r0 + wave * NG < r1) fetch(r0 + wave * NG, cnt_n, mt_n);
    for (int gbase = r0 + wave * NG; gbase < r1; gbase = kPf ? nb : take()) {
        int cnt = 0, mt = 0;
        if constexpr (kPf) {
            nb = take();
            cnt = cnt_n;
            mt = mt_n;
            if (nb < r1) fetch(nb, cnt_n, mt_n);
        }
        const int gi = gbase + seg;
        const bool gvalid = gi < r1;
        const long grp = long(b) * a.n_refs + (gvalid ? gi : r0);
        if constexpr (!kPf) cnt = gvalid ? count_[grp] : 0;
        const int K = gvalid ? safe_count(cnt, a.gmax) : 0;
        const int lk = 31 - __clz(max(K, 1));
        const bool act = jl < K;
        if constexpr (!kPf) mt = act ? match_[grp * a.gmax + jl] : 0;
        const int org = safe_origin(act ? mt : 0, omax);
        const float* __restrict__ yo = yb + org;   // the member's first sample
        const int sup = jl == 0 ? max(K, 1) : 2 * (jl & -jl);   // support of the lane's Haar row
        const float f = 1.f / fsqrt(float(sup));
        const float f2 = 1.f / float(sup);

        float x[P];      // observation -> Y -> C -> p
        float v[P];      // variance source -> sigma^2 (HT); Wiener: gains
        float rl = 0.f;  // weight surrogate of the lane's Haar row
        // thresholding, sweep 1: the final decisions, and those the FP64
        // re-decision kept (recorded for sweep 2)
        unsigned long long keep_out = 0, fixed = 0;
        float gn2 = 0.f;

        if constexpr (WIE) {
            // ---- pilot: Gamma and sigma^2, then the gains
            float gm[P];
            load_patch<D, J>(pb + org, g, gm);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const float pv = act ? gm[i] : 0.f;
                gm[i] = pv;
                v[i] = fmaxf(pv, 0.f);
            }
            if (poisson) {
                spatial_reg<D, J, kT2>(v, T2m);
                haar_sq<GM, P, kMask>(v, jl, lk);
                const float sc = a.s_p * f2;
#pragma unroll
                for (int i = 0; i < P; ++i) v[i] *= sc;
            } else {
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const float rn = axis_prod<D, J>(tab, a.t.rn, i);
                    v[i] = a.sigma2 * rn * rn;
                }
            }
            spatial_reg<D, J, kT>(gm, Tm);
            haar_fwd<GM, P, kMask>(gm, jl, lk);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const float vv = fmaxf(v[i], 0.f);
                const float gam = gm[i] * f;
                const float shat = fmaxf(gam * gam - a.power_a * vv, 0.f);
                const float den = shat + a.s_v * vv;
                // the gain from a hardware reciprocal (1 ulp) instead of a
                // correctly rounded division: the same gain to FP32 accuracy
                const float G = den > 0.f ? shat * __builtin_amdgcn_rcpf(den) : 0.f;
                float t;
                if (a.wmodel == BMND_WEIGHT_CLASSIC) t = G * G;
                else if (a.wmodel == BMND_WEIGHT_VARIANCE) t = G * G * vv;
                else t = G * G * vv + (1.f - G) * (1.f - G) * shat;
                if (a.wdomain == BMND_WDOMAIN_WINDOWED) t *= nd_window_metric<D, J>(tab, a, i);
                rl += act ? t : 0.f;
                v[i] = G * f;   // the gain with the row scale of Y folded in
            }
            if constexpr (OM != 2) {
                // ---- observation: C = G Y
                load_patch<D, J>(yo, g, x);
#pragma unroll
                for (int i = 0; i < P; ++i) x[i] = act ? x[i] : 0.f;
                spatial_reg<D, J, kT>(x, Tm);
                haar_fwd<GM, P, kMask>(x, jl, lk);
#pragma unroll
                for (int i = 0; i < P; ++i) x[i] *= v[i];
            }
        } else if constexpr (kRecHT) {
            load_patch<D, J>(yo, g, x);
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] = act ? x[i] : 0.f;
            spatial_reg<D, J, kT>(x, Tm);
            haar_fwd<GM, P, kMask>(x, jl, lk);
            // the decisions of the first sweep: kept (FP32 values), and among
            // them those kept by the FP64 re-decision (their FP64 values)
            const long slot = grp * a.gmax + jl;
            uint4 m = make_uint4(0u, 0u, 0u, 0u);
            if (act) m = reinterpret_cast<const uint4*>(a.hmask)[slot];
            const unsigned long long keep = (unsigned long long)m.y << 32 | m.x;
            unsigned long long fx = (unsigned long long)m.w << 32 | m.z;
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] = ((keep >> i) & 1ull) ? x[i] * f : 0.f;
            const unsigned long long segbits =
                (GM >= 64 ? ~0ull : ((1ull << GM) - 1ull)) << (seg * GM);
            for (;;) {
                const unsigned long long mk = __ballot(fx != 0);
                if (mk == 0) break;
                const unsigned long long sk = mk & segbits;
                const bool segact = sk != 0;
                const int src = segact ? __ffsll((long long)sk) - 1 : lane;
                const unsigned nlo = unsigned(__shfl(int(unsigned(fx & 0xffffffffull)), src));
                const unsigned nhi = unsigned(__shfl(int(unsigned(fx >> 32)), src));
                const int q = nlo != 0 ? __ffs(int(nlo)) - 1 : (nhi != 0 ? 32 + __ffs(int(nhi)) - 1 : 0);
                double cy = 0.0, cv = 0.0;
                (void)ht_decide64<D, J, GM>(a, tab64, yo, segact && act, src % GM, jl, K, q, &cy,
                                            &cv);
                if (segact && lane == src) {
                    fx &= ~(1ull << q);
                    const float cq = float(cy);
#pragma unroll
                    for (int i = 0; i < P; ++i) x[i] = i == q ? cq : x[i];
                }
            }
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] *= f;   // B^T F: the synthesis scale
        } else {
            // ---- observation and its variance map
            load_patch<D, J>(yo, g, x);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const float yv = act ? x[i] : 0.f;
                x[i] = yv;
                gn2 = __builtin_fmaf(yv, yv, gn2);
                v[i] = fmaxf(yv, 0.f);
            }
            spatial_reg<D, J, kT>(x, Tm);
            haar_fwd<GM, P, kMask>(x, jl, lk);
            if (poisson) {
                spatial_reg<D, J, kT2>(v, T2m);
                haar_sq<GM, P, kMask>(v, jl, lk);
                const float sc = a.s_p * f2;
#pragma unroll
                for (int i = 0; i < P; ++i) v[i] *= sc;
            } else {
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const float rn = axis_prod<D, J>(tab, a.t.rn, i);
                    v[i] = a.sigma2 * rn * rn;
                }
            }
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] *= f;
            if constexpr (SH == BMND_SHRINK_HARD) {
                // the largest row norm of the spatial transform times the
                // group norm bounds the magnitude of every coefficient's terms
                float rnmax = 1.f;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    float m = 0.f;
#pragma unroll
                    for (int c = 0; c < J; ++c) m = fmaxf(m, tab[a.t.rn[kAx - D + d] + c]);
                    rnmax *= m;
                }
                const float gb = rnmax * fsqrt(seg_sum<GM>(gn2));
                // FP32 decisions and weight terms at once (the variances die
                // here); the coefficients in the FP32 error band are recorded
                unsigned long long keep = 0, near = 0;
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const float vv = fmaxf(v[i], 0.f);
                    const float thr = a.lambda * fsqrt(vv);
                    const float ay = fabsf(x[i]);
                    // FP32 error band: the coefficient's round-off is at most
                    // about 18 unit roundoffs (the transform's sequential
                    // operations) times the magnitude of its terms, which is at
                    // most the row norm times the group norm; the threshold's
                    // relative error is half its variance's; 3e-6 keeps a
                    // factor of 2 over both
                    const float band = 3e-6f * (gb + thr);
                    const bool kp = act && ay > thr;
                    keep |= (unsigned long long)kp << i;
                    near |= (unsigned long long)(act && fabsf(ay - thr) <= band) << i;
                    float t = kp ? 1.f : 0.f;
                    if (a.wmodel == BMND_WEIGHT_VARIANCE) t *= vv;
                    if (a.wdomain == BMND_WDOMAIN_WINDOWED) t *= nd_window_metric<D, J>(tab, a, i);
                    rl += t;
                    x[i] = kp ? x[i] : 0.f;
                }
                // FP64 decisions in the band, one coefficient per segment at a
                // time; a changed decision sets the coefficient from its FP64
                // value and corrects the weight term
                const unsigned long long segbits =
                    (GM >= 64 ? ~0ull : ((1ull << GM) - 1ull)) << (seg * GM);
                for (;;) {
                    const unsigned long long mk = __ballot(near != 0);
                    if (mk == 0) break;
                    const unsigned long long sk = mk & segbits;
                    const bool segact = sk != 0;
                    const int src = segact ? __ffsll((long long)sk) - 1 : lane;
                    const unsigned nlo = unsigned(__shfl(int(unsigned(near & 0xffffffffull)), src));
                    const unsigned nhi = unsigned(__shfl(int(unsigned(near >> 32)), src));
                    const int q = nlo != 0 ? __ffs(int(nlo)) - 1 : (nhi != 0 ? 32 + __ffs(int(nhi)) - 1 : 0);
                    double cy = 0.0, cv = 0.0;
                    const bool kp = ht_decide64<D, J, GM>(a, tab64, yo, segact && act, src % GM,
                                                          jl, K, q, &cy, &cv);
                    if (segact && lane == src) {
                        near &= ~(1ull << q);
                        const bool was = (keep >> q) & 1ull;
                        if (kp != was) {
                            keep ^= 1ull << q;
                            if (kp) fixed |= 1ull << q;
                            float t = 1.f;
                            if (a.wmodel == BMND_WEIGHT_VARIANCE) t *= float(fmax(cv, 0.0));
                            if (a.wdomain == BMND_WDOMAIN_WINDOWED)
                                t *= nd_window_metric<D, J>(tab, a, q);
                            rl += kp ? t : -t;
                            const float cq = kp ? float(cy) : 0.f;
#pragma unroll
                            for (int i = 0; i < P; ++i) x[i] = i == q ? cq : x[i];
                        }
                    }
                }
                keep_out = keep;
            } else {
                // soft threshold (eq. soft-threshold), attenuation |C| / |Y|
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const float vv = fmaxf(v[i], 0.f);
                    const float Yv = x[i];
                    const float m = fmaxf(fabsf(Yv) - a.lambda * fsqrt(vv), 0.f);
                    const float at = Yv != 0.f ? m / fabsf(Yv) : 0.f;
                    float t = at * at;
                    if (a.wmodel == BMND_WEIGHT_VARIANCE) t *= vv;
                    if (a.wdomain == BMND_WDOMAIN_WINDOWED) t *= nd_window_metric<D, J>(tab, a, i);
                    rl += act ? t : 0.f;
                    x[i] = Yv > 0.f ? m : (Yv < 0.f ? -m : 0.f);
                }
            }
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] *= f;   // B^T F: the synthesis scale
        }
        if constexpr (WIE && OM != 2) {
            // x holds G f Y; the synthesis scale f again
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] *= f;
        }

        // ---- weights (Def. aggregation-weight scope): group R = sum_l r_l;
        // patch R_j = sum over the rows whose support holds j of r_l / support
        float wj;
        if constexpr (kRecHT) {
            wj = act ? a.hwt[grp * a.gmax + jl] : 0.f;
        } else if (a.wscope == BMND_SCOPE_GROUP) {
            const float R = seg_sum<GM>(rl);
            wj = R > 0.f ? 1.f / R : 1.f;
        } else {
            const float rs = rl * f2;     // r_l / support of the lane's row
            const int sbase = seg * GM;
            float R = __shfl(rs, sbase);  // scaling row
#pragma unroll
            for (int t = 0; (1 << t) < GM; ++t) {
                const int d = 1 << t;
                const float r = __shfl(rs, sbase + ((jl & ~(2 * d - 1)) | d));
                R += t < lk ? r : 0.f;
            }
            wj = R > 0.f ? 1.f / R : 1.f;
        }
        wj = act ? wj : 0.f;

        if constexpr (OM == 2) {
            // mass conservation, sweep 1: the weights only (and, thresholding,
            // the decisions and weight of every member for sweep 2)
            if (act) unsafeAtomicAdd(&wfield[vb + org], double(wj));
            if constexpr (!WIE && SH == BMND_SHRINK_HARD) {
                if (act) {
                    const long slot = grp * a.gmax + jl;
                    reinterpret_cast<uint4*>(a.hmask)[slot] =
                        make_uint4(unsigned(keep_out), unsigned(keep_out >> 32), unsigned(fixed),
                                   unsigned(fixed >> 32));
                    a.hwt[slot] = wj;
                }
            }
            continue;
        } else {
            // ---- synthesis: B^T (scales applied above), then U on every axis
            haar_inv<GM, P, kMask>(x, jl, lk);
            spatial_reg<D, J, kU>(x, Um);
            if constexpr (OM == 0) {
                // patches (no window) and weights of every slot up to group_max
                if (gvalid) {
                    float* po = a.patches + (grp * a.gmax + jl) * long(P);
#pragma unroll
                    for (int i = 0; i < P; ++i) po[i] = act ? x[i] : 0.f;
                    a.weights[grp * a.gmax + jl] = wj;
                }
                continue;
            } else {
                double alpha = 0.0;
                if constexpr (OM == 3) {
                    // alpha_g = sum zeta (y - p) / sum zeta, zeta = w omega / eta
                    // (dend holds 1 / eta here: a product per sample, and the
                    // conservation holds to FP64 round-off all the same)
                    double zs = 0.0, zr = 0.0;
                    if (act) {
                        // four partial sums: independent FP64 chains
                        double zs4[4] = {0.0, 0.0, 0.0, 0.0}, zr4[4] = {0.0, 0.0, 0.0, 0.0};
                        // kZr rows of four samples at a time: their loads of
                        // 1 / eta and y are all issued before the first use,
                        // so one memory round trip serves kZr rows
                        constexpr int kZr = 4;
#pragma unroll
                        for (int r0 = 0; r0 < P; r0 += 4 * kZr) {
                            d4u re[kZr];
                            f4u yr[kZr];
#pragma unroll
                            for (int k = 0; k < kZr; ++k) {
                                const int u = org + patch_off<D, J>(r0 + 4 * k, g);
                                re[k] = *reinterpret_cast<const d4u*>(dend + vb + u);
                                yr[k] = *reinterpret_cast<const f4u*>(yb + u);
                            }
#pragma unroll
                            for (int k = 0; k < kZr; ++k) {
                                const double rev[4] = {re[k].x, re[k].y, re[k].z, re[k].w};
                                const float yv[4] = {yr[k].x, yr[k].y, yr[k].z, yr[k].w};
#pragma unroll
                                for (int c = 0; c < 4; ++c) {
                                    const int i = r0 + 4 * k + c;
                                    const float w = axis_prod<D, J>(tab, a.t.win, i);
                                    const double zeta = double(wj) * double(w) * rev[c];
                                    zs4[c] += zeta;
                                    zr4[c] += zeta * (double(yv[c]) - double(x[i]));
                                }
                            }
                        }
                        zs = (zs4[0] + zs4[1]) + (zs4[2] + zs4[3]);
                        zr = (zr4[0] + zr4[1]) + (zr4[2] + zr4[3]);
                    }
                    zs = seg_sum64<GM>(zs);
                    zr = seg_sum64<GM>(zr);
                    alpha = zs > 0.0 ? zr / zs : 0.0;
                }
                if (!act) continue;
                if constexpr (OM == 1) unsafeAtomicAdd(&wfield[vb + org], double(wj));
                // ---- overlap-add of w omega (p [+ alpha]) into the box (or the array)
                bool inbox = BLK;
                int tb = 0;
                if constexpr (BLK) {
                    int rem = org;
#pragma unroll
                    for (int d = kAx - 1; d >= 0; --d) {
                        const int c = rem % g.L[d] - blo[d];
                        rem /= g.L[d];
                        inbox = inbox && c >= 0 && c + g.j[d] <= blk.FE[d];
                        tb += c * blk.FS[d];
                    }
                }
                // w omega exactly (FP64 product of the two floats), as in
                // eta = W * omega and in zeta: the sums then conserve mass to
                // FP64 round-off.  In chunks of kOc samples: the window
                // values (scalar loads) of a chunk are read before its LDS
                // atomics, so waiting for them does not wait for the atomics
                // sample by sample.
                const double wjd = double(wj);
                auto value = [&](int i) {
                    const double ww = wjd * double(axis_prod<D, J>(tab, a.t.win, i));
                    if constexpr (OM == 3) return ww * (double(x[i]) + alpha);
                    else return ww * double(x[i]);
                };
                if (inbox) {
                    constexpr int kOc = 16;
#pragma unroll
                    for (int i0 = 0; i0 < P; i0 += kOc) {
                        double val[kOc];
#pragma unroll
                        for (int k = 0; k < kOc; ++k) val[k] = value(i0 + k);
#pragma unroll
                        for (int k = 0; k < kOc; ++k) {
                            int qq = i0 + k, toff = 0;
#pragma unroll
                            for (int d = D - 1; d >= 0; --d) {
                                toff += (qq % J) * blk.FS[kAx - D + d];
                                qq /= J;
                            }
                            atomicAdd(&box[tb + toff], val[k]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < P; ++i)
                        unsafeAtomicAdd(&numd[vb + org + patch_off<D, J>(i, g)], value(i));
                }
            }
        }
    }

    // ---- flush the box: one FP64 atomic per touched voxel, rows contiguous
    // (the padding between rows and planes is never written and stays 0).
    // kFb cells per thread at a time, their LDS reads issued together; box
    // coordinates by a float-reciprocal quotient with one correction step
    // (exact: the index is below 2^24 and the quotient's error below 1)
    if constexpr (BLK && (OM == 1 || OM == 3)) {
        __syncthreads();
        float inv[kAx - 1];
#pragma unroll
        for (int d = 0; d < kAx - 1; ++d) inv[d] = 1.f / float(blk.FS[d]);
        constexpr int kFb = 4;
        for (int e0 = threadIdx.x; e0 < blk.fbox; e0 += kFb * kThreads) {
            Acc val[kFb];
#pragma unroll
            for (int k = 0; k < kFb; ++k) {
                const int e = e0 + k * kThreads;
                val[k] = e < blk.fbox ? box[e] : Acc(0);
            }
#pragma unroll
            for (int k = 0; k < kFb; ++k) {
                if (val[k] == Acc(0)) continue;
                int rem = e0 + k * kThreads;
                long u = vb;
                bool in = true;
#pragma unroll
                for (int d = 0; d < kAx - 1; ++d) {
                    int cb = int(float(rem) * inv[d]);
                    int r = rem - cb * blk.FS[d];
                    if (r < 0) {
                        --cb;
                        r += blk.FS[d];
                    } else if (r >= blk.FS[d]) {
                        ++cb;
                        r -= blk.FS[d];
                    }
                    rem = r;
                    const int c = cb + blo[d];
                    in = in && cb < blk.FE[d] && c >= 0 && c < g.L[d];
                    u += long(c) * g.st[d];
                }
                const int c3 = rem + blo[kAx - 1];
                in = in && rem < blk.FE[kAx - 1] && c3 >= 0 && c3 < g.L[kAx - 1];
                if (in) unsafeAtomicAdd(&numd[u + c3], double(val[k]));
            }
        }
    }
}

inline size_t box_bytes(const NdBlocks& blk, int out_mode)
{
    if (out_mode != 1 && out_mode != 3) return 0;
    return size_t(blk.fbox) * sizeof(double);
}

template <int D, int J, int GM, int SH, int OM, int SPK>
hipError_t launch_om_f(const FilterArgs& a, const NdBlocks* blk, hipStream_t s)
{
    const Geo& g = a.g;
    if constexpr (OM != 0) {
        const size_t lds = box_bytes(*blk, OM);
        const void* fn = reinterpret_cast<const void*>(&k_filter_nd<D, J, GM, SH, OM, true, SPK>);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
            if (e != hipSuccess) return e;
        }
        const dim3 grid(unsigned(long(blk->nblocks) * g.batch));
        hipLaunchKernelGGL((k_filter_nd<D, J, GM, SH, OM, true, SPK>), grid, dim3(kThreads), lds, s, a,
                           *blk, a.y, a.pilot, a.match, a.count, a.t.f32, a.t.f64, blk->start,
                           a.numd, a.dend, a.wfield);
    } else {
        const long per = long(kWaves) * (kWave / GM);
        const long nchunk = (a.n_refs + per - 1) / per;
        NdBlocks none{};
        hipLaunchKernelGGL((k_filter_nd<D, J, GM, SH, 0, false, SPK>), dim3(unsigned(nchunk * g.batch)),
                           dim3(kThreads), 0, s, a, none, a.y, a.pilot, a.match, a.count, a.t.f32,
                           a.t.f64, nullptr, a.numd, a.dend, a.wfield);
    }
    return hipGetLastError();
}

template <int D, int J, int GM, int SH, int OM>
hipError_t launch_om(const FilterArgs& a, const NdBlocks* blk, hipStream_t s)
{
    // 4- and 8-point transforms by their structure: the DCT (Wiener stage)
    // and bior1.5 (thresholding stages)
    if constexpr ((J == 4 || J == 8) && SH == BMND_SHRINK_WIENER) {
        if (a.spatial == BMND_SPATIAL_DCT) return launch_om_f<D, J, GM, SH, OM, 1>(a, blk, s);
    }
    if constexpr ((J == 4 || J == 8) && SH != BMND_SHRINK_WIENER) {
        if (a.spatial == BMND_SPATIAL_BIOR15) return launch_om_f<D, J, GM, SH, OM, 2>(a, blk, s);
    }
    return launch_om_f<D, J, GM, SH, OM, 0>(a, blk, s);
}

template <int D, int J, int GM, int SH>
hipError_t launch_sh(const FilterArgs& a, const NdBlocks* blk, hipStream_t s)
{
    switch (a.out_mode) {
    case 0: return launch_om<D, J, GM, SH, 0>(a, blk, s);
    case 1: return launch_om<D, J, GM, SH, 1>(a, blk, s);
    case 2: return launch_om<D, J, GM, SH, 2>(a, blk, s);
    default: return launch_om<D, J, GM, SH, 3>(a, blk, s);
    }
}

}  // namespace nd
}  // namespace bmnd
