// Coefficient variances of a group under stationary correlated Gaussian
// noise (section Observation Models, Def. wide-sense stationary Gaussian
// noise; Lemma covariance propagation).
//
// With Sigma_g[a][b] = c(u_b - u_a) over the group entries' sampling
// locations and T = H (x) T_sp, the variance of coefficient (l, q) is
//   sigma^2_(l,q) = sum_(j,j') H_lj H_lj' D(o_j' - o_j, q),
//   D(Delta, q)   = sum_(i,i') T_qi T_qi' c(Delta + i' - i),
// where o_j are the member origins; D is tabulated per stage over the
// member displacements of the search window.  For the orthonormal Haar rows
// (the scaling row; detail rows over dyadic blocks B, +1/sqrt|B| on the
// first half B+, -1/sqrt|B| on the second half B-), h_l^T G h_l with the
// symmetric G[j][j'] = D(o_j' - o_j, q) reduces to block sums:
//   scaling row:   S(all) / K
//   detail row B:  (S(B+) + S(B-) - 2 X(B)) / |B|
// with S(B) the sum of G over B x B and X(B) the sum over B+ x B-; S
// follows bottom-up, S(B) = S(B+) + S(B-) + 2 X(B), from S({j}) = D(0, q).
// Every pair j < j' belongs to exactly one X(B), so one table read per pair
// and coefficient gives all K variances of that coefficient.
#pragma once

#include "filter_common.h"

namespace bmnd {

// Member-box coordinate of an origin: sum_d coord_d * stride_d over the
// member box of extents cbw (wrapping 32-bit arithmetic; differences of two
// members of one search window are exact).
__device__ inline unsigned corr_member_key(const FilterArgs& a, int origin)
{
    unsigned key = 0, stride = 1;
#pragma unroll
    for (int d = kAx - 1; d >= 0; --d) {
        const int c = (origin / a.g.st[d]) % a.g.L[d];
        key += unsigned(c) * stride;
        stride *= unsigned(a.cbw[d]);
    }
    return key;
}

__device__ inline unsigned corr_box_size(const FilterArgs& a)
{
    return unsigned(a.cbw[0]) * a.cbw[1] * a.cbw[2] * a.cbw[3];
}

// Table row of the displacement between two members (key difference plus
// the box centre, cut to the table: members outside one search window read
// some entry of it, memory-safely).
__device__ inline unsigned corr_pair_row(const FilterArgs& a, unsigned kj, unsigned kjp)
{
    unsigned centre = 0, stride = 1;
#pragma unroll
    for (int d = kAx - 1; d >= 0; --d) {
        centre += unsigned((a.cbw[d] - 1) / 2) * stride;
        stride *= unsigned(a.cbw[d]);
    }
    const unsigned r = centre + kjp - kj;
    return min(r, stride - 1u);
}

// Number of member pairs j < j' of a group of K.
__host__ __device__ constexpr int corr_npairs(int K) { return K * (K - 1) / 2; }

// Table rows of every pair, in the order corr_var_q visits them: levels of
// half-size h = 1, 2, ..., K/2; blocks b of 2h members; then j in the first
// half, j' in the second.  keys[j] = corr_member_key of member j.
__device__ inline void corr_pair_rows(const FilterArgs& a, const unsigned* keys, int K,
                                      int* rows, int lane, int nl)
{
    const int np = corr_npairs(K);
    for (int p = lane; p < np; p += nl) {
        int r = p, h = 1;
        while (r >= (K / (2 * h)) * h * h) {
            r -= (K / (2 * h)) * h * h;
            h *= 2;
        }
        const int b = r / (h * h);
        const int rem = r - b * h * h;
        const int j = b * 2 * h + rem / h;
        const int jp = b * 2 * h + h + rem % h;
        rows[p] = int(corr_pair_row(a, keys[j], keys[jp]));
    }
}

// All KK variances of spatial coefficient q into V[l * P + q]: dq = table
// + q (rows of P entries), rows[] from corr_pair_rows, d0 = D(0, q).
template <int KK>
__device__ inline void corr_var_q(const double* __restrict__ dq, int P, const int* rows, double d0,
                                  float* V, int q)
{
    double S[KK];
#pragma unroll
    for (int j = 0; j < KK; ++j) S[j] = d0;
    int p = 0;
#pragma unroll
    for (int h = 1; h < KK; h *= 2) {
        const int nb = KK / (2 * h);
        const double inv = 1.0 / double(2 * h);
#pragma unroll
        for (int b = 0; b < nb; ++b) {
            double x = 0.0;
#pragma unroll
            for (int t = 0; t < h * h; ++t) x += dq[rows[p + t] * P];
            p += h * h;
            const double sp = S[2 * b], sm = S[2 * b + 1];
            V[(nb + b) * P + q] = float((sp + sm - 2.0 * x) * inv);
            S[b] = sp + sm + 2.0 * x;
        }
    }
    V[q] = float(S[0] * (1.0 / double(KK)));
}

// Variances of every coefficient of a group of K <= GM members into
// V[l * P + q] (FP32), for the spatial coefficients q = lane, lane + nl, ...
template <int GM>
__device__ inline void corr_group_variances(const FilterArgs& a, const int* rows, int K, float* V,
                                            int lane, int nl)
{
    const int P = a.g.P;
    const int c0 = int(corr_pair_row(a, 0u, 0u));
    for (int q = lane; q < P; q += nl) {
        const double* dq = a.cdtab + q;
        const double d0 = dq[c0 * P];
        switch (K) {
        case 2: if constexpr (GM >= 2) corr_var_q<2>(dq, P, rows, d0, V, q); break;
        case 4: if constexpr (GM >= 4) corr_var_q<4>(dq, P, rows, d0, V, q); break;
        case 8: if constexpr (GM >= 8) corr_var_q<8>(dq, P, rows, d0, V, q); break;
        case 16: if constexpr (GM >= 16) corr_var_q<16>(dq, P, rows, d0, V, q); break;
        case 32: if constexpr (GM >= 32) corr_var_q<32>(dq, P, rows, d0, V, q); break;
        default: V[q] = float(d0); break;  // K = 1
        }
    }
}

// FP64 variance of one coefficient (l, q) for the near-tie decisions:
// this thread's share of sum_(j,j') H_lj H_lj' D(o_j' - o_j, q) over the
// pairs of row l's support; the caller sums the shares.  haar(l, j) gives
// the Haar entry.
template <class HaarF>
__device__ inline double corr_var_part(const FilterArgs& a, const int* org, int K, int l, int q,
                                       HaarF haar, int lane, int nl)
{
    const int P = a.g.P;
    double s = 0.0;
    for (int e = lane; e < K * K; e += nl) {
        const int j = e / K, jp = e - j * K;
        const double w = haar(l, j) * haar(l, jp);
        if (w == 0.0) continue;
        const unsigned r = corr_pair_row(a, corr_member_key(a, org[j]), corr_member_key(a, org[jp]));
        s += w * a.cdtab[int(r) * P + q];
    }
    return s;
}

}  // namespace bmnd
