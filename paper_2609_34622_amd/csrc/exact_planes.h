// Exact noise variances of the leading Haar planes (Def. effective transform
// weights, Def. partial shared-source Poisson variance model).
//
// Members of a group may share voxels; the diagonal propagation treats
// every group entry as independent, the exact planes combine the entries
// that come from one voxel before squaring.  For plane l and spatial
// coefficient q, with T_q(i) = prod_d T_d[q_d][i_d] and the variance map m,
//   sigma2[l][q] = sum_u ( sum_{(j,i): org_j + i = u} H[l][j] T_q(i) )^2 m(u)
//                = sum_{j, j'} H[l][j] H[l][j'] G_q(j, j'),
//   G_q(j, j')   = sum over the voxels u that members j and j' share of
//                  T_q(u - org_j) T_q(u - org_j') m(u).
// Two members share voxels only if their origins differ by less than the
// patch extent on every axis; G_q(j, j) is the diagonal term.  Everything
// is evaluated in FP64.  Device code only.
#pragma once

#include "filter_common.h"

namespace bmnd {

// Haar entry H[l][j] for K = 2^lk members (rows: scaling, then detail rows
// with support K, K/2, ..., 2), in double precision.
__device__ __forceinline__ double exact_haar(int K, int l, int j)
{
    if (l == 0) return 1.0 / sqrt(double(K));
    const int t = 31 - __clz(l);
    const int support = K >> t;
    const int first = (l - (1 << t)) * support;
    if (j < first || j >= first + support) return 0.0;
    const double v = 1.0 / sqrt(double(support));
    return (j - first) < support / 2 ? v : -v;
}

// coordinates of a lin on the canonical axes
__device__ __forceinline__ void exact_coords(const Geo& g, int lin, int* c)
{
#pragma unroll
    for (int d = kAx - 1; d >= 0; --d) {
        c[d] = lin % g.L[d];
        lin /= g.L[d];
    }
}

// the p-th pair (j <= j') of K members, row by row
__device__ __forceinline__ void exact_pair(int p, int K, int* j, int* jp)
{
    int r = 0;
    while (p >= K - r) {
        p -= K - r;
        ++r;
    }
    *j = r;
    *jp = r + p;
}

// G_q(j, j') for spatial coefficient q (per-axis indices qd); cj, cjp are the
// members' origin coordinates.  Returns 0 when the members share no voxel.
__device__ inline double exact_gram(const FilterArgs& a, const float* msrc, int oj, const int* cj,
                                    const int* cjp, const int* qd)
{
    const Geo& g = a.g;
    int lo[kAx], hi[kAx], dl[kAx];
#pragma unroll
    for (int d = 0; d < kAx; ++d) {
        dl[d] = cjp[d] - cj[d];
        lo[d] = max(0, dl[d]);
        hi[d] = min(g.j[d], g.j[d] + dl[d]);
        if (lo[d] >= hi[d]) return 0.0;
    }
    const double* T0 = a.t.f64 + a.t.T64[0] + qd[0] * g.j[0];
    const double* T1 = a.t.f64 + a.t.T64[1] + qd[1] * g.j[1];
    const double* T2 = a.t.f64 + a.t.T64[2] + qd[2] * g.j[2];
    const double* T3 = a.t.f64 + a.t.T64[3] + qd[3] * g.j[3];
    const bool poisson = a.noise == BMND_NOISE_POISSON;
    double s = 0.0;
    for (int i0 = lo[0]; i0 < hi[0]; ++i0) {
        const double w0 = T0[i0] * T0[i0 - dl[0]];
        for (int i1 = lo[1]; i1 < hi[1]; ++i1) {
            const double w1 = w0 * T1[i1] * T1[i1 - dl[1]];
            for (int i2 = lo[2]; i2 < hi[2]; ++i2) {
                const double w2 = w1 * T2[i2] * T2[i2 - dl[2]];
                const int ub = oj + i0 * g.st[0] + i1 * g.st[1] + i2 * g.st[2];
                for (int i3 = lo[3]; i3 < hi[3]; ++i3) {
                    const double w3 = w2 * T3[i3] * T3[i3 - dl[3]];
                    const double m = poisson ? a.s_p64 * fmax(double(msrc[ub + i3]), 0.0)
                                             : a.sigma2_64;
                    s += w3 * m;
                }
            }
        }
    }
    return s;
}

// This thread's share (pairs t, t + nt, ...) of sigma2[l][q] for one plane
// and one spatial coefficient; the caller sums the shares.
__device__ inline double exact_partial(const FilterArgs& a, const float* msrc, const int* org,
                                       int K, int l, int qidx, int t, int nt)
{
    const Geo& g = a.g;
    int qd[kAx];
    {
        int r = qidx;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            qd[d] = r % g.j[d];
            r /= g.j[d];
        }
    }
    const int npairs = K * (K + 1) / 2;
    double acc = 0.0;
    for (int p = t; p < npairs; p += nt) {
        int j, jp;
        exact_pair(p, K, &j, &jp);
        const double h = exact_haar(K, l, j) * exact_haar(K, l, jp);
        if (h == 0.0) continue;
        int cj[kAx], cjp[kAx];
        exact_coords(g, org[j], cj);
        exact_coords(g, org[jp], cjp);
        const double G = exact_gram(a, msrc, org[j], cj, cjp, qd);
        acc += (j == jp ? 1.0 : 2.0) * h * G;
    }
    return acc;
}

// sigma2[l][q] for all planes l < L and coefficients q, written as float to
// V[l * P + q]; threads t = 0 .. nt-1 take coefficients q = t, t + nt, ...
__device__ inline void exact_plane_variances(const FilterArgs& a, const float* msrc,
                                             const int* org, int K, int L, float* V, int t,
                                             int nt)
{
    const Geo& g = a.g;
    const int P = g.P;
    constexpr int kChunkPlanes = 8;
    for (int q = t; q < P; q += nt) {
        int qd[kAx];
        {
            int r = q;
#pragma unroll
            for (int d = kAx - 1; d >= 0; --d) {
                qd[d] = r % g.j[d];
                r /= g.j[d];
            }
        }
        for (int l0 = 0; l0 < L; l0 += kChunkPlanes) {
            double acc[kChunkPlanes];
#pragma unroll
            for (int k = 0; k < kChunkPlanes; ++k) acc[k] = 0.0;
            for (int j = 0; j < K; ++j) {
                int cj[kAx];
                exact_coords(g, org[j], cj);
                for (int jp = j; jp < K; ++jp) {
                    int cjp[kAx];
                    exact_coords(g, org[jp], cjp);
                    const double G = exact_gram(a, msrc, org[j], cj, cjp, qd);
                    if (G == 0.0) continue;
                    const double c = j == jp ? G : 2.0 * G;
#pragma unroll
                    for (int k = 0; k < kChunkPlanes; ++k)
                        if (l0 + k < L) acc[k] += c * exact_haar(K, l0 + k, j) * exact_haar(K, l0 + k, jp);
                }
            }
#pragma unroll
            for (int k = 0; k < kChunkPlanes; ++k)
                if (l0 + k < L) V[(l0 + k) * P + q] = float(acc[k]);
        }
    }
}

}  // namespace bmnd
