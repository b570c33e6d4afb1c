// Collaborative filtering for cube patches (extent J per axis, J | 64):
// one wavefront filters one group, in a persistent loop over groups.
//
// A group of K members is a K x P tensor (P = J^D) in the wave's LDS.
// Spatial transform (the same J x J matrix on every axis): each lane owns
// one output row q of the matrix (held in registers) and sweeps the
// fibres of the current innermost axis with 128-bit LDS reads; it writes
// its result with the transformed axis moved to the front of the patch
// axes, so after D passes the layout is back in order and every pass reads
// its axis contiguously.  Haar along the member axis: one lane per patch
// sample, butterflies in registers (orthonormal multilevel Haar, rows:
// scaling, coarsest ... finest detail), block sums for the squared rows.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bmnd_internal.h"
#include "filter_common.h"
#include "exact_planes.h"
#include "corr_noise.h"

namespace bmnd {

namespace {

constexpr int kWave = 64;
constexpr float kRsqrt2 = 0.70710678118654752440f;

// Orders the LDS accesses of one wavefront (its LDS operations complete in
// issue order; this keeps the compiler from moving accesses across).
__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int J>
__device__ __forceinline__ void load_row(const float* __restrict__ M, int q, float* r)
{
#pragma unroll
    for (int t = 0; t < J; ++t) r[t] = M[q * J + t];
}

// One transform pass along the innermost axis of the current layout
// (k, rest, t) -> (k, q, rest).  Each lane sweeps up to NF fibres at once,
// each with two partial sums (even and odd t), so the multiply-adds form
// independent chains instead of one serial chain per fibre.
template <int J, int P>
__device__ __forceinline__ void pass_axis(const float* __restrict__ in, float* __restrict__ out,
                                          const float* row, int K)
{
    constexpr int FPI = kWave / J;   // fibres per sweep step
    constexpr int R = P / J;         // fibres per member
    constexpr int NF = 4;            // fibres per lane per step
    const int lane = threadIdx.x % kWave;
    const int q = lane % J;
    const int fs = lane / J;
    const int F = K * R;
    for (int fb = 0; fb < F; fb += FPI * NF) {
        float se[NF], so[NF];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            se[k] = 0.f;
            so[k] = 0.f;
        }
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const int f = fb + fs + k * FPI;
            if (f < F) {
                const float* x = in + f * J;
                if constexpr (J >= 4) {
#pragma unroll
                    for (int t = 0; t < J; t += 4) {
                        const float4 v = *reinterpret_cast<const float4*>(x + t);
                        se[k] = __builtin_fmaf(row[t], v.x, se[k]);
                        so[k] = __builtin_fmaf(row[t + 1], v.y, so[k]);
                        se[k] = __builtin_fmaf(row[t + 2], v.z, se[k]);
                        so[k] = __builtin_fmaf(row[t + 3], v.w, so[k]);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < J; ++t) se[k] = __builtin_fmaf(row[t], x[t], se[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const int f = fb + fs + k * FPI;
            if (f < F) {
                const int kk = f / R;
                const int rest = f - kk * R;
                out[kk * P + q * R + rest] = se[k] + so[k];
            }
        }
    }
}

// D passes with the same matrix; returns the buffer holding the result.
template <int D, int J, int P>
__device__ __forceinline__ float* spatial(float* x, float* tmp, const float* __restrict__ M, int K)
{
    float row[J];
    load_row<J>(M, threadIdx.x % J, row);
    float* in = x;
    float* out = tmp;
#pragma unroll
    for (int s = 0; s < D; ++s) {
        pass_axis<J, P>(in, out, row, K);
        wsync();
        float* t = in;
        in = out;
        out = t;
    }
    return in;
}

// ---- Haar butterflies on K values held in registers
template <int KK>
__device__ __forceinline__ void haar_fwd(float* r)
{
    float a[KK], o[KK];
#pragma unroll
    for (int i = 0; i < KK; ++i) a[i] = r[i];
    int n = KK;
#pragma unroll
    for (int lev = 0; (1 << lev) < KK; ++lev) {
        const int h = KK >> (lev + 1);
#pragma unroll
        for (int i = 0; i < h; ++i) {
            o[h + i] = (a[2 * i] - a[2 * i + 1]) * kRsqrt2;
            a[i] = (a[2 * i] + a[2 * i + 1]) * kRsqrt2;
        }
        n = h;
    }
    o[0] = a[0];
#pragma unroll
    for (int i = 0; i < KK; ++i) r[i] = o[i];
    (void)n;
}

template <int KK>
__device__ __forceinline__ void haar_inv(float* r)
{
    float a[KK];
    a[0] = r[0];
#pragma unroll
    for (int n = 1; n < KK; n *= 2) {
        float b[KK];
#pragma unroll
        for (int i = 0; i < n; ++i) {
            const float d = r[n + i];
            b[2 * i] = (a[i] + d) * kRsqrt2;
            b[2 * i + 1] = (a[i] - d) * kRsqrt2;
        }
#pragma unroll
        for (int i = 0; i < 2 * n; ++i) a[i] = b[i];
    }
#pragma unroll
    for (int i = 0; i < KK; ++i) r[i] = a[i];
}

// variance through the squared Haar rows: block sums over the row support
template <int KK>
__device__ __forceinline__ void haar_sq(float* r)
{
    float s[KK], o[KK];
#pragma unroll
    for (int i = 0; i < KK; ++i) s[i] = r[i];
    int b = 1;  // members per block
#pragma unroll
    for (int lev = 0; (1 << lev) < KK; ++lev) {
        const int h = KK >> (lev + 1);
        const float inv = 1.f / float(2 * b);
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const float t = s[2 * i] + s[2 * i + 1];
            o[h + i] = t * inv;
            s[i] = t;
        }
        b *= 2;
    }
    o[0] = s[0] / float(KK);
#pragma unroll
    for (int i = 0; i < KK; ++i) r[i] = o[i];
}

// mode 0: forward, 1: inverse, 2: squared
template <int KK, int P>
__device__ __forceinline__ void haar_column(float* X, int p, int mode)
{
    float r[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) r[k] = X[k * P + p];
    if (mode == 0) haar_fwd<KK>(r);
    else if (mode == 1) haar_inv<KK>(r);
    else haar_sq<KK>(r);
#pragma unroll
    for (int k = 0; k < KK; ++k) X[k * P + p] = r[k];
}

// Apply the Haar operator along the member axis to up to three arrays
// (x0 forward, x1 squared, x2 forward; or x0 inverse when `inverse`);
// lanes take (array, sample) pairs.
template <int GM, int P>
__device__ void haar_arrays(float* x0, float* x1, float* x2, int narr, bool inverse, int K)
{
    for (int idx = threadIdx.x % kWave; idx < narr * P; idx += kWave) {
        const int a = idx / P;
        const int p = idx - a * P;
        float* X = a == 0 ? x0 : (a == 1 ? x1 : x2);
        const int mode = inverse ? 1 : (a == 1 ? 2 : 0);
        switch (K) {
        case 2: if constexpr (GM >= 2) haar_column<2, P>(X, p, mode); break;
        case 4: if constexpr (GM >= 4) haar_column<4, P>(X, p, mode); break;
        case 8: if constexpr (GM >= 8) haar_column<8, P>(X, p, mode); break;
        case 16: if constexpr (GM >= 16) haar_column<16, P>(X, p, mode); break;
        case 32: if constexpr (GM >= 32) haar_column<32, P>(X, p, mode); break;
        default: break;  // K = 1: identity
        }
    }
    wsync();
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Haar entry H[l][j] for K members in double precision (same definition as
// the table: scaling row, then detail rows with support K, K/2, ..., 2).
__device__ __forceinline__ double haar64(int K, int l, int j)
{
    if (l == 0) return 1.0 / sqrt(double(K));
    int t = 31 - __clz(l);
    const int support = K >> t;
    const int first = (l - (1 << t)) * support;
    if (j < first || j >= first + support) return 0.0;
    const double v = 1.0 / sqrt(double(support));
    return (j - first) < support / 2 ? v : -v;
}

// Waves per workgroup: up to four groups of K x P <= 512 samples share one
// workgroup; larger groups get fewer waves.
template <int KP>
constexpr int waves_for() { return KP <= 512 ? 4 : (KP <= 1024 ? 2 : 1); }

// VM: variance model, 0 diagonal, 1 with exact shared-source planes,
// 2 stationary correlated Gaussian noise
template <int D, int J, int GM, int VM>
__global__ __launch_bounds__(kWave * waves_for<GM * ipow_c(J, D)>())
void k_filter_cube(FilterArgs a, int chunk_refs)
{
    constexpr bool EXACT = VM == 1;
    constexpr bool CORR = VM == 2;
    constexpr int P = ipow_c(J, D);
    constexpr int KP = GM * P;
    constexpr int NW = waves_for<KP>();
    __shared__ __align__(16) float A_[NW][KP];
    __shared__ __align__(16) float B_[NW][KP];
    __shared__ __align__(16) float V_[NW][KP];
    __shared__ __align__(16) float T_[NW][KP];
    __shared__ int off[P];
    __shared__ float win[P];
    __shared__ int org_[NW][GM];
    __shared__ float rpl_[NW][GM];
    __shared__ float wj_[NW][GM];
    __shared__ int nres_[NW];
    __shared__ unsigned keys_[CORR ? NW : 1][CORR ? GM : 1];

    const Geo& g = a.g;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    float* A = A_[wave];
    float* Bb = B_[wave];
    float* Vb = V_[wave];
    float* Tb = T_[wave];
    int* org = org_[wave];
    float* rpl = rpl_[wave];
    float* wj = wj_[wave];
    int& nres = nres_[wave];

    const int cax = kAx - D;  // first canonical axis of the patch
    const int omax = last_origin(g);
    for (int p = threadIdx.x; p < P; p += kWave * NW) {
        int rem = p, o = 0;
        float w = 1.f;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            const int c = rem % J;
            rem /= J;
            o += c * g.st[cax + d];
            w *= a.t.f32[a.t.win[cax + d] + c];
        }
        off[p] = o;
        win[p] = w;
    }
    const float* Tm = a.t.f32 + a.t.T[kAx - 1];
    const float* T2m = a.t.f32 + a.t.T2[kAx - 1];
    const float* Um = a.t.f32 + a.t.U[kAx - 1];
    const float* rn1 = a.t.f32 + a.t.rn[kAx - 1];
    const double* T64 = a.t.f64 + a.t.T64[kAx - 1];

    // this workgroup: references [g0, g1) of array b
    const int nchunk = (a.n_refs + chunk_refs - 1) / chunk_refs;
    const int b = blockIdx.x / nchunk;
    const int g0 = (blockIdx.x - b * nchunk) * chunk_refs;
    const int g1 = min(a.n_refs, g0 + chunk_refs);
    const long vb = long(b) * g.V;
    __syncthreads();

    for (int gi = g0 + wave; gi < g1; gi += NW) {
        const long grp = long(b) * a.n_refs + gi;
        const int K = safe_count(a.count[grp], a.gmax);
        const int n = K * P;
        const float* yb = a.y + vb;
        const float* pb = a.pilot ? a.pilot + vb : nullptr;
        if (lane < K) {
            org[lane] = safe_origin(a.match[grp * a.gmax + lane], omax);
            rpl[lane] = 0.f;
        }
        if (lane == 0) nres = 0;
        wsync();

        float* res = A;
        if (a.patches_in == nullptr) {
            // ---- gather y, pilot, variance map; group norm
            const bool wiener = a.stage == BMND_STAGE_WIENER;
            const float* mvsrc = wiener ? pb : yb;
            float gn2 = 0.f;
            for (int e = lane; e < n; e += kWave) {
                const int k = e / P;
                const int u = org[k] + off[e - k * P];
                const float yv = yb[u];
                A[e] = yv;
                gn2 = __builtin_fmaf(yv, yv, gn2);
                if (wiener) Bb[e] = pb[u];
                Vb[e] = a.noise == BMND_NOISE_POISSON ? a.s_p * fmaxf(mvsrc[u], 0.f) : a.sigma2;
            }
            const float gn = sqrtf(wave_sum(gn2));
            wsync();

            // ---- forward transforms: spatial passes, then Haar
            float* Y = spatial<D, J, P>(A, Tb, Tm, K);
            if (Y != A) {
                for (int e = lane; e < n; e += kWave) A[e] = Y[e];
                wsync();
            }
            if constexpr (!CORR) {
                float* Vr = spatial<D, J, P>(Vb, Tb, T2m, K);
                if (Vr != Vb) {
                    for (int e = lane; e < n; e += kWave) Vb[e] = Vr[e];
                    wsync();
                }
            }
            if (wiener) {
                float* Gr = spatial<D, J, P>(Bb, Tb, Tm, K);
                if (Gr != Bb) {
                    for (int e = lane; e < n; e += kWave) Bb[e] = Gr[e];
                    wsync();
                }
            }
            haar_arrays<GM, P>(A, Vb, Bb, wiener ? 3 : 2, false, K);
            if constexpr (CORR) {
                // correlated noise: sigma^2 from the variance table; the pair
                // rows live in Tb until the shrinkage reuses it
                int* pix = reinterpret_cast<int*>(Tb);
                if (lane < K) keys_[wave][lane] = corr_member_key(a, org[lane]);
                wsync();
                corr_pair_rows(a, keys_[wave], K, pix, lane, kWave);
                wsync();
                corr_group_variances<GM>(a, pix, K, Vb, lane, kWave);
                wsync();
            }
            // exact shared-source variances of the leading planes
            const int kex = EXACT ? min(a.kex, K) : 0;
            if constexpr (EXACT) {
                exact_plane_variances(a, mvsrc, org, K, kex, Vb, lane, kWave);
                wsync();
            }

            // ---- shrinkage and per-plane risk surrogates
            for (int e = lane; e < n; e += kWave) {
                const int l = e / P;
                const float Yv = A[e];
                const float v = fmaxf(Vb[e], 0.f);
                float att, C;
                if (a.shrink == BMND_SHRINK_HARD) {
                    const float thr = a.lambda * sqrtf(v);
                    const bool keep = fabsf(Yv) > thr;
                    int qq = e - l * P;
                    float rn = 1.f;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        rn *= rn1[qq % J];
                        qq /= J;
                    }
                    // FP32 error band of the decision (transform round-off
                    // is bounded by the row norm times the group norm)
                    const float band = 1e-5f * (rn * gn + thr);
                    if (fabsf(fabsf(Yv) - thr) <= band) {
                        const int slot = atomicAdd(&nres, 1);
                        reinterpret_cast<int*>(Bb)[slot] = e;
                    }
                    att = keep ? 1.f : 0.f;
                    C = Yv;
                } else if (a.shrink == BMND_SHRINK_SOFT) {
                    const float m = fmaxf(fabsf(Yv) - a.lambda * sqrtf(v), 0.f);
                    C = Yv > 0.f ? m : (Yv < 0.f ? -m : 0.f);
                    att = Yv != 0.f ? m / fabsf(Yv) : 0.f;
                } else {
                    const float gam = Bb[e];
                    const float shat = fmaxf(gam * gam - a.power_a * v, 0.f);
                    const float den = shat + a.s_v * v;
                    att = den > 0.f ? shat / den : 0.f;
                    C = att * Yv;
                    Bb[e] = shat;
                }
                A[e] = C;
                Tb[e] = att;
                Vb[e] = v;
            }
            wsync();
            if (a.shrink == BMND_SHRINK_HARD) {
                const int nr = nres;
                for (int r = 0; r < nr; ++r) {
                    const int e = reinterpret_cast<int*>(Bb)[r];
                    const int l = e / P;
                    int q[D];
                    {
                        int qq = e - l * P;
#pragma unroll
                        for (int d = D - 1; d >= 0; --d) {
                            q[d] = qq % J;
                            qq /= J;
                        }
                    }
                    double sy = 0.0, sv = 0.0, sm = 0.0;
                    for (int f = lane; f < n; f += kWave) {
                        const int j = f / P;
                        const int i = f - j * P;
                        double w = haar64(K, l, j);
                        int ii = i;
#pragma unroll
                        for (int d = D - 1; d >= 0; --d) {
                            w *= T64[q[d] * J + ii % J];
                            ii /= J;
                        }
                        const int u = org[j] + off[i];
                        sy += w * double(yb[u]);
                        sm += fabs(w * double(yb[u]));
                        const double mv = a.noise == BMND_NOISE_POISSON
                                              ? a.s_p64 * fmax(double(yb[u]), 0.0)
                                              : a.sigma2_64;
                        sv += w * w * mv;
                    }
                    if constexpr (CORR)
                        sv = corr_var_part(a, org, K, l, e - l * P,
                                           [&](int r, int j) { return haar64(K, r, j); }, lane,
                                           kWave);
                    if constexpr (EXACT) {
                        if (l < kex) sv = exact_partial(a, yb, org, K, l, e - l * P, lane, kWave);
                    }
                    sy = wave_sum64(sy);
                    sv = wave_sum64(sv);
                    sm = wave_sum64(sm);
                    // strict inequality with the 1e-9 relative tie margin; with
                    // zero variance, coefficients up to 1e-9 of the magnitude
                    // of their terms are rounding residues of exact zeros
                    const bool keep = sv > 0.0 ? fabs(sy) > a.lambda64 * sqrt(sv) * (1.0 + 1e-9)
                                               : fabs(sy) > 1e-9 * sm;
                    if (lane == 0) Tb[e] = keep ? 1.f : 0.f;
                    wsync();
                }
                for (int e = lane; e < n; e += kWave)
                    if (Tb[e] == 0.f) A[e] = 0.f;
                wsync();
            }
            for (int e = lane; e < n; e += kWave) {
                const int l = e / P;
                const float at = Tb[e];
                const float v = Vb[e];
                float r;
                if (a.wmodel == BMND_WEIGHT_CLASSIC) r = at * at;
                else if (a.wmodel == BMND_WEIGHT_VARIANCE) r = at * at * v;
                else r = at * at * v + (1.f - at) * (1.f - at) * Bb[e];
                if (a.wdomain == BMND_WDOMAIN_WINDOWED) r *= window_metric(a, e - l * P);
                atomicAdd(&rpl[l], r);
            }
            wsync();
            if (a.wscope == BMND_SCOPE_GROUP) {
                float R = 0.f;
                for (int l = 0; l < K; ++l) R += rpl[l];
                if (lane < K) wj[lane] = R > 0.f ? 1.f / R : 1.f;
            } else if (lane < K) {
                // R_j = sum_l H[l][j]^2 r_l
                float R = 0.f;
                for (int l = 0; l < K; ++l) {
                    const float h = float(haar64(K, l, lane));
                    R += h * h * rpl[l];
                }
                wj[lane] = R > 0.f ? 1.f / R : 1.f;
            }
            wsync();

            // ---- synthesis: Haar^T, then U along every axis
            haar_arrays<GM, P>(A, nullptr, nullptr, 1, true, K);
            res = spatial<D, J, P>(A, Tb, Um, K);
        } else {
            const float* pin = a.patches_in + grp * long(a.gmax) * P;
            for (int e = lane; e < n; e += kWave) A[e] = pin[e];
            if (lane < K) wj[lane] = a.weights_in[grp * a.gmax + lane];
            wsync();
        }

        // ---- outputs
        if (a.out_mode == 0) {
            float* pout = a.patches + grp * long(a.gmax) * P;
            for (int e = lane; e < a.gmax * P; e += kWave) pout[e] = e < n ? res[e] : 0.f;
            if (lane < a.gmax) a.weights[grp * a.gmax + lane] = lane < K ? wj[lane] : 0.f;
        } else if (a.out_mode == 1) {
            for (int e = lane; e < n; e += kWave) {
                const int k = e / P;
                const int p = e - k * P;
                const long u = vb + org[k] + off[p];
                // FP64 sums: the float result does not depend on the order
                const float ww = wj[k] * win[p];
                unsafeAtomicAdd(&a.numd[u], double(ww * res[e]));
                unsafeAtomicAdd(&a.dend[u], double(ww));
            }
        } else if (a.out_mode == 2) {
            for (int e = lane; e < n; e += kWave) {
                const int k = e / P;
                const int p = e - k * P;
                const long u = vb + org[k] + off[p];
                unsafeAtomicAdd(&a.dend[u], double(wj[k]) * double(win[p]));
            }
        } else {
            double zs = 0.0, zr = 0.0;
            for (int e = lane; e < n; e += kWave) {
                const int k = e / P;
                const int p = e - k * P;
                const long u = vb + org[k] + off[p];
                const double zeta = double(wj[k]) * double(win[p]) / a.dend[u];
                zs += zeta;
                zr += zeta * (double(a.y[u]) - double(res[e]));
            }
            zs = wave_sum64(zs);
            zr = wave_sum64(zr);
            const double alpha = zs > 0.0 ? zr / zs : 0.0;
            for (int e = lane; e < n; e += kWave) {
                const int k = e / P;
                const int p = e - k * P;
                const long u = vb + org[k] + off[p];
                unsafeAtomicAdd(&a.numd[u],
                                double(wj[k]) * double(win[p]) * (double(res[e]) + alpha));
            }
        }
        wsync();
    }

}

template <int D, int J>
hipError_t launch_cube_gm(const FilterArgs& a, int step_last, hipStream_t s)
{
    // references per workgroup: up to 256, fewer for small arrays so that
    // the launch still fills the device
    const Geo& g = a.g;
    const long groups = long(a.n_refs) * g.batch;
    const int chunk = int(std::max(1L, std::min(256L, groups / 8192)));
    const int nchunk = (a.n_refs + chunk - 1) / chunk;
    const dim3 grid(unsigned(long(nchunk) * g.batch));
#define BMND_CUBE_LAUNCH(GMV)                                                              \
    if (a.cdtab)                                                                            \
        hipLaunchKernelGGL((k_filter_cube<D, J, GMV, 2>),                                   \
                           dim3(grid), dim3(kWave * waves_for<GMV * ipow_c(J, D)>()), 0, s, a, \
                           chunk);                                                          \
    else if (a.kex > 0)                                                                     \
        hipLaunchKernelGGL((k_filter_cube<D, J, GMV, 1>),                                   \
                           dim3(grid), dim3(kWave * waves_for<GMV * ipow_c(J, D)>()), 0, s, a, \
                           chunk);                                                          \
    else                                                                                    \
    hipLaunchKernelGGL((k_filter_cube<D, J, GMV, 0>),                                       \
                       dim3(grid), dim3(kWave * waves_for<GMV * ipow_c(J, D)>()), 0, s, a, \
                       chunk)
    switch (a.gmax) {
    case 1: BMND_CUBE_LAUNCH(1); break;
    case 2: BMND_CUBE_LAUNCH(2); break;
    case 4: BMND_CUBE_LAUNCH(4); break;
    case 8: BMND_CUBE_LAUNCH(8); break;
    case 16: BMND_CUBE_LAUNCH(16); break;
    default: BMND_CUBE_LAUNCH(32); break;
    }
#undef BMND_CUBE_LAUNCH
    return hipGetLastError();
}

}  // namespace

bool cube_filter_supported(const Geo& g, int gmax)
{
    int D = 0, J = 0;
    for (int d = 0; d < kAx; ++d) {
        if (g.j[d] == 1 && D == 0) continue;
        if (J == 0) J = g.j[d];
        if (g.j[d] != J) return false;
        ++D;
    }
    if (D == 0) return false;
    const bool shape_ok = (D == 1 && J == 32) || (D == 2 && J == 8) || (D == 3 && J == 4);
    return shape_ok && gmax * g.P <= kMaxKP && g.P * gmax * 16 <= 65536;
}

hipError_t launch_filter_cube(const FilterArgs& a, int step_last, hipStream_t s)
{
    const Geo& g = a.g;
    if (g.P == 32) return launch_cube_gm<1, 32>(a, step_last, s);
    if (g.j[kAx - 1] == 8) return launch_cube_gm<2, 8>(a, step_last, s);
    return launch_cube_gm<3, 4>(a, step_last, s);
}

}  // namespace bmnd
