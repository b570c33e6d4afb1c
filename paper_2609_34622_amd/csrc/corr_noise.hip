// Stationary correlated Gaussian noise: the device tables derived from the
// power spectral density (section Observation Models: Def. wide-sense
// stationary Gaussian noise and the discrete Wiener-Khinchin relation
// c = ifftn(S) / |Omega|; Prop. Gaussian SSD noise bias; Lemma covariance
// propagation).
//
// Only the displacements the method uses are needed: |tau_d| <= R_d, the
// largest member displacement of a search window plus a patch offset.  The
// autocovariance over that box is a separable partial inverse DFT, one axis
// at a time (last axis first), each output a plain sum over the axis'
// frequencies with exact twiddles e^(2 pi i k / L) from a table, in FP64.
// The per-stage variance table D(Delta, q) then sums the autocorrelation of
// the spatial transform's rows against c.
#include <hip/hip_runtime.h>

#include "bmnd_internal.h"

namespace bmnd {

namespace {

constexpr int kThreads = 256;

__global__ void k_corr_twiddle(double2* __restrict__ tw, int L)
{
    const int k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= L) return;
    double s, c;
    sincospi(2.0 * double(k) / double(L), &s, &c);
    tw[k] = make_double2(c, s);
}

struct DftPass {
    int in[kAx];    // input extents
    int out[kAx];   // output extents (out[axis] = 2 R + 1)
    int axis, L, R;
    double scale;   // applied to the real part of the final pass
};

// out[.., t, ..] = sum_w in[.., w, ..] e^(2 pi i w (t - R) / L) along `axis`.
// The first pass reads the real spectrum (inr), later ones complex data;
// the final pass writes scale * Re(.) to outr.
__global__ void k_corr_dft(const double* __restrict__ inr, const double2* __restrict__ inc,
                           const double2* __restrict__ tw, double2* __restrict__ outc,
                           double* __restrict__ outr, DftPass p, long nout)
{
    const long e = long(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= nout) return;
    int co[kAx];
    long rem = e;
#pragma unroll
    for (int d = kAx - 1; d >= 0; --d) {
        co[d] = int(rem % p.out[d]);
        rem /= p.out[d];
    }
    long base = 0, stride = 1, sax = 1;
#pragma unroll
    for (int d = kAx - 1; d >= 0; --d) {
        if (d == p.axis) sax = stride;
        else base += long(co[d]) * stride;
        stride *= p.in[d];
    }
    const int tau = co[p.axis] - p.R;
    int tm = tau % p.L;
    if (tm < 0) tm += p.L;
    double re = 0.0, im = 0.0;
    int k = 0;
    for (int w = 0; w < p.L; ++w) {
        const double2 t = tw[k];
        const long i = base + long(w) * sax;
        if (inr) {
            const double v = inr[i];
            re = fma(v, t.x, re);
            im = fma(v, t.y, im);
        } else {
            const double2 v = inc[i];
            re = fma(v.x, t.x, fma(-v.y, t.y, re));
            im = fma(v.x, t.y, fma(v.y, t.x, im));
        }
        k += tm;
        if (k >= p.L) k -= p.L;
    }
    if (outr) outr[e] = re * p.scale;
    else outc[e] = make_double2(re, im);
}

struct DtabArgs {
    int Bc[kAx], R[kAx];   // autocovariance box and its centre
    int j[kAx], bw[kAx];   // patch extents, member box extents
    int P;
    const double* ac[kAx]; // row autocorrelations, j x (2 j - 1) per axis
    long n;                // box rows * P
};

// D(Delta, q) = sum_tau A_q(tau) c(Delta + tau), A_q = prod_d A^d_(q_d).
__global__ void k_corr_dtab(const double* __restrict__ cbox, DtabArgs t, double* __restrict__ dtab)
{
    const long e = long(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= t.n) return;
    const int bi = int(e / t.P);
    int q = int(e - long(bi) * t.P);
    int dl[kAx], qd[kAx];
    int rem = bi;
#pragma unroll
    for (int d = kAx - 1; d >= 0; --d) {
        dl[d] = rem % t.bw[d] - (t.bw[d] - 1) / 2;
        rem /= t.bw[d];
        qd[d] = q % t.j[d];
        q /= t.j[d];
    }
    int cst[kAx];
    {
        int s = 1;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            cst[d] = s;
            s *= t.Bc[d];
        }
    }
    const double* a0 = t.ac[0] + qd[0] * (2 * t.j[0] - 1);
    const double* a1 = t.ac[1] + qd[1] * (2 * t.j[1] - 1);
    const double* a2 = t.ac[2] + qd[2] * (2 * t.j[2] - 1);
    const double* a3 = t.ac[3] + qd[3] * (2 * t.j[3] - 1);
    double sum = 0.0;
    for (int t0 = 1 - t.j[0]; t0 < t.j[0]; ++t0) {
        const double w0 = a0[t0 + t.j[0] - 1];
        const int c0 = (dl[0] + t0 + t.R[0]) * cst[0];
        for (int t1 = 1 - t.j[1]; t1 < t.j[1]; ++t1) {
            const double w1 = w0 * a1[t1 + t.j[1] - 1];
            const int c1 = c0 + (dl[1] + t1 + t.R[1]) * cst[1];
            for (int t2 = 1 - t.j[2]; t2 < t.j[2]; ++t2) {
                const double w2 = w1 * a2[t2 + t.j[2] - 1];
                const int c2 = c1 + (dl[2] + t2 + t.R[2]) * cst[2];
                for (int t3 = 1 - t.j[3]; t3 < t.j[3]; ++t3) {
                    const double w3 = w2 * a3[t3 + t.j[3] - 1];
                    sum = fma(w3, cbox[c2 + dl[3] + t3 + t.R[3]], sum);
                }
            }
        }
    }
    dtab[e] = sum;
}

struct BiasArgs {
    int Bc[kAx], R[kAx], W[kAx];
    int P;
    double gamma;
    long n;   // window offsets
};

// bias(o) = gamma 2 P (c(0) - c(Delta)), Delta_d = o_d - floor(W_d / 2);
// offsets beyond the autocovariance box are never a candidate (they leave
// the array) and get 0.  One workgroup also writes max |bias|.
__global__ void k_corr_bias(const double* __restrict__ cbox, BiasArgs t, double* __restrict__ b64,
                            float* __restrict__ b32, double* __restrict__ bound)
{
    __shared__ double red[kThreads];
    int cst[kAx];
    long centre = 0;
    {
        int s = 1;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            cst[d] = s;
            centre += long(t.R[d]) * s;
            s *= t.Bc[d];
        }
    }
    const double c0 = cbox[centre];
    double mx = 0.0;
    for (long e = threadIdx.x; e < t.n; e += kThreads) {
        long rem = e, idx = 0;
        bool inside = true;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            const int dl = int(rem % t.W[d]) - t.W[d] / 2;
            rem /= t.W[d];
            inside = inside && dl >= -t.R[d] && dl <= t.R[d];
            idx += long(dl + t.R[d]) * cst[d];
        }
        const double b = inside ? t.gamma * (2.0 * double(t.P) * (c0 - cbox[idx])) : 0.0;
        b64[e] = b;
        b32[e] = float(b);
        mx = fmax(mx, fabs(b));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *bound = red[0];
}

unsigned grid_of(long n) { return unsigned((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_corr_autocov(const double* psd, const int L[kAx], const int R[kAx], double2* tw,
                               double2* x0, double2* x1, double* cbox, hipStream_t s)
{
    long V = 1;
    for (int d = 0; d < kAx; ++d) V *= L[d];
    int cur[kAx];
    for (int d = 0; d < kAx; ++d) cur[d] = L[d];
    int last = -1;  // the final pass transforms the first non-trivial axis
    for (int d = 0; d < kAx && last < 0; ++d)
        if (L[d] > 1) last = d;
    if (last < 0) last = kAx - 1;
    const double2* inc = nullptr;
    const double* inr = psd;
    double2* bufs[2] = {x0, x1};
    int nb = 0;
    for (int axis = kAx - 1; axis >= 0; --axis) {
        if (L[axis] == 1 && axis != last) continue;
        hipLaunchKernelGGL(k_corr_twiddle, dim3(grid_of(L[axis])), dim3(kThreads), 0, s, tw,
                           L[axis]);
        DftPass p{};
        for (int d = 0; d < kAx; ++d) {
            p.in[d] = cur[d];
            p.out[d] = cur[d];
        }
        p.axis = axis;
        p.L = L[axis];
        p.R = R[axis];
        p.out[axis] = 2 * R[axis] + 1;
        p.scale = 1.0 / (double(V) * double(V));
        long nout = 1;
        for (int d = 0; d < kAx; ++d) nout *= p.out[d];
        const bool final = axis == last;
        double2* oc = final ? nullptr : bufs[nb];
        hipLaunchKernelGGL(k_corr_dft, dim3(grid_of(nout)), dim3(kThreads), 0, s, inr, inc, tw, oc,
                           final ? cbox : nullptr, p, nout);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (final) break;
        inr = nullptr;
        inc = oc;
        nb ^= 1;
        cur[axis] = p.out[axis];
    }
    return hipGetLastError();
}

hipError_t launch_corr_dtab(const double* cbox, const int Bc[kAx], const int R[kAx],
                            const int j[kAx], const int bw[kAx], int P,
                            const double* const ac[kAx], double* dtab, hipStream_t s)
{
    DtabArgs t{};
    long rows = 1;
    for (int d = 0; d < kAx; ++d) {
        t.Bc[d] = Bc[d];
        t.R[d] = R[d];
        t.j[d] = j[d];
        t.bw[d] = bw[d];
        t.ac[d] = ac[d];
        rows *= bw[d];
    }
    t.P = P;
    t.n = rows * P;
    hipLaunchKernelGGL(k_corr_dtab, dim3(grid_of(t.n)), dim3(kThreads), 0, s, cbox, t, dtab);
    return hipGetLastError();
}

hipError_t launch_corr_bias(const double* cbox, const int Bc[kAx], const int R[kAx],
                            const int W[kAx], int P, double gamma, double* b64, float* b32,
                            double* bound, hipStream_t s)
{
    BiasArgs t{};
    long n = 1;
    for (int d = 0; d < kAx; ++d) {
        t.Bc[d] = Bc[d];
        t.R[d] = R[d];
        t.W[d] = W[d];
        n *= W[d];
    }
    t.P = P;
    t.gamma = gamma;
    t.n = n;
    hipLaunchKernelGGL(k_corr_bias, dim3(1), dim3(kThreads), 0, s, cbox, t, b64, b32, bound);
    return hipGetLastError();
}

}  // namespace bmnd
