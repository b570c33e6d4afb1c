// N-D filter dispatch (the kernel is in filter_nd_impl.h, instantiated per
// patch shape and stage) and the overlap-add denominator from per-origin
// weights.
#include <hip/hip_runtime.h>

#include "bmnd_internal.h"
#include "filter_common.h"
#include "filter_nd.h"

namespace bmnd {

hipError_t launch_nd_2d_ht(const FilterArgs& a, const NdBlocks* blk, hipStream_t s);
hipError_t launch_nd_2d_wie(const FilterArgs& a, const NdBlocks* blk, hipStream_t s);
hipError_t launch_nd_3d_ht(const FilterArgs& a, const NdBlocks* blk, hipStream_t s);
hipError_t launch_nd_3d_wie(const FilterArgs& a, const NdBlocks* blk, hipStream_t s);

namespace {

// eta(u) = sum over the patch offsets t of W(u - t) omega(t): the weighted
// overlap-add denominator from the per-origin weights (W is 0 off the
// origins); reta (nullable) receives 1 / eta (0 where eta = 0)
template <int D, int J>
__global__ __launch_bounds__(256) void k_window_conv(Geo g, const double* __restrict__ W,
                                                    double* __restrict__ eta,
                                                    double* __restrict__ reta, const float* win_tab,
                                                    int w1, int w2, int w3, long n)
{
    for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += long(gridDim.x) * blockDim.x) {
        const long vb = (e / g.V) * g.V;
        const int u = int(e - vb);
        int c[kAx];
        int rem = u;
#pragma unroll
        for (int d = kAx - 1; d >= 0; --d) {
            c[d] = rem % g.L[d];
            rem /= g.L[d];
        }
        double s = 0.0;
        if constexpr (D == 2) {
#pragma unroll
            for (int t0 = 0; t0 < J; ++t0) {
                const int o0 = c[kAx - 2] - t0;
                if (o0 < 0 || o0 > g.ell[kAx - 2]) continue;
#pragma unroll
                for (int t1 = 0; t1 < J; ++t1) {
                    const int o1 = c[kAx - 1] - t1;
                    if (o1 < 0 || o1 > g.ell[kAx - 1]) continue;
                    const double wv = W[vb + u - t0 * g.st[kAx - 2] - t1];
                    s += wv * double(win_tab[w2 + t0] * win_tab[w3 + t1]);
                }
            }
        } else {
#pragma unroll
            for (int t0 = 0; t0 < J; ++t0) {
                const int o0 = c[kAx - 3] - t0;
                if (o0 < 0 || o0 > g.ell[kAx - 3]) continue;
#pragma unroll
                for (int t1 = 0; t1 < J; ++t1) {
                    const int o1 = c[kAx - 2] - t1;
                    if (o1 < 0 || o1 > g.ell[kAx - 2]) continue;
#pragma unroll
                    for (int t2 = 0; t2 < J; ++t2) {
                        const int o2 = c[kAx - 1] - t2;
                        if (o2 < 0 || o2 > g.ell[kAx - 1]) continue;
                        const double wv =
                            W[vb + u - t0 * g.st[kAx - 3] - t1 * g.st[kAx - 2] - t2];
                        s += wv * double(win_tab[w1 + t0] * win_tab[w2 + t1] * win_tab[w3 + t2]);
                    }
                }
            }
        }
        eta[e] = s;
        if (reta) reta[e] = s > 0.0 ? 1.0 / s : 0.0;
    }
}

// The same sums from an LDS tile of W: a workgroup of 256 threads takes a
// tile of outputs (4 x 4 x 16 for 3-D, 16 x 16 for 2-D), one per thread,
// and stages W over the tile plus J - 1 samples before it on every patch
// axis (zeros outside the array; W is 0 past the last origin), so each
// output reads its J^D taps from LDS.  The taps are summed in the order of
// k_window_conv (a tap off the origins adds an exact zero), so eta is the
// same bit for bit.
template <int D, int J>
__global__ __launch_bounds__(256) void k_window_conv_tiled(Geo g, const double* __restrict__ W,
                                                          double* __restrict__ eta,
                                                          double* __restrict__ reta,
                                                          const float* win_tab, int w1, int w2,
                                                          int w3, int nt0, int nt1, int nt2)
{
    constexpr int T0 = D == 3 ? 4 : 1, T1 = D == 3 ? 4 : 16, T2 = 16;
    constexpr int H0 = D == 3 ? T0 + J - 1 : 1, H1 = T1 + J - 1, H2 = T2 + J - 1;
    __shared__ double tw[H0 * H1 * H2];
    int rem = int(blockIdx.x);
    const int b2 = rem % nt2;
    rem /= nt2;
    const int b1 = rem % nt1;
    rem /= nt1;
    const int b0 = rem % nt0;
    // the array and its position on the axes before the patch axes (patch
    // extent 1): sub-volumes of the patch axes, one after another
    const int sub = rem / nt0;
    const long vb = long(sub) * (D == 3 ? long(g.st[kAx - 4]) : long(g.st[kAx - 3]));
    const int L0 = D == 3 ? g.L[kAx - 3] : 1, L1 = g.L[kAx - 2], L2 = g.L[kAx - 1];
    const int s0 = D == 3 ? g.st[kAx - 3] : 0, s1 = g.st[kAx - 2];
    const int o0 = b0 * T0 - (H0 - T0), o1 = b1 * T1 - (H1 - T1), o2 = b2 * T2 - (H2 - T2);
    for (int e = threadIdx.x; e < H0 * H1 * H2; e += 256) {
        const int h2 = e % H2, h1 = (e / H2) % H1, h0 = e / (H2 * H1);
        const int x0 = o0 + h0, x1 = o1 + h1, x2 = o2 + h2;
        double v = 0.0;
        if (x0 >= 0 && x0 < L0 && x1 >= 0 && x1 < L1 && x2 >= 0 && x2 < L2)
            v = W[vb + long(x0) * s0 + long(x1) * s1 + x2];
        tw[e] = v;
    }
    __syncthreads();
    const int l2 = threadIdx.x % T2, l1 = (threadIdx.x / T2) % T1, l0 = threadIdx.x / (T2 * T1);
    const int c0 = b0 * T0 + l0, c1 = b1 * T1 + l1, c2 = b2 * T2 + l2;
    if (c0 >= L0 || c1 >= L1 || c2 >= L2) return;
    // position of output (l0, l1, l2) in the tile: offset H - T on every axis
    const int base = ((l0 + H0 - T0) * H1 + (l1 + H1 - T1)) * H2 + (l2 + H2 - T2);
    double sum = 0.0;
    if constexpr (D == 2) {
#pragma unroll
        for (int t0 = 0; t0 < J; ++t0)
#pragma unroll
            for (int t1 = 0; t1 < J; ++t1)
                sum += tw[base - t0 * H2 - t1] * double(win_tab[w2 + t0] * win_tab[w3 + t1]);
    } else {
#pragma unroll
        for (int t0 = 0; t0 < J; ++t0)
#pragma unroll
            for (int t1 = 0; t1 < J; ++t1)
#pragma unroll
                for (int t2 = 0; t2 < J; ++t2)
                    sum += tw[base - (t0 * H1 + t1) * H2 - t2] *
                           double(win_tab[w1 + t0] * win_tab[w2 + t1] * win_tab[w3 + t2]);
    }
    const long e = vb + long(c0) * s0 + long(c1) * s1 + c2;
    eta[e] = sum;
    if (reta) reta[e] = sum > 0.0 ? 1.0 / sum : 0.0;
}

}  // namespace

bool nd_filter_supported(const Geo& g, int gmax, int kex, bool corr, int noise, int shrink)
{
    if (kex > 0 || corr || (gmax != 16 && gmax != 32)) return false;
    if (shrink == BMND_SHRINK_SOFT) return false;
    if (noise != BMND_NOISE_POISSON && noise != BMND_NOISE_GAUSSIAN) return false;
    const bool two = g.j[0] == 1 && g.j[1] == 1 && g.j[2] == 8 && g.j[3] == 8;
    const bool three = g.j[0] == 1 && g.j[1] == 4 && g.j[2] == 4 && g.j[3] == 4;
    return two || three;
}

bool nd_blocks_fit(const NdBlocks& blk)
{
    // the FP64 box of mass conservation within a compute unit's LDS
    return size_t(blk.fbox) * sizeof(double) <= 160u * 1024u;
}

hipError_t launch_filter_nd(const FilterArgs& a, const NdBlocks* blk, hipStream_t s)
{
    const bool three = a.g.j[1] == 4;
    const bool wie = a.shrink == BMND_SHRINK_WIENER;
    if (three) return wie ? launch_nd_3d_wie(a, blk, s) : launch_nd_3d_ht(a, blk, s);
    return wie ? launch_nd_2d_wie(a, blk, s) : launch_nd_2d_ht(a, blk, s);
}

hipError_t launch_window_conv(const Geo& g, const DevTables& t, const double* W, double* eta,
                              double* reta, hipStream_t s)
{
    // tiles of 4 x 4 x 16 (3-D) or 16 x 16 (2-D) outputs
    const bool three = g.j[1] == 4;
    const int nt0 = three ? (g.L[1] + 3) / 4 : 1;
    const int nt1 = three ? (g.L[2] + 3) / 4 : (g.L[2] + 15) / 16;
    const int nt2 = (g.L[3] + 15) / 16;
    long subs = g.batch;   // sub-volumes of the patch axes
    for (int d = 0; d < (three ? 1 : 2); ++d) subs *= g.L[d];
    const long grid = long(nt0) * nt1 * nt2 * subs;
    if (grid <= 0x7fffffffL) {
        if (three)
            hipLaunchKernelGGL((k_window_conv_tiled<3, 4>), dim3(unsigned(grid)), dim3(256), 0, s, g,
                               W, eta, reta, t.f32, t.win[1], t.win[2], t.win[3], nt0, nt1, nt2);
        else
            hipLaunchKernelGGL((k_window_conv_tiled<2, 8>), dim3(unsigned(grid)), dim3(256), 0, s, g,
                               W, eta, reta, t.f32, t.win[1], t.win[2], t.win[3], nt0, nt1, nt2);
        return hipGetLastError();
    }
    const long n = long(g.batch) * g.V;
    long grid1 = (n + 255) / 256;
    if (grid1 > 65536L * 4) grid1 = 65536L * 4;
    if (three)
        hipLaunchKernelGGL((k_window_conv<3, 4>), dim3(unsigned(grid1)), dim3(256), 0, s, g, W, eta,
                           reta, t.f32, t.win[1], t.win[2], t.win[3], n);
    else
        hipLaunchKernelGGL((k_window_conv<2, 8>), dim3(unsigned(grid1)), dim3(256), 0, s, g, W, eta,
                           reta, t.f32, t.win[1], t.win[2], t.win[3], n);
    return hipGetLastError();
}

}  // namespace bmnd
