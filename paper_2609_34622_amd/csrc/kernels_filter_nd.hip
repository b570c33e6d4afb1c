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
    return size_t(blk.box_size) * sizeof(double) <= 160u * 1024u;
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
    const long n = long(g.batch) * g.V;
    long grid = (n + 255) / 256;
    if (grid > 65536L * 4) grid = 65536L * 4;
    if (g.j[1] == 4)
        hipLaunchKernelGGL((k_window_conv<3, 4>), dim3(unsigned(grid)), dim3(256), 0, s, g, W, eta,
                           reta, t.f32, t.win[1], t.win[2], t.win[3], n);
    else
        hipLaunchKernelGGL((k_window_conv<2, 8>), dim3(unsigned(grid)), dim3(256), 0, s, g, W, eta,
                           reta, t.f32, t.win[1], t.win[2], t.win[3], n);
    return hipGetLastError();
}

}  // namespace bmnd
