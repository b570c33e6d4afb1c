// Memory-safe reading of origins and group sizes that come from device
// buffers (device code only).
#pragma once

#include "bmnd_internal.h"

namespace bmnd {

// Reference and match lists are read memory-safely whatever they hold: a
// group size is cut to a power of two in [1, gmax] and an origin to
// [0, omax], where omax is the last origin whose patch ends inside the array
// (valid lists are never changed by this).
__device__ __forceinline__ int safe_count(int k, int gmax)
{
    k = min(max(k, 1), gmax);
    return 1 << (31 - __clz(k));
}
__device__ __forceinline__ int safe_origin(int o, int omax) { return min(max(o, 0), omax); }
__device__ __forceinline__ int last_origin(const Geo& g)
{
    int span = 0;
    for (int d = 0; d < kAx; ++d) span += (g.j[d] - 1) * g.st[d];
    return g.V - 1 - span;
}

}  // namespace bmnd
