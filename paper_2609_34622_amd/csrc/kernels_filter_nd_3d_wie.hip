// N-D filter instantiations: 3-D patches of 4^3 samples, Wiener stage
// (the kernel is in filter_nd_impl.h).
#include "filter_nd_impl.h"

namespace bmnd {

hipError_t launch_nd_3d_wie(const FilterArgs& a, const NdBlocks* blk, hipStream_t s)
{
    if (a.gmax == 16) return nd::launch_sh<3, 4, 16, BMND_SHRINK_WIENER>(a, blk, s);
    return nd::launch_sh<3, 4, 32, BMND_SHRINK_WIENER>(a, blk, s);
}

}  // namespace bmnd
