// N-D filter instantiations: 2-D patches of 8^2 samples, hard-threshold stage
// (the kernel is in filter_nd_impl.h).
#include "filter_nd_impl.h"

namespace bmnd {

hipError_t launch_nd_2d_ht(const FilterArgs& a, const NdBlocks* blk, hipStream_t s)
{
    if (a.gmax == 16) return nd::launch_sh<2, 8, 16, BMND_SHRINK_HARD>(a, blk, s);
    return nd::launch_sh<2, 8, 32, BMND_SHRINK_HARD>(a, blk, s);
}

}  // namespace bmnd
