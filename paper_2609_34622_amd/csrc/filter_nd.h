// Spatial blocks of reference origins for the N-D filter's LDS overlap-add
// boxes (kernels_filter_nd.hip).
#pragma once

#include "bmnd_internal.h"

namespace bmnd {

// References grouped by block: block c (C-order over nb) holds the origins
// r with floor(r_d / B_d) = c_d on every canonical axis, list positions
// start[c] .. start[c + 1] - 1.  The box of a block spans, per axis, the
// block, the search window and a patch: E_d = B_d + W_d + j_d - 2 samples
// from c_d B_d - floor(W_d / 2); S_d are its C-order strides.
struct NdBlocks {
    const int* start = nullptr;  // [nblocks + 1] (device)
    int nblocks = 0;
    int nb[kAx] = {1, 1, 1, 1};
    int B[kAx] = {1, 1, 1, 1};
    int E[kAx] = {1, 1, 1, 1};
    int S[kAx] = {1, 1, 1, 1};
    int box_size = 0;
    // The matcher's LDS copies of the same box: 32-bit samples at strides
    // MS (mbox words in all), and four byte copies of counts at strides MSb
    // (mbox_b bytes each, copy c at byte c * mcst).  Rows and planes are
    // padded so that the wavefront's lanes, one run of candidates each,
    // read distinct LDS banks (see nd_match_layout).
    int MS[kAx] = {1, 1, 1, 1};
    int MSb[kAx] = {1, 1, 1, 1};
    int mbox = 0;
    int mbox_b = 0;
    int mcst = 0;
    // The filter's FP64 numerator box: extents FE (E without the last
    // axis's rounding to 4) at strides FS (fbox doubles in all), rows and
    // planes padded so that the members of a group, whose patches are added
    // one sample at a time, fall on distinct LDS banks as often as possible
    // (see nd_filter_layout)
    int FE[kAx] = {1, 1, 1, 1};
    int FS[kAx] = {1, 1, 1, 1};
    int fbox = 0;
};

struct FilterArgs;
bool nd_filter_supported(const Geo& g, int gmax, int kex, bool corr, int noise, int shrink);
// whether the blocks' boxes fit a compute unit's LDS (else the older filter runs)
bool nd_blocks_fit(const NdBlocks& blk);
hipError_t launch_filter_nd(const FilterArgs& a, const NdBlocks* blk, hipStream_t s);
// eta = W convolved with the patch window (the overlap-add denominator from
// the per-origin weights W), and 1 / eta into reta when it is not null
hipError_t launch_window_conv(const Geo& g, const DevTables& t, const double* W, double* eta,
                              double* reta, hipStream_t s);

// Rules for the size of a spatial block of references: blocks grow by 3
// lattice positions, innermost axis first, while the box stays within
// box_cap samples and a block holds at most max(refs_floor, refs *
// batch / min_blocks) references.  Rule 0 is the default; the others are
// the autotuner's candidates.
struct BlockRule {
    long box_cap;
    long min_blocks;
    long refs_floor;
};
constexpr BlockRule kBlockRules[] = {
    {9216, 2048, 16}, {4096, 2048, 16}, {6144, 2048, 16}, {12288, 2048, 16},
    {9216, 512, 64},  {16384, 1024, 32},
};
constexpr int kNumBlockRules = int(sizeof(kBlockRules) / sizeof(kBlockRules[0]));

// Host: block sizes for a geometry under block rule `rule` and the block
// order of a sorted origin list (refs_out: the origins in block order,
// start: block offsets).
void nd_make_blocks(const Geo& g, const std::vector<int64_t>& refs, int rule,
                    std::vector<int64_t>& refs_out, std::vector<int>& start, NdBlocks& blk);

// Host: the filter's padded box strides (FS, fbox); nd_make_blocks calls it.
void nd_filter_layout(const Geo& g, NdBlocks& blk);

// Host: the matcher's padded LDS layouts of a block's box (MS, MSb, mbox,
// mbox_b, mcst) for the geometry's window and patch; nd_make_blocks calls it.
void nd_match_layout(const Geo& g, NdBlocks& blk);

}  // namespace bmnd
