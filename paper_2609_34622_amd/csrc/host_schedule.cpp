// Reference-origin schedules (section Reference-Patch Schedule).
//
// The coarse lattice of axis d has Z_d = ceil(ell_d / h_d) + 1 slots with
// nominal origins min(q h, ell) (Def. clipped reference origin).  Each of
// the K_s passes gives every slot tuple one offset vector o; the origin is
// clip(min(q h, ell) - o, 0, ell) per axis, and the last slot is pinned to
// ell.  Offsets come from the per-axis candidate shift list (eq.
// number-shifts, eq. candidate-shift-list), indexed by the rule of the
// selected schedule (Defs. generated / balanced / sparse / off).
#include <algorithm>
#include <cstdint>
#include <cmath>

#include "bmnd_internal.h"
#include "filter_nd.h"

namespace bmnd {

namespace {

// Rounded, uniformly spaced samples of [0, j - 1]; n = min(j, max(1,
// ceil(rho (j - 1) / h))).  Rounding floor(x + 1/2) is done on the exact
// rational i (j - 1) / (n - 1).
std::vector<int64_t> shift_candidates(int j, int h, double rho)
{
    double want = std::ceil(rho * double(j - 1) / double(h));
    int64_t n = want < 1.0 ? 1 : int64_t(want);
    n = std::min<int64_t>(n, j);
    std::vector<int64_t> s(size_t(n), 0);
    for (int64_t i = 1; i < n; ++i) {
        const int64_t num = i * (j - 1);  // value = num / (n - 1)
        const int64_t den = n - 1;
        s[size_t(i)] = (2 * num + den) / (2 * den);
    }
    return s;
}

}  // namespace

std::vector<int64_t> reference_origins(const bmnd_geometry& geom, const bmnd_stage_params& sp)
{
    const int D = geom.ndim;
    std::vector<int64_t> ell(D), Z(D), stride(D);
    std::vector<std::vector<int64_t>> S(D);
    int64_t acc = 1;
    for (int d = D - 1; d >= 0; --d) {
        stride[d] = acc;
        acc *= geom.shape[d];
    }
    for (int d = 0; d < D; ++d) {
        ell[d] = geom.shape[d] - sp.patch[d];
        Z[d] = (ell[d] + sp.step[d] - 1) / sp.step[d] + 1;
        S[d] = shift_candidates(sp.patch[d], sp.step[d], sp.shift_density);
    }
    // next active axis for the sparse schedule (active: Z_d > 1 or j_d > 1)
    std::vector<int> next_active(D, -1);
    for (int d = D - 1, nxt = -1; d >= 0; --d) {
        next_active[d] = nxt;
        if (Z[d] > 1 || sp.patch[d] > 1) nxt = d;
    }
    std::vector<int64_t> slot_origin_cache;
    const int passes = sp.schedule == BMND_SCHED_OFF ? 1 : sp.passes;

    std::vector<int64_t> out;
    int64_t tuples = 1;
    for (int d = 0; d < D; ++d) tuples *= Z[d];
    out.reserve(size_t(tuples * passes));
    std::vector<int64_t> q(D, 0);
    for (int64_t t = 0; t < tuples; ++t) {
        int64_t qsum = 0;
        for (int d = 0; d < D; ++d) qsum += q[d];
        for (int k = 0; k < passes; ++k) {
            int64_t lin = 0;
            for (int d = 0; d < D; ++d) {
                const auto& Sd = S[d];
                const int64_t n = int64_t(Sd.size());
                int64_t off = 0;
                if (sp.schedule == BMND_SCHED_GENERATED) {
                    if (d + 1 < D) off = Sd[size_t((q[d + 1] + k) % n)];
                } else if (sp.schedule == BMND_SCHED_BALANCED) {
                    off = Sd[size_t((k + qsum - q[d]) % n)];
                } else if (sp.schedule == BMND_SCHED_SPARSE) {
                    const bool act = Z[d] > 1 || sp.patch[d] > 1;
                    if (act && next_active[d] >= 0) off = Sd[size_t((q[next_active[d]] + k) % n)];
                }
                int64_t r;
                if (q[d] == Z[d] - 1) {
                    r = ell[d];
                } else {
                    r = std::min<int64_t>(q[d] * sp.step[d], ell[d]) - off;
                    r = std::max<int64_t>(0, std::min<int64_t>(r, ell[d]));
                }
                lin += r * stride[d];
            }
            out.push_back(lin);
        }
        // advance the slot tuple (last axis fastest)
        for (int d = D - 1; d >= 0; --d) {
            if (++q[d] < Z[d]) break;
            q[d] = 0;
        }
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
}

// Spatial blocks for the N-D filter's overlap-add boxes.  Block extents
// start at 3 and grow by 3 samples at a time, innermost axis first, while the box
// (block + search window + patch per axis) stays within kBoxCap samples and
// the launch keeps at least kMinBlocks workgroups.  The origins are listed
// block by block (C-order over the block grid), ascending inside a block.
void nd_make_blocks(const Geo& g, const std::vector<int64_t>& refs, int rule,
                    std::vector<int64_t>& refs_out, std::vector<int>& start, NdBlocks& blk)
{
    // default: boxes of 72 KiB of FP64 (two workgroups per compute unit),
    // at least 2048 workgroups per launch summed over the batch
    const BlockRule& R = kBlockRules[rule >= 0 && rule < kNumBlockRules ? rule : 0];
    const long kBoxCap = R.box_cap;
    blk = NdBlocks{};
    const long nref = long(refs.size());
    const long max_refs = std::max(R.refs_floor, nref * std::max(1, g.batch) / R.min_blocks);
    int B[kAx];
    for (int d = 0; d < kAx; ++d) B[d] = std::min(g.L[d], 3);
    auto box = [&](const int* b) {
        long v = 1;
        for (int d = 0; d < kAx; ++d) v *= long(b[d] + g.W[d] + g.j[d] - 2);
        return v;
    };
    auto refs_per_block = [&](const int* b) {
        double f = 1.0;
        for (int d = 0; d < kAx; ++d)
            if (g.L[d] > 1) f *= double(b[d]) / double(std::max(1, g.L[d])) ;
        return f * double(nref);
    };
    for (bool grew = true; grew;) {
        grew = false;
        for (int d = kAx - 1; d >= 0; --d) {
            if (g.L[d] == 1 || B[d] >= g.L[d]) continue;
            int t[kAx];
            std::copy(B, B + kAx, t);
            t[d] = std::min(g.L[d], B[d] + 3);
            if (box(t) > kBoxCap || refs_per_block(t) > double(max_refs)) continue;
            B[d] = t[d];
            grew = true;
        }
    }
    long nblocks = 1;
    for (int d = 0; d < kAx; ++d) {
        blk.B[d] = B[d];
        blk.nb[d] = (g.L[d] + B[d] - 1) / B[d];
        blk.E[d] = B[d] + g.W[d] + g.j[d] - 2;
        // last axis padded to a multiple of 4 samples: rows of a byte copy
        // of the box then start on word boundaries
        if (d == kAx - 1) blk.E[d] = (blk.E[d] + 3) & ~3;
        nblocks *= blk.nb[d];
    }
    int s = 1;
    for (int d = kAx - 1; d >= 0; --d) {
        blk.S[d] = s;
        s *= blk.E[d];
    }
    blk.box_size = s;
    blk.nblocks = int(nblocks);
    nd_match_layout(g, blk);
    // counting sort by block
    std::vector<int> bid(refs.size());
    start.assign(size_t(nblocks) + 1, 0);
    for (size_t k = 0; k < refs.size(); ++k) {
        int id = 0;
        for (int d = 0; d < kAx; ++d) {
            const int c = int((refs[k] / g.st[d]) % g.L[d]);
            id = id * blk.nb[d] + c / B[d];
        }
        bid[k] = id;
        ++start[size_t(id) + 1];
    }
    for (long b = 0; b < nblocks; ++b) start[size_t(b) + 1] += start[size_t(b)];
    refs_out.assign(refs.size(), 0);
    std::vector<int> pos(start.begin(), start.end() - 1);
    for (size_t k = 0; k < refs.size(); ++k) refs_out[size_t(pos[size_t(bid[k])]++)] = refs[k];
}

// Coverage map of a schedule (section Experiments, Shift Schedule
// Analysis): C(x) = number of scheduled reference patches containing x.
// Built separably: a count of 1 at every origin, then along each axis the
// running sum over the last j_d samples (a patch starting at r covers
// r .. r + j_d - 1), so each axis costs one pass over the array.
std::vector<uint32_t> coverage_map(const bmnd_geometry& geom, const bmnd_stage_params& sp)
{
    const int D = geom.ndim;
    int64_t V = 1;
    for (int d = 0; d < D; ++d) V *= geom.shape[d];
    std::vector<uint32_t> c(size_t(V), 0u);
    for (int64_t o : reference_origins(geom, sp)) c[size_t(o)] = 1u;
    std::vector<uint32_t> line;
    int64_t inner = 1;
    for (int d = D - 1; d >= 0; --d) {
        const int64_t L = geom.shape[d], j = sp.patch[d];
        const int64_t outer = V / (L * inner);
        line.resize(size_t(L));
        for (int64_t a = 0; a < outer; ++a)
            for (int64_t b = 0; b < inner; ++b) {
                uint32_t* base = c.data() + a * L * inner + b;
                for (int64_t i = 0; i < L; ++i) line[size_t(i)] = base[i * inner];
                uint32_t run = 0;
                for (int64_t i = 0; i < L; ++i) {
                    run += line[size_t(i)];
                    if (i >= j) run -= line[size_t(i - j)];
                    base[i * inner] = run;
                }
            }
        inner *= L;
    }
    return c;
}

}  // namespace bmnd
