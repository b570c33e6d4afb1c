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
    nd_filter_layout(g, blk);
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

// The filter adds a group's patches to its block's FP64 box one sample
// offset at a time: in one LDS instruction the lanes (members) write at
// addresses that differ by their origins.  The LDS serves a 64-bit access
// 16 lanes at a time, one double per bank pair (16 pairs); lanes of a pass
// that share a pair wait for each other.  Members lie anywhere in the search
// window, often along an edge or a plane of the volume, so the strides are
// chosen by their cost on fixed pseudo-random member sets of the window:
// uniform, within one axis-aligned plane or a slab three samples thick, and
// clustered about the reference.  Rows and planes may grow by up to 15
// doubles within max(the C-order box, 10112 doubles): two workgroups still
// share a compute unit's LDS.
void nd_filter_layout(const Geo& g, NdBlocks& blk)
{
    std::copy(blk.E, blk.E + kAx, blk.FE);
    std::copy(blk.S, blk.S + kAx, blk.FS);
    blk.fbox = blk.box_size;
    int act[kAx], na = 0;   // active axes, outermost first
    for (int d = 0; d < kAx; ++d)
        if (blk.E[d] > 1) act[na++] = d;
    if (na < 2) return;
    int FE[kAx];
    std::copy(blk.E, blk.E + kAx, FE);
    // the last axis without its rounding to 4 (no patch reaches past it)
    FE[kAx - 1] = std::min(blk.E[kAx - 1], blk.B[kAx - 1] + g.W[kAx - 1] + g.j[kAx - 1] - 2);
    int n[kAx];   // window positions per axis
    for (int d = 0; d < kAx; ++d) n[d] = std::max(1, std::min(g.W[d], g.ell[d] + 1));

    // member sets: 32 window positions each, as coordinates
    constexpr int kM = 32, kPer = 8;
    const int npos = n[0] * n[1] * n[2] * n[3];
    std::vector<int> xyz(size_t(npos) * kAx);   // coordinates, innermost axis first
    std::vector<double> r2(size_t(npos), 0.0);  // squared distance from the centre
    for (int q = 0; q < npos; ++q) {
        int rem = q;
        for (int d = kAx - 1; d >= 0; --d) {
            const int x = rem % n[d];
            rem /= n[d];
            xyz[size_t(q) * kAx + size_t(kAx - 1 - d)] = x;
            const double c = x - 0.5 * (n[d] - 1);
            r2[size_t(q)] += c * c;
        }
    }
    std::vector<int> sets;   // [set][member]: a position, or -1
    uint64_t st = 0x9e3779b97f4a7c15ull;
    auto rnd = [&](int m) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return int((st >> 33) % uint64_t(m));
    };
    std::vector<int> pool;
    auto add_set = [&]() {
        // 32 distinct positions of the pool (all of it when smaller)
        const int take = std::min<int>(kM, int(pool.size()));
        for (int k = 0; k < take; ++k)
            std::swap(pool[size_t(k)], pool[size_t(k + rnd(int(pool.size()) - k))]);
        for (int k = 0; k < kM; ++k) sets.push_back(k < take ? pool[size_t(k)] : -1);
    };
    for (int k = 0; k < kPer; ++k) {
        pool.resize(size_t(npos));
        for (int q = 0; q < npos; ++q) pool[size_t(q)] = q;
        add_set();
    }
    for (int a = 0; a < na; ++a) {
        const int d = act[a], xi = kAx - 1 - d;
        for (int k = 0; k < kPer; ++k) {
            const int c = rnd(n[d]), c3 = rnd(std::max(1, n[d] - 2));
            pool.clear();
            for (int q = 0; q < npos; ++q)
                if (xyz[size_t(q) * kAx + size_t(xi)] == c) pool.push_back(q);
            add_set();
            pool.clear();
            for (int q = 0; q < npos; ++q) {
                const int x = xyz[size_t(q) * kAx + size_t(xi)];
                if (x >= c3 && x < c3 + 3) pool.push_back(q);
            }
            add_set();
        }
    }
    {
        // the positions nearest the centre, distances jittered
        std::vector<std::pair<double, int>> dist;
        for (int q = 0; q < npos; ++q)
            if (r2[size_t(q)] <= 16.0 + 1e-9) dist.push_back({r2[size_t(q)], q});
        for (int k = 0; k < kPer; ++k) {
            for (auto& e : dist) e.first = r2[size_t(e.second)] + 6.0 * rnd(1000) / 1000.0;
            std::sort(dist.begin(), dist.end());
            pool.clear();
            for (int m = 0; m < kM && m < int(dist.size()); ++m) pool.push_back(dist[size_t(m)].second);
            add_set();
        }
    }
    const int nsets = int(sets.size()) / kM;
    std::vector<long> addr(static_cast<size_t>(npos));
    auto cost = [&](const int* S) {
        for (int q = 0; q < npos; ++q) {
            long v = 0;
            for (int d = 0; d < kAx; ++d) v += long(xyz[size_t(q) * kAx + size_t(d)]) * S[kAx - 1 - d];
            addr[size_t(q)] = v;
        }
        long c = 0;
        for (int t = 0; t < nsets; ++t)
            for (int pass = 0; pass < kM; pass += 16) {
                int cnt[16] = {0};
                int mx = 0;
                for (int m = pass; m < pass + 16; ++m) {
                    const int q = sets[size_t(t * kM + m)];
                    if (q < 0) continue;
                    mx = std::max(mx, ++cnt[addr[size_t(q)] & 15]);
                }
                c += mx;
            }
        return c;
    };
    const long cap = std::max<long>(blk.box_size, 10112);
    const int mid = act[na - 2], out3 = na >= 3 ? act[na - 3] : -1;
    long best = -1, best_size = 0;
    int S[kAx];
    for (int p1 = 0; p1 < 16; ++p1)
        for (int p0 = 0; p0 < (out3 >= 0 ? 16 : 1); ++p0) {
            // C-order strides over FE, the rows (stride of axis mid) longer
            // by p1 and the planes (stride of axis out3) by p0
            S[kAx - 1] = 1;
            for (int d = kAx - 2; d >= 0; --d)
                S[d] = FE[d + 1] * S[d + 1] + (d == mid ? p1 : (d == out3 ? p0 : 0));
            const long size = long(FE[0]) * S[0];
            if (size > cap) continue;
            const long k = cost(S);
            if (best < 0 || k < best || (k == best && size < best_size)) {
                best = k;
                best_size = size;
                std::copy(S, S + kAx, blk.FS);
            }
        }
    if (best >= 0) {
        std::copy(FE, FE + kAx, blk.FE);
        blk.fbox = int(best_size);
    }
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
