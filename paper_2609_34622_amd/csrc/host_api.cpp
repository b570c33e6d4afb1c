// C ABI of the BMND library: validation, library-owned caches, workspace
// layout and launch orchestration.  See include/bmnd.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "bmnd_internal.h"
#include "denoise_plan.h"

namespace bmnd {

static thread_local std::string t_error;

void set_error(const std::string& msg) { t_error = msg; }

size_t filter_lds_bytes(const Geo& g, int gmax);

namespace {

bool is_pow2(int v) { return v >= 1 && (v & (v - 1)) == 0; }

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bmnd_status fail(bmnd_status st, const std::string& msg)
{
    set_error(msg);
    return st;
}

bmnd_status check_geometry(const bmnd_geometry* g)
{
    if (!g) return fail(BMND_E_ARG, "geometry is NULL");
    if (g->ndim < 1 || g->ndim > BMND_MAX_AXES) return fail(BMND_E_SHAPE, "ndim out of range");
    if (g->ndim > BMND_GPU_AXES) {
        // singleton axes are dropped for the kernels (kernel_axes)
        int wide = 0;
        for (int d = 0; d < g->ndim; ++d) wide += g->shape[d] > 1;
        if (wide > BMND_GPU_AXES)
            return fail(BMND_E_UNSUPPORTED,
                        "the GPU kernels accept at most 4 axes of extent > 1");
    }
    if (g->reserved != 0) return fail(BMND_E_ARG, "geometry.reserved must be 0");
    if (g->batch < 1) return fail(BMND_E_SHAPE, "batch must be >= 1");
    double total = double(g->batch);
    for (int d = 0; d < g->ndim; ++d) {
        if (g->shape[d] < 1) return fail(BMND_E_SHAPE, "shape entries must be >= 1");
        total *= double(g->shape[d]);
    }
    if (total >= 2147483647.0) return fail(BMND_E_SHAPE, "batch * volume must be < 2^31");
    return BMND_OK;
}

bmnd_status check_stage(const bmnd_geometry* g, const bmnd_stage_params* sp, int stage)
{
    if (!sp) return fail(BMND_E_ARG, "stage parameters are NULL");
    int P = 1;
    for (int d = 0; d < g->ndim; ++d) {
        if (sp->patch[d] < 1 || sp->patch[d] > g->shape[d])
            return fail(BMND_E_ARG, "patch must satisfy 1 <= j_d <= L_d");
        if (sp->patch[d] > kMaxPatch) return fail(BMND_E_UNSUPPORTED, "patch extent > 32");
        if (sp->step[d] < 1) return fail(BMND_E_ARG, "step must be >= 1");
        if (sp->search[d] < 1) return fail(BMND_E_ARG, "search must be >= 1");
        P *= sp->patch[d];
    }
    if (sp->schedule < BMND_SCHED_GENERATED || sp->schedule > BMND_SCHED_OFF)
        return fail(BMND_E_ARG, "unknown schedule");
    if (sp->passes < 1) return fail(BMND_E_ARG, "passes must be >= 1");
    if (!(sp->shift_density >= 0.0)) return fail(BMND_E_ARG, "shift_density must be >= 0");
    if (!is_pow2(sp->group_max) || sp->group_max > kMaxGroup)
        return fail(BMND_E_ARG, "group_max must be a power of two <= 32");
    if (!is_pow2(sp->group_min) || sp->group_min > sp->group_max)
        return fail(BMND_E_ARG, "group_min must be a power of two <= group_max");
    if (sp->group_max * P > kMaxKP) return fail(BMND_E_UNSUPPORTED, "group_max * P > 4096");
    if (sp->spatial < BMND_SPATIAL_IDENTITY || sp->spatial > BMND_SPATIAL_BIOR15)
        return fail(BMND_E_ARG, "unknown spatial transform");
    if (stage == BMND_STAGE_HT) {
        if (sp->shrink != BMND_SHRINK_HARD && sp->shrink != BMND_SHRINK_SOFT)
            return fail(BMND_E_ARG, "the HT stage needs hard or soft thresholding");
        if (sp->weight_model == BMND_WEIGHT_RISK)
            return fail(BMND_E_ARG, "the HT stage has no risk weight model");
        if (!(sp->lambda >= 0.0)) return fail(BMND_E_ARG, "lambda must be >= 0");
        if (!(sp->gamma >= 0.0)) return fail(BMND_E_ARG, "gamma must be >= 0");
    } else if (stage == BMND_STAGE_WIENER) {
        if (sp->shrink != BMND_SHRINK_WIENER)
            return fail(BMND_E_ARG, "the Wiener stage needs Wiener shrinkage");
        if (sp->gamma != 0.0) return fail(BMND_E_ARG, "the Wiener stage matches with plain SSD");
        if (!(sp->s_v >= 0.0) || !(sp->power_a >= 0.0))
            return fail(BMND_E_ARG, "s_v and power_a must be >= 0");
    } else {
        return fail(BMND_E_ARG, "unknown stage");
    }
    if (sp->weight_model < BMND_WEIGHT_CLASSIC || sp->weight_model > BMND_WEIGHT_RISK)
        return fail(BMND_E_ARG, "unknown weight model");
    if (sp->weight_scope != BMND_SCOPE_GROUP && sp->weight_scope != BMND_SCOPE_PATCH)
        return fail(BMND_E_ARG, "unknown weight scope");
    if (sp->k_exact < 0) return fail(BMND_E_ARG, "k_exact must be >= 0");
    if (!(sp->kaiser_beta >= 0.0)) return fail(BMND_E_ARG, "kaiser_beta must be >= 0");
    if (sp->weight_domain != BMND_WDOMAIN_COEFFICIENT && sp->weight_domain != BMND_WDOMAIN_WINDOWED)
        return fail(BMND_E_ARG, "unknown weight domain");
    if (sp->reserved2 != 0) return fail(BMND_E_ARG, "reserved field must be 0");
    if (sp->match_metric < BMND_METRIC_SSD || sp->match_metric > BMND_METRIC_ANSCOMBE)
        return fail(BMND_E_ARG, "unknown matching metric");
    if (sp->match_policy < BMND_POLICY_FIXED || sp->match_policy > BMND_POLICY_STANDARDIZED)
        return fail(BMND_E_ARG, "unknown matching policy");
    if (sp->match_metric != BMND_METRIC_SSD && stage != BMND_STAGE_HT)
        return fail(BMND_E_ARG, "Poisson-likelihood matching is an HT-stage option");
    if (sp->match_metric == BMND_METRIC_SSD && sp->match_policy != BMND_POLICY_FIXED)
        return fail(BMND_E_ARG, "SSD matching uses the fixed policy");
    if (sp->match_metric != BMND_METRIC_SSD &&
        (!(sp->match_t >= 0.0) || !(sp->struct_beta >= 0.0) || !(sp->struct_kappa > 0.0) ||
         !std::isfinite(sp->match_t) || !std::isfinite(sp->struct_beta) ||
         !std::isfinite(sp->struct_kappa)))
        return fail(BMND_E_ARG, "match_t and struct_beta must be >= 0, struct_kappa > 0");
    return BMND_OK;
}

bmnd_status check_noise(const bmnd_noise* n)
{
    if (!n) return fail(BMND_E_ARG, "noise is NULL");
    if (n->kind == BMND_NOISE_POISSON) {
        if (!(n->s_p > 0.0)) return fail(BMND_E_ARG, "Poisson s_p must be > 0");
    } else if (n->kind == BMND_NOISE_GAUSSIAN) {
        if (!(n->sigma >= 0.0)) return fail(BMND_E_ARG, "Gaussian sigma must be >= 0");
    } else if (n->kind == BMND_NOISE_CORRELATED) {
        if (!n->d_corr) return fail(BMND_E_ARG, "correlated noise needs prepared tables");
    } else {
        return fail(BMND_E_ARG, "unknown noise kind");
    }
    return BMND_OK;
}

// The axes the kernels see, in order: every axis of an array of at most 4
// axes; of a larger one, the axes of extent > 1.  A singleton axis has one
// patch position (j = 1, origin 0) and one candidate, so dropping it changes
// no patch, window, stride or linear index; the reference origins are still
// computed on the full geometry, where a singleton axis takes part in the
// generated schedule's axis hierarchy.
int kernel_axes(const bmnd_geometry* g, int* ax)
{
    int n = 0;
    for (int d = 0; d < g->ndim; ++d)
        if (g->ndim <= kAx || g->shape[d] > 1) ax[n++] = d;
    return n;
}

Geo make_geo(const bmnd_geometry* g, const bmnd_stage_params* sp)
{
    Geo o{};
    int ax[BMND_MAX_AXES];
    const int na = kernel_axes(g, ax);
    const int pad = kAx - na;
    for (int k = 0; k < kAx; ++k) {
        const int d = k - pad >= 0 ? ax[k - pad] : -1;
        o.L[k] = d >= 0 ? int(g->shape[d]) : 1;
        o.j[k] = d >= 0 ? sp->patch[d] : 1;
        o.W[k] = d >= 0 ? sp->search[d] : 1;
    }
    int acc = 1;
    for (int k = kAx - 1; k >= 0; --k) {
        o.st[k] = acc;
        acc *= o.L[k];
        o.ell[k] = o.L[k] - o.j[k];
    }
    o.V = acc;
    o.P = o.j[0] * o.j[1] * o.j[2] * o.j[3];
    o.batch = int(g->batch);
    return o;
}

bmnd_status make_stage(const bmnd_geometry* g, const bmnd_noise* n, const bmnd_stage_params* sp,
                       int stage, StageCfg& c)
{
    bmnd_status st = check_geometry(g);
    if (st != BMND_OK) return st;
    if ((st = check_stage(g, sp, stage)) != BMND_OK) return st;
    if (n && (st = check_noise(n)) != BMND_OK) return st;
    if (n && sp->match_metric != BMND_METRIC_SSD) {
        if (n->kind != BMND_NOISE_POISSON)
            return fail(BMND_E_ARG, "Poisson-likelihood matching needs Poisson noise");
        if (sp->match_policy != BMND_POLICY_FIXED && !n->counts_integral)
            return fail(BMND_E_ARG, "finite-count calibration needs integral counts");
    }
    c = StageCfg{};
    c.g = make_geo(g, sp);
    c.stage = stage;
    c.noise = n ? n->kind : BMND_NOISE_GAUSSIAN;
    c.s_p = n ? n->s_p : 1.0;
    c.sigma = n ? n->sigma : 0.0;
    c.gamma = sp->gamma;
    c.integral = n && stage == BMND_STAGE_HT && n->kind == BMND_NOISE_POISSON &&
                 n->counts_integral && sp->gamma == std::floor(sp->gamma);
    c.tau = sp->tau >= 0.0 ? sp->tau
                           : (stage == BMND_STAGE_HT ? 3000.0 : 400.0) * c.g.P / (255.0 * 255.0);
    c.gmin = sp->group_min;
    c.gmax = sp->group_max;
    c.spatial = sp->spatial;
    c.shrink = sp->shrink;
    c.lambda = sp->lambda;
    c.s_v = sp->s_v;
    c.power_a = sp->power_a;
    c.k_exact = sp->k_exact;
    c.wmodel = sp->weight_model;
    c.wscope = sp->weight_scope;
    c.mc = sp->mass_conservation ? 1 : 0;
    c.beta = sp->kaiser_beta;
    {
        int ax[BMND_MAX_AXES];
        const int na = kernel_axes(g, ax);
        c.step_last = sp->step[na > 0 ? ax[na - 1] : g->ndim - 1];
    }
    c.metric = sp->match_metric;
    c.policy = sp->match_policy;
    c.match_t = sp->match_t;
    c.sbeta = sp->struct_beta;
    c.skappa = sp->struct_kappa;
    c.counts_integral = n && n->kind == BMND_NOISE_POISSON && n->counts_integral;
    c.wdomain = sp->weight_domain;
    if (n && n->kind == BMND_NOISE_CORRELATED) {
        if (g->ndim > BMND_GPU_AXES)
            return fail(BMND_E_UNSUPPORTED, "correlated noise: at most 4 axes");
        c.k_exact = 0;  // the full covariance is exact in every plane
        return correlated_bind(n->d_corr, g, sp, stage, c);
    }
    return BMND_OK;
}

// ------------------------------------------------------------- caches

std::mutex g_cache_mu;

using TabKey = std::tuple<int, int, int, int, int, int, double>;
std::map<TabKey, DevTables> g_tables;


}  // namespace

void build_tables_host(const StageCfg& c, std::vector<float>& f, std::vector<double>& f64,
                       DevTables& t)
{
    t = DevTables{};
    f.clear();
    f64.clear();
    for (int d = 0; d < kAx; ++d) {
        const int n = c.g.j[d];
        std::vector<double> T, U;
        spatial_matrices(n > 1 ? c.spatial : BMND_SPATIAL_IDENTITY, n, T, U);
        t.T[d] = int(f.size());
        for (double v : T) f.push_back(float(v));
        t.U[d] = int(f.size());
        for (double v : U) f.push_back(float(v));
        t.T2[d] = int(f.size());
        for (double v : T) f.push_back(float(v * v));
        t.win[d] = int(f.size());
        for (double v : kaiser_window(n, c.beta)) f.push_back(float(v));
        // diagonal of the windowed synthesis metric per coefficient q:
        // sum_i (w_i U[i][q])^2 (U stored sample-major, U[i][q] = U[i * n + q])
        t.hw[d] = int(f.size());
        {
            const std::vector<double> w = kaiser_window(n, c.beta);
            for (int q = 0; q < n; ++q) {
                double s = 0.0;
                for (int i = 0; i < n; ++i) {
                    const double v = w[size_t(i)] * U[size_t(i * n + q)];
                    s += v * v;
                }
                f.push_back(float(s));
            }
        }
        t.rn[d] = int(f.size());
        for (int q = 0; q < n; ++q) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += T[size_t(q * n + k)] * T[size_t(q * n + k)];
            f.push_back(float(std::sqrt(s)));
        }
        t.T64[d] = int(f64.size());
        for (double v : T) f64.push_back(v);
        t.T264[d] = int(f64.size());
        for (double v : T) f64.push_back(v * v);
        // autocorrelation of every row of T: A[q][tau + n - 1] =
        // sum_i T[q][i] T[q][i + tau] over the i with both inside the patch
        t.ac64[d] = int(f64.size());
        for (int q = 0; q < n; ++q)
            for (int tau = 1 - n; tau < n; ++tau) {
                double s = 0.0;
                for (int i = std::max(0, -tau); i < n && i + tau < n; ++i)
                    s += T[size_t(q * n + i)] * T[size_t(q * n + i + tau)];
                f64.push_back(s);
            }
    }
    t.haar = int(f.size());
    t.haar64 = int(f64.size());
    for (int K = 1; K <= kMaxGroup; K *= 2) {
        std::vector<double> H;
        haar_matrix(K, H);
        for (double v : H) {
            f.push_back(float(v));
            f64.push_back(v);
        }
    }
    t.f32_count = int(f.size());
    t.f64_count = int(f64.size());
}

const DevTables* device_tables(const StageCfg& c, std::string& err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return nullptr;
    }
    TabKey key{dev, c.spatial, c.g.j[0], c.g.j[1], c.g.j[2], c.g.j[3], c.beta};
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_tables.find(key);
    if (it != g_tables.end()) return &it->second;

    DevTables t{};
    std::vector<float> f;
    std::vector<double> f64;
    build_tables_host(c, f, f64, t);
    float* df = nullptr;
    double* dd = nullptr;
    if (hipMalloc(&df, f.size() * sizeof(float)) != hipSuccess ||
        hipMalloc(&dd, f64.size() * sizeof(double)) != hipSuccess) {
        err = "hipMalloc of the transform tables failed";
        return nullptr;
    }
    if (hipMemcpy(df, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dd, f64.data(), f64.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess) {
        err = "upload of the transform tables failed";
        return nullptr;
    }
    t.f32 = df;
    t.f64 = dd;
    t.f32_count = int(f.size());
    t.f64_count = int(f64.size());
    return &(g_tables[key] = t);
}

namespace {

using HostOrgKey = std::tuple<std::vector<int64_t>, std::vector<int>, int, int, double>;
std::map<TabKey, HostTables> g_host_tables;

HostOrgKey host_org_key(const bmnd_geometry& geom, const bmnd_stage_params& sp)
{
    std::vector<int64_t> shape(geom.shape, geom.shape + geom.ndim);
    std::vector<int> ps(size_t(2 * geom.ndim));
    for (int d = 0; d < geom.ndim; ++d) {
        ps[size_t(d)] = sp.patch[d];
        ps[size_t(geom.ndim + d)] = sp.step[d];
    }
    return HostOrgKey{shape, ps, sp.schedule, sp.passes, sp.shift_density};
}

// A map of shared entries that keeps the most recently used ones within a
// byte budget.  Users hold an entry's shared pointer while they need it;
// evicted entries are handed back to the caller, to be released outside
// the cache lock.  Callers hold g_cache_mu.
template <class K, class V>
class LruCache {
public:
    explicit LruCache(size_t cap) : cap_(cap) {}
    std::shared_ptr<V> find(const K& k)
    {
        auto it = map_.find(k);
        if (it == map_.end()) return nullptr;
        order_.splice(order_.begin(), order_, it->second.pos);
        return it->second.v;
    }
    std::shared_ptr<V> insert(const K& k, std::shared_ptr<V> v, size_t bytes,
                              std::vector<std::shared_ptr<V>>& dropped)
    {
        if (auto old = find(k)) return old;
        order_.push_front(k);
        map_.emplace(k, Entry{v, bytes, order_.begin()});
        total_ += bytes;
        trim(1, dropped);
        return v;
    }
    void set_cap(size_t cap, std::vector<std::shared_ptr<V>>& dropped)
    {
        cap_ = cap;
        trim(0, dropped);
    }

private:
    // over the budget: evict from the least recently used end down to half
    // of it (so that device copies are released many at a time, behind one
    // wait for the device), keeping at least `keep` entries (the one just
    // inserted)
    void trim(size_t keep, std::vector<std::shared_ptr<V>>& dropped)
    {
        if (total_ <= cap_) return;
        while (total_ > cap_ / 2 && order_.size() > keep) {
            auto e = map_.find(order_.back());
            total_ -= e->second.bytes;
            dropped.push_back(std::move(e->second.v));
            map_.erase(e);
            order_.pop_back();
        }
    }

    struct Entry {
        std::shared_ptr<V> v;
        size_t bytes;
        typename std::list<K>::iterator pos;
    };
    size_t cap_, total_ = 0;
    std::list<K> order_;
    std::map<K, Entry> map_;
};

constexpr size_t kHostCacheBytes = size_t(1) << 30;    // schedules and block lists
constexpr size_t kDeviceCacheBytes = size_t(1) << 30;  // their device copies, all devices

// The caches live until the process ends (never destroyed: device entries
// must not be freed after the HIP runtime has shut down).
LruCache<HostOrgKey, const std::vector<int64_t>>& host_origin_cache()
{
    static auto* c = new LruCache<HostOrgKey, const std::vector<int64_t>>(kHostCacheBytes);
    return *c;
}

// blocks depend on the search window too (the box spans it), and on the
// block rule in force for that shape and window (the autotuner's choice,
// else rule 0)
using TuneKey = std::pair<HostOrgKey, std::vector<int>>;
std::map<TuneKey, int> g_block_rule;   // guarded by g_cache_mu
using BlkKey = std::tuple<HostOrgKey, std::vector<int>, int>;
TuneKey tune_key(const bmnd_geometry& geom, const bmnd_stage_params& sp)
{
    return TuneKey{host_org_key(geom, sp), std::vector<int>(sp.search, sp.search + geom.ndim)};
}
int block_rule(const TuneKey& k)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_block_rule.find(k);
    return it == g_block_rule.end() ? 0 : it->second;
}
BlkKey blk_key(const bmnd_geometry& geom, const bmnd_stage_params& sp)
{
    TuneKey t = tune_key(geom, sp);
    const int rule = block_rule(t);
    return BlkKey{std::move(t.first), std::move(t.second), rule};
}
LruCache<BlkKey, const HostBlocks>& host_block_cache()
{
    static auto* c = new LruCache<BlkKey, const HostBlocks>(kHostCacheBytes);
    return *c;
}

// A device copy of a stage's origin list (and, for the N-D filter, of its
// block offsets).  It is freed only after the device has finished all
// queued work, so no launch that read it can still be running.
// The upload runs on the stream of the call that first needs the list, from
// host lists this entry keeps alive; `ready` marks its end for other streams.
struct DevList {
    int dev = 0;
    int64_t* refs = nullptr;
    int* start = nullptr;
    int64_t n = 0;
    NdBlocks blk;
    hipEvent_t ready = nullptr;
    std::shared_ptr<const void> host;   // the host lists the upload reads
    ~DevList()
    {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return;
        if (hipSetDevice(dev) == hipSuccess) {
            (void)hipDeviceSynchronize();
            if (refs) (void)hipFree(refs);
            if (start) (void)hipFree(start);
            if (ready) (void)hipEventDestroy(ready);
        }
        (void)hipSetDevice(cur);
    }
};
// key: device, blocked (0 / 1), origin key, search window (blocked only)
using DevKey = std::tuple<int, int, BlkKey>;
LruCache<DevKey, const DevList>& device_list_cache()
{
    static auto* c = new LruCache<DevKey, const DevList>(kDeviceCacheBytes);
    return *c;
}

}  // namespace

std::shared_ptr<const std::vector<int64_t>> host_origins_cached(const bmnd_geometry& geom,
                                                                const bmnd_stage_params& sp)
{
    const HostOrgKey key = host_org_key(geom, sp);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (auto v = host_origin_cache().find(key)) return v;
    }
    auto o = std::make_shared<const std::vector<int64_t>>(reference_origins(geom, sp));
    std::vector<std::shared_ptr<const std::vector<int64_t>>> dropped;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return host_origin_cache().insert(key, o, o->size() * sizeof(int64_t), dropped);
}

const HostTables& host_tables_cached(const StageCfg& c)
{
    TabKey key{-1, c.spatial, c.g.j[0], c.g.j[1], c.g.j[2], c.g.j[3], c.beta};
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_host_tables.find(key);
    if (it != g_host_tables.end()) return it->second;
    HostTables h;
    build_tables_host(c, h.f, h.f64, h.t);
    return g_host_tables.emplace(key, std::move(h)).first->second;
}

bool stage_uses_nd(const StageCfg& c)
{
    return nd_filter_supported(c.g, c.gmax, c.k_exact, c.noise == BMND_NOISE_CORRELATED, c.noise,
                               c.shrink);
}

std::shared_ptr<const HostBlocks> host_blocks_cached(const bmnd_geometry& geom,
                                                     const bmnd_stage_params& sp, const Geo& g)
{
    const BlkKey key = blk_key(geom, sp);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (auto v = host_block_cache().find(key)) return v;
    }
    const auto o = host_origins_cached(geom, sp);
    auto h = std::make_shared<HostBlocks>();
    Geo g1 = g;
    g1.batch = 1;
    nd_make_blocks(g1, *o, std::get<2>(key), h->refs, h->start, h->blk);
    const size_t bytes = h->refs.size() * sizeof(int64_t) + h->start.size() * sizeof(int);
    std::vector<std::shared_ptr<const HostBlocks>> dropped;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return host_block_cache().insert(key, std::move(h), bytes, dropped);
}

namespace {

// Device copy of a stage's origins: in block order with the block offsets
// (blocked), or ascending.  Uploaded once per device and kept while it is
// among the recently used lists.
std::shared_ptr<const DevList> device_list(const bmnd_geometry& geom, const bmnd_stage_params& sp,
                                           const Geo& g, bool blocked, hipStream_t s,
                                           std::string& err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return nullptr;
    }
    const DevKey key{dev, blocked ? 1 : 0,
                     blocked ? blk_key(geom, sp) : BlkKey{host_org_key(geom, sp), {}, 0}};
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (auto v = device_list_cache().find(key)) return v;
    }
    std::shared_ptr<const HostBlocks> hb;
    std::shared_ptr<const std::vector<int64_t>> ho;
    if (blocked) hb = host_blocks_cached(geom, sp, g);
    else ho = host_origins_cached(geom, sp);
    const std::vector<int64_t>& refs = blocked ? hb->refs : *ho;
    auto d = std::make_shared<DevList>();
    d->dev = dev;
    d->n = int64_t(refs.size());
    if (blocked) d->host = hb;
    else d->host = ho;
    size_t bytes = std::max<size_t>(1, refs.size()) * sizeof(int64_t);
    if (hipEventCreateWithFlags(&d->ready, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&d->refs, bytes) != hipSuccess ||
        hipMemcpyAsync(d->refs, refs.data(), refs.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                       s) != hipSuccess) {
        err = "allocation of the reference-origin list failed";
        return nullptr;
    }
    if (blocked) {
        d->blk = hb->blk;
        bytes += hb->start.size() * sizeof(int);
        if (hipMalloc(&d->start, hb->start.size() * sizeof(int)) != hipSuccess ||
            hipMemcpyAsync(d->start, hb->start.data(), hb->start.size() * sizeof(int),
                           hipMemcpyHostToDevice, s) != hipSuccess) {
            err = "allocation of the block offsets failed";
            return nullptr;
        }
        d->blk.start = d->start;
    }
    if (hipEventRecord(d->ready, s) != hipSuccess) {
        err = "event record failed";
        return nullptr;
    }
    std::vector<std::shared_ptr<const DevList>> dropped;
    std::shared_ptr<const DevList> out;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        out = device_list_cache().insert(key, std::move(d), bytes, dropped);
    }
    return out;   // `dropped` (and a duplicate `d`) released here, outside the lock
}

}  // namespace

// ------------------------------------------------------------- tracing

namespace {

struct ProfRec {
    int id;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

// Records an event pair around one kernel launch when tracing is on.
struct KernelSpan {
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    KernelSpan(int id_, hipStream_t s_) : id(id_), s(s_)
    {
        if (!g_prof_on || id < 0) return;
        if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
    }
    ~KernelSpan()
    {
        if (!a || !b) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back({id, a, b});
    }
};

}  // namespace

}  // namespace bmnd

using namespace bmnd;

namespace {

// bytes of the match-stage scratch (counts + patch sums)
size_t match_ws(const Geo& g) { return 2 * align256(size_t(g.batch) * g.V * sizeof(int)); }
size_t agg_ws(const Geo& g) { return 2 * align256(size_t(g.batch) * g.V * sizeof(double)); }

bmnd_status hip_fail(hipError_t e, const char* what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return BMND_E_HIP;
}

bmnd_stage_params preset_stage(int32_t preset, int32_t ndim, int stage)
{
    bmnd_stage_params p{};
    const int j = ndim == 1 ? 32 : (ndim == 2 ? 8 : 4);
    const int h = ndim == 1 ? 4 : 3;
    const int w = ndim == 1 ? 256 : (ndim == 2 ? 19 : 7);
    for (int d = 0; d < ndim; ++d) {
        p.patch[d] = j;
        p.step[d] = h;
        p.search[d] = w;
    }
    p.schedule = BMND_SCHED_GENERATED;
    p.passes = 2;
    p.shift_density = 2.0;
    p.group_min = 2;
    p.group_max = stage == BMND_STAGE_HT ? 16 : 32;
    p.tau = -1.0;
    p.gamma = stage == BMND_STAGE_HT ? 3.0 : 0.0;
    p.spatial = stage == BMND_STAGE_HT ? BMND_SPATIAL_BIOR15 : BMND_SPATIAL_DCT;
    p.shrink = stage == BMND_STAGE_HT ? BMND_SHRINK_HARD : BMND_SHRINK_WIENER;
    p.lambda = 3.0;
    p.s_v = 0.4;
    p.power_a = 0.0;
    p.k_exact = preset == BMND_PRESET_STANDARD ? 4 : 0;
    p.weight_model = preset == BMND_PRESET_STANDARD ? BMND_WEIGHT_VARIANCE : BMND_WEIGHT_CLASSIC;
    p.weight_scope = preset == BMND_PRESET_STANDARD ? BMND_SCOPE_PATCH : BMND_SCOPE_GROUP;
    p.mass_conservation = 0;
    p.kaiser_beta = 2.0;
    p.match_metric = BMND_METRIC_SSD;
    p.match_policy = BMND_POLICY_FIXED;
    p.match_t = 3.0;
    p.struct_beta = 0.1;
    p.struct_kappa = 1.0;
    p.weight_domain = BMND_WDOMAIN_COEFFICIENT;
    return p;
}

}  // namespace

// ------------------------------------------------ correlated Gaussian noise

namespace bmnd {

hipError_t launch_corr_autocov(const double* psd, const int L[kAx], const int R[kAx], double2* tw,
                               double2* x0, double2* x1, double* cbox, hipStream_t s);
hipError_t launch_corr_dtab(const double* cbox, const int Bc[kAx], const int R[kAx],
                            const int j[kAx], const int bw[kAx], int P,
                            const double* const ac[kAx], double* dtab, hipStream_t s);
hipError_t launch_corr_bias(const double* cbox, const int Bc[kAx], const int R[kAx],
                            const int W[kAx], int P, double gamma, double* b64, float* b32,
                            double* bound, hipStream_t s);

namespace {

// Layout of a prepared table buffer (every region 256-byte aligned).
struct CorrLayout {
    int L[kAx], R[kAx], Bc[kAx];
    size_t off_c = 0, off_tw = 0, off_x0 = 0, off_x1 = 0, off_bound = 0;
    struct Stage {
        int j[kAx], W[kAx], bw[kAx];
        int P = 1, spatial = 0;
        double gamma = 0.0;
        long rows = 1, nwin = 1;
        size_t off_d = 0, off_b64 = 0, off_b32 = 0;
    } st[2];
    size_t bytes = 0;
};

bmnd_status corr_layout(const bmnd_geometry* geom, const bmnd_params* params, CorrLayout& o,
                        StageCfg cfg[2])
{
    if (!geom || !params) return fail(BMND_E_ARG, "NULL argument");
    if (geom->ndim > BMND_GPU_AXES)
        return fail(BMND_E_UNSUPPORTED, "correlated noise: at most 4 axes");
    bmnd_geometry g1 = *geom;
    g1.batch = 1;
    bmnd_status st = make_stage(&g1, nullptr, &params->ht, BMND_STAGE_HT, cfg[0]);
    if (st != BMND_OK) return st;
    if ((st = make_stage(&g1, nullptr, &params->wiener, BMND_STAGE_WIENER, cfg[1])) != BMND_OK)
        return st;
    o = CorrLayout{};
    for (int d = 0; d < kAx; ++d) {
        o.L[d] = cfg[0].g.L[d];
        int r = 0;
        for (int k = 0; k < 2; ++k) {
            const Geo& gg = cfg[k].g;
            const int wm = std::min(gg.W[d], gg.L[d] - gg.j[d] + 1);  // member origins per axis
            r = std::max(r, wm - 1 + gg.j[d] - 1);
            o.st[k].j[d] = gg.j[d];
            o.st[k].W[d] = gg.W[d];
            o.st[k].bw[d] = 2 * wm - 1;
        }
        o.R[d] = r;
        o.Bc[d] = 2 * r + 1;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    long nc = 1, lmax = 1;
    for (int d = 0; d < kAx; ++d) {
        nc *= o.Bc[d];
        lmax = std::max<long>(lmax, o.L[d]);
    }
    // largest intermediate of the separable DFT (every pass but the last)
    long scratch = 1;
    {
        long cur[kAx];
        for (int d = 0; d < kAx; ++d) cur[d] = o.L[d];
        int last = -1;
        for (int d = 0; d < kAx && last < 0; ++d)
            if (o.L[d] > 1) last = d;
        for (int axis = kAx - 1; axis > last; --axis) {
            if (o.L[axis] == 1) continue;
            cur[axis] = o.Bc[axis];
            long n = 1;
            for (int d = 0; d < kAx; ++d) n *= cur[d];
            scratch = std::max(scratch, n);
        }
    }
    o.off_c = take(sizeof(double) * size_t(nc));
    o.off_tw = take(2 * sizeof(double) * size_t(lmax));
    o.off_x0 = take(2 * sizeof(double) * size_t(scratch));
    o.off_x1 = take(2 * sizeof(double) * size_t(scratch));
    o.off_bound = take(sizeof(double));
    for (int k = 0; k < 2; ++k) {
        CorrLayout::Stage& S = o.st[k];
        S.P = cfg[k].g.P;
        S.spatial = cfg[k].spatial;
        S.gamma = cfg[k].gamma;
        S.rows = 1;
        S.nwin = 1;
        for (int d = 0; d < kAx; ++d) {
            S.rows *= S.bw[d];
            S.nwin *= S.W[d];
        }
        if (double(S.rows) * S.P >= 2147483647.0 || double(S.nwin) >= 2147483647.0)
            return fail(BMND_E_UNSUPPORTED, "correlated-noise tables too large for this window");
        S.off_d = take(sizeof(double) * size_t(S.rows) * size_t(S.P));
        if (k == 0) {
            S.off_b64 = take(sizeof(double) * size_t(S.nwin));
            S.off_b32 = take(sizeof(float) * size_t(S.nwin));
        }
    }
    o.bytes = off;
    return BMND_OK;
}

struct CorrEntry {
    int ndim = 0;
    int64_t shape[BMND_MAX_AXES] = {};
    CorrLayout lay;
};

std::map<const void*, CorrEntry> g_corr;

bool same_shape(const CorrEntry& e, const bmnd_geometry* g)
{
    if (e.ndim != g->ndim) return false;
    for (int d = 0; d < g->ndim; ++d)
        if (e.shape[d] != g->shape[d]) return false;
    return true;
}

}  // namespace

bmnd_status correlated_size(const bmnd_geometry* geom, const bmnd_params* params, size_t* bytes)
{
    if (!bytes) return fail(BMND_E_ARG, "NULL argument");
    CorrLayout lay;
    StageCfg cfg[2];
    bmnd_status st = corr_layout(geom, params, lay, cfg);
    if (st != BMND_OK) return st;
    *bytes = lay.bytes;
    return BMND_OK;
}

bmnd_status correlated_prepare(const double* d_psd, const bmnd_geometry* geom,
                               const bmnd_params* params, void* d_tables, size_t bytes,
                               hipStream_t s)
{
    if (!d_psd || !d_tables) return fail(BMND_E_ARG, "NULL device pointer");
    CorrLayout lay;
    StageCfg cfg[2];
    bmnd_status st = corr_layout(geom, params, lay, cfg);
    if (st != BMND_OK) return st;
    if (bytes < lay.bytes) return fail(BMND_E_WORKSPACE, "correlated-noise table buffer too small");
    if ((reinterpret_cast<uintptr_t>(d_tables) & 255u) != 0)
        return fail(BMND_E_WORKSPACE, "correlated-noise table buffer must be 256-byte aligned");
    unsigned char* base = static_cast<unsigned char*>(d_tables);
    double* cbox = reinterpret_cast<double*>(base + lay.off_c);
    hipError_t e = launch_corr_autocov(d_psd, lay.L, lay.R,
                                       reinterpret_cast<double2*>(base + lay.off_tw),
                                       reinterpret_cast<double2*>(base + lay.off_x0),
                                       reinterpret_cast<double2*>(base + lay.off_x1), cbox, s);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        std::string err;
        const DevTables* t = device_tables(cfg[k], err);
        if (!t) return fail(BMND_E_NOMEM, err);
        const double* ac[kAx];
        for (int d = 0; d < kAx; ++d) ac[d] = t->f64 + t->ac64[d];
        const CorrLayout::Stage& S = lay.st[k];
        e = launch_corr_dtab(cbox, lay.Bc, lay.R, S.j, S.bw, S.P, ac,
                             reinterpret_cast<double*>(base + S.off_d), s);
    }
    if (e == hipSuccess)
        e = launch_corr_bias(cbox, lay.Bc, lay.R, lay.st[0].W, lay.st[0].P, lay.st[0].gamma,
                             reinterpret_cast<double*>(base + lay.st[0].off_b64),
                             reinterpret_cast<float*>(base + lay.st[0].off_b32),
                             reinterpret_cast<double*>(base + lay.off_bound), s);
    if (e != hipSuccess) return fail(BMND_E_HIP, std::string("HIP: ") + hipGetErrorString(e));
    CorrEntry ent;
    ent.ndim = geom->ndim;
    for (int d = 0; d < geom->ndim; ++d) ent.shape[d] = geom->shape[d];
    ent.lay = lay;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_corr[d_tables] = ent;
    return BMND_OK;
}

bmnd_status correlated_bind(const void* d_corr, const bmnd_geometry* geom,
                            const bmnd_stage_params* sp, int stage, StageCfg& c)
{
    CorrEntry ent;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_corr.find(d_corr);
        if (it == g_corr.end())
            return fail(BMND_E_ARG, "noise.d_corr was not written by bmnd_correlated_prepare");
        ent = it->second;
    }
    const int k = stage == BMND_STAGE_HT ? 0 : 1;
    const CorrLayout::Stage& S = ent.lay.st[k];
    bool same = same_shape(ent, geom) && S.spatial == sp->spatial && S.gamma == sp->gamma;
    for (int d = 0; d < kAx; ++d) same = same && S.j[d] == c.g.j[d] && S.W[d] == c.g.W[d];
    if (!same)
        return fail(BMND_E_ARG, "noise.d_corr was prepared for another shape or stage parameters");
    const unsigned char* base = static_cast<const unsigned char*>(d_corr);
    c.corr.dtab = reinterpret_cast<const double*>(base + S.off_d);
    if (k == 0) {
        c.corr.bias = reinterpret_cast<const double*>(base + S.off_b64);
        c.corr.bias32 = reinterpret_cast<const float*>(base + S.off_b32);
        c.corr.bias_bound = reinterpret_cast<const double*>(base + ent.lay.off_bound);
    }
    for (int d = 0; d < kAx; ++d) c.corr.bw[d] = S.bw[d];
    return BMND_OK;
}

}  // namespace bmnd

extern "C" {

const char* bmnd_last_error(void) { return t_error.c_str(); }

const char* bmnd_version(void) { return "bmnd-mi355x 0.1 (gfx950)"; }

bmnd_status bmnd_params_default(int32_t preset, int32_t ndim, bmnd_params* out)
{
    if (!out) return fail(BMND_E_ARG, "out is NULL");
    if (preset != BMND_PRESET_PLAIN && preset != BMND_PRESET_STANDARD)
        return fail(BMND_E_ARG, "unknown preset");
    if (ndim < 1 || ndim > BMND_MAX_AXES) return fail(BMND_E_ARG, "ndim out of range");
    out->ht = preset_stage(preset, ndim, BMND_STAGE_HT);
    out->wiener = preset_stage(preset, ndim, BMND_STAGE_WIENER);
    return BMND_OK;
}

bmnd_status bmnd_reference_origins(const bmnd_geometry* geom, const bmnd_stage_params* sp,
                                   int64_t* out_lin, int64_t cap, int64_t* n_out)
{
    if (!n_out) return fail(BMND_E_ARG, "n_out is NULL");
    bmnd_status st = check_geometry(geom);
    if (st != BMND_OK) return st;
    if (!sp) return fail(BMND_E_ARG, "stage parameters are NULL");
    for (int d = 0; d < geom->ndim; ++d) {
        if (sp->patch[d] < 1 || sp->patch[d] > geom->shape[d])
            return fail(BMND_E_ARG, "patch must satisfy 1 <= j_d <= L_d");
        if (sp->step[d] < 1) return fail(BMND_E_ARG, "step must be >= 1");
    }
    if (sp->passes < 1 || !(sp->shift_density >= 0.0) || sp->schedule < 0 || sp->schedule > 3)
        return fail(BMND_E_ARG, "bad schedule parameters");
    std::vector<int64_t> o = reference_origins(*geom, *sp);
    *n_out = int64_t(o.size());
    if (out_lin && cap > 0)
        std::memcpy(out_lin, o.data(), sizeof(int64_t) * size_t(std::min<int64_t>(cap, *n_out)));
    return BMND_OK;
}

bmnd_status bmnd_cache_limits(size_t host_bytes, size_t device_bytes)
{
    std::vector<std::shared_ptr<const std::vector<int64_t>>> d1;
    std::vector<std::shared_ptr<const HostBlocks>> d2;
    std::vector<std::shared_ptr<const DevList>> d3;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        host_origin_cache().set_cap(host_bytes ? host_bytes : kHostCacheBytes, d1);
        host_block_cache().set_cap(host_bytes ? host_bytes : kHostCacheBytes, d2);
        device_list_cache().set_cap(device_bytes ? device_bytes : kDeviceCacheBytes, d3);
    }
    return BMND_OK;   // evicted entries are released here, outside the lock
}

bmnd_status bmnd_reference_coverage(const bmnd_geometry* geom, const bmnd_stage_params* sp,
                                    uint32_t* out_map, double* stats)
{
    int64_t n = 0;
    bmnd_status st = bmnd_reference_origins(geom, sp, nullptr, 0, &n);
    if (st != BMND_OK) return st;
    const std::vector<uint32_t> c = coverage_map(*geom, *sp);
    if (stats) {
        // mean and population standard deviation from the histogram of C
        std::map<uint32_t, int64_t> hist;
        int64_t sum = 0;
        for (uint32_t v : c) {
            ++hist[v];
            sum += v;
        }
        const double V = double(c.size());
        const double mean = double(sum) / V;
        double ss = 0.0;
        for (const auto& kv : hist) {
            const double dv = double(kv.first) - mean;
            ss += double(kv.second) * dv * dv;
        }
        const double sd = std::sqrt(ss / V);
        stats[0] = mean;
        stats[1] = sd;
        stats[2] = mean > 0.0 ? sd / mean : 0.0;
    }
    if (out_map) std::memcpy(out_map, c.data(), c.size() * sizeof(uint32_t));
    return BMND_OK;
}

bmnd_status bmnd_transform_matrices(int32_t spatial, int32_t n, double* T, double* U)
{
    if (n < 1 || n > 1024) return fail(BMND_E_ARG, "n out of range");
    if (spatial < BMND_SPATIAL_IDENTITY || spatial > BMND_SPATIAL_BIOR15)
        return fail(BMND_E_ARG, "unknown spatial transform");
    std::vector<double> t, u;
    spatial_matrices(spatial, n, t, u);
    if (T) std::memcpy(T, t.data(), sizeof(double) * t.size());
    if (U) std::memcpy(U, u.data(), sizeof(double) * u.size());
    return BMND_OK;
}

bmnd_status bmnd_count_moments(int32_t metric, int32_t nmax, double* mu, double* v)
{
    if (metric < BMND_METRIC_DEVIANCE || metric > BMND_METRIC_ANSCOMBE)
        return fail(BMND_E_ARG, "moments exist for the Poisson metrics only");
    if (nmax < 0 || nmax > BMND_MOMENT_MAX_COUNT || !mu || !v)
        return fail(BMND_E_ARG, "nmax out of range or NULL output");
    std::vector<double> m, w;
    count_moments_host(metric, nmax, m, w);
    std::copy(m.begin(), m.end(), mu);
    std::copy(w.begin(), w.end(), v);
    return BMND_OK;
}

bmnd_status bmnd_correlated_size(const bmnd_geometry* geom, const bmnd_params* params,
                                 size_t* bytes)
{
    set_error("");
    return correlated_size(geom, params, bytes);
}

bmnd_status bmnd_correlated_prepare(const double* d_psd, const bmnd_geometry* geom,
                                    const bmnd_params* params, void* d_tables, size_t bytes,
                                    void* stream)
{
    set_error("");
    return correlated_prepare(d_psd, geom, params, d_tables, bytes,
                              static_cast<hipStream_t>(stream));
}

bmnd_status bmnd_haar_matrix(int32_t K, double* H)
{
    if (!is_pow2(K) || K > 1024) return fail(BMND_E_ARG, "K must be a power of two");
    std::vector<double> h;
    haar_matrix(K, h);
    if (H) std::memcpy(H, h.data(), sizeof(double) * h.size());
    return BMND_OK;
}

bmnd_status bmnd_kaiser_window(int32_t n, double beta, double* w)
{
    if (n < 1 || !(beta >= 0.0)) return fail(BMND_E_ARG, "bad window arguments");
    std::vector<double> v = kaiser_window(n, beta);
    if (w) std::memcpy(w, v.data(), sizeof(double) * v.size());
    return BMND_OK;
}

bmnd_status bmnd_match_workspace_size(const bmnd_geometry* geom, const bmnd_stage_params* sp,
                                      size_t* bytes)
{
    if (!bytes) return fail(BMND_E_ARG, "bytes is NULL");
    StageCfg c;
    bmnd_status st = make_stage(geom, nullptr, sp, BMND_STAGE_HT, c);
    if (st != BMND_OK && st != BMND_E_ARG) return st;
    Geo g = make_geo(geom, sp);
    *bytes = match_ws(g);
    return BMND_OK;
}

bmnd_status bmnd_aggregate_workspace_size(const bmnd_geometry* geom,
                                          const bmnd_stage_params* sp, size_t* bytes)
{
    if (!bytes) return fail(BMND_E_ARG, "bytes is NULL");
    bmnd_status st = check_geometry(geom);
    if (st != BMND_OK) return st;
    if (!sp) return fail(BMND_E_ARG, "stage parameters are NULL");
    *bytes = agg_ws(make_geo(geom, sp));
    return BMND_OK;
}

static bmnd_status denoise_layout(const bmnd_geometry* geom, const bmnd_params* params,
                                  int64_t n_ht, int64_t n_wie, size_t* offs, size_t* total)
{
    const Geo g = make_geo(geom, &params->ht);
    const size_t vox = size_t(g.batch) * g.V;
    const size_t nm = std::max(size_t(n_ht) * params->ht.group_max,
                               size_t(n_wie) * params->wiener.group_max);
    const size_t nr = size_t(std::max(n_ht, n_wie));
    size_t o = 0;
    offs[0] = o; o += align256(size_t(g.batch) * nm * sizeof(int));      // match
    offs[1] = o; o += align256(size_t(g.batch) * nr * sizeof(int));      // count
    offs[2] = o; o += align256(vox * sizeof(int));                        // kappa
    offs[3] = o; o += align256(vox * sizeof(int));                        // psum
    offs[4] = o; o += align256(vox * sizeof(double));                     // num
    offs[5] = o; o += align256(vox * sizeof(double));                     // den
    offs[6] = o; o += align256(vox * sizeof(float));                      // pilot
    offs[7] = o; o += align256(vox * sizeof(double));                     // per-origin weights
    // 1 / eta for the second mass-conservation sweep of the N-D filter
    const bool rd = params->ht.mass_conservation || params->wiener.mass_conservation;
    offs[8] = o; o += rd ? align256(vox * sizeof(double)) : 0;
    // hard-threshold stage with mass conservation: each member's decisions
    // and weight from the filter's first sweep to its second
    const bool hs = params->ht.mass_conservation != 0;
    offs[9] = o;
    o += hs ? align256(nd_sweep_state_bytes(long(g.batch) * n_ht, params->ht.group_max)) : 0;
    *total = o;
    return BMND_OK;
}

bmnd_status bmnd_workspace_size(const bmnd_geometry* geom, const bmnd_noise* noise,
                                const bmnd_params* params, size_t* bytes)
{
    if (!bytes || !params) return fail(BMND_E_ARG, "NULL argument");
    StageCfg c1, c2;
    bmnd_status st = make_stage(geom, noise, &params->ht, BMND_STAGE_HT, c1);
    if (st != BMND_OK) return st;
    if ((st = make_stage(geom, noise, &params->wiener, BMND_STAGE_WIENER, c2)) != BMND_OK) return st;
    bmnd_geometry one = *geom;
    one.batch = 1;
    const int64_t n1 = int64_t(host_origins_cached(one, params->ht)->size());
    const int64_t n2 = int64_t(host_origins_cached(one, params->wiener)->size());
    size_t offs[10];
    return denoise_layout(geom, params, n1, n2, offs, bytes);
}

bmnd_status bmnd_workspace_sums(const bmnd_geometry* geom, const bmnd_noise* noise,
                                const bmnd_params* params, size_t* num_offset,
                                size_t* den_offset)
{
    if (!num_offset || !den_offset || !params) return fail(BMND_E_ARG, "NULL argument");
    size_t total = 0;
    bmnd_status st = bmnd_workspace_size(geom, noise, params, &total);
    if (st != BMND_OK) return st;
    bmnd_geometry one = *geom;
    one.batch = 1;
    size_t offs[10];
    st = denoise_layout(geom, params, int64_t(host_origins_cached(one, params->ht)->size()),
                        int64_t(host_origins_cached(one, params->wiener)->size()), offs, &total);
    if (st != BMND_OK) return st;
    *num_offset = offs[4];
    *den_offset = offs[5];
    return BMND_OK;
}

bmnd_status bmnd_request_bytes(const bmnd_geometry* geom, const bmnd_noise* noise,
                               const bmnd_params* params, size_t budget, size_t* bytes)
{
    if (!bytes) return fail(BMND_E_ARG, "NULL argument");
    size_t ws = 0;
    bmnd_status st = bmnd_workspace_size(geom, noise, params, &ws);
    if (st != BMND_OK) return st;
    size_t arrays = 2 * sizeof(float) * size_t(geom->batch);
    for (int d = 0; d < geom->ndim; ++d) arrays *= size_t(geom->shape[d]);
    *bytes = ws + arrays;
    if (budget > 0 && *bytes > budget)
        return fail(BMND_E_BUDGET, "the request needs " + std::to_string(*bytes) +
                                       " bytes of device memory, more than the budget of " +
                                       std::to_string(budget));
    return BMND_OK;
}

bmnd_status bmnd_match(int32_t stage, const float* d_src, const bmnd_geometry* geom,
                       const bmnd_noise* noise, const bmnd_stage_params* sp,
                       const int64_t* d_refs, int64_t n_refs, int32_t* d_match,
                       int32_t* d_count, float* d_score, void* d_ws, size_t ws_bytes,
                       void* stream)
{
    StageCfg c;
    bmnd_status st = make_stage(geom, noise, sp, stage, c);
    if (st != BMND_OK) return st;
    if (!noise) return fail(BMND_E_ARG, "noise is NULL");
    if (!d_src || !d_match || !d_count || (n_refs > 0 && !d_refs))
        return fail(BMND_E_ARG, "NULL device pointer");
    if (n_refs < 0 || n_refs * int64_t(c.g.batch) >= 2147483647LL)
        return fail(BMND_E_ARG, "n_refs out of range");
    if (n_refs == 0) return BMND_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int* kappa = nullptr;
    int* psum = nullptr;
    if (c.integral) {
        if (!d_ws || ws_bytes < match_ws(c.g))
            return fail(BMND_E_WORKSPACE, "workspace missing or smaller than bmnd_match_workspace_size");
        kappa = static_cast<int*>(d_ws);
        psum = reinterpret_cast<int*>(static_cast<char*>(d_ws) + match_ws(c.g) / 2);
    }
    const MomentTables* mom = nullptr;
    if (c.metric != BMND_METRIC_SSD) {
        std::string err;
        if (!(mom = device_moments(c.metric, err))) return fail(BMND_E_NOMEM, err);
    }
    hipError_t e = launch_match(c, d_src, kappa, psum, d_refs, int(n_refs), d_match, d_count, s,
                                mom);
    if (e != hipSuccess) return hip_fail(e, "matching kernel");
    if (d_score) {
        e = launch_member_scores(c, d_src, d_match, d_count, int(n_refs), d_score, mom, s);
        if (e != hipSuccess) return hip_fail(e, "member score kernel");
    }
    return BMND_OK;
}

bmnd_status bmnd_filter(int32_t stage, const float* d_y, const float* d_pilot,
                        const bmnd_geometry* geom, const bmnd_noise* noise,
                        const bmnd_stage_params* sp, int64_t n_refs, const int32_t* d_match,
                        const int32_t* d_count, float* d_patches, float* d_weights,
                        void* stream)
{
    StageCfg c;
    bmnd_status st = make_stage(geom, noise, sp, stage, c);
    if (st != BMND_OK) return st;
    if (!noise) return fail(BMND_E_ARG, "noise is NULL");
    if (!d_y || !d_match || !d_count || !d_patches || !d_weights)
        return fail(BMND_E_ARG, "NULL device pointer");
    if (stage == BMND_STAGE_WIENER && !d_pilot)
        return fail(BMND_E_ARG, "the Wiener stage needs the pilot");
    if (n_refs < 0 || n_refs * int64_t(c.g.batch) >= 2147483647LL)
        return fail(BMND_E_ARG, "n_refs out of range");
    if (n_refs == 0) return BMND_OK;
    std::string err;
    const DevTables* t = device_tables(c, err);
    if (!t) return fail(BMND_E_NOMEM, err);
    hipError_t e = launch_filter(c, *t, 0, d_y, d_pilot, int(n_refs), d_match, d_count, d_patches,
                                 d_weights, nullptr, nullptr, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "filter kernel");
    return BMND_OK;
}

bmnd_status bmnd_aggregate(const float* d_y, const bmnd_geometry* geom,
                           const bmnd_stage_params* sp, int64_t n_refs,
                           const int32_t* d_match, const int32_t* d_count,
                           const float* d_patches, const float* d_weights, float* d_out,
                           void* d_ws, size_t ws_bytes, void* stream)
{
    bmnd_status st = check_geometry(geom);
    if (st != BMND_OK) return st;
    if (!sp) return fail(BMND_E_ARG, "stage parameters are NULL");
    // the stage only matters for validation of the shrink/stage pairing
    const int stage = sp->shrink == BMND_SHRINK_WIENER ? BMND_STAGE_WIENER : BMND_STAGE_HT;
    StageCfg c;
    if ((st = make_stage(geom, nullptr, sp, stage, c)) != BMND_OK) return st;
    if (!d_match || !d_count || !d_patches || !d_weights || !d_out || (c.mc && !d_y))
        return fail(BMND_E_ARG, "NULL device pointer");
    if (!d_ws || ws_bytes < agg_ws(c.g))
        return fail(BMND_E_WORKSPACE, "workspace missing or smaller than bmnd_aggregate_workspace_size");
    if (n_refs < 0 || n_refs * int64_t(c.g.batch) >= 2147483647LL)
        return fail(BMND_E_ARG, "n_refs out of range");
    std::string err;
    const DevTables* t = device_tables(c, err);
    if (!t) return fail(BMND_E_NOMEM, err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* num = d_ws;
    void* den = static_cast<char*>(d_ws) + agg_ws(c.g) / 2;
    hipError_t e = launch_zero(d_ws, agg_ws(c.g), s);
    if (e == hipSuccess && n_refs > 0) {
        if (c.mc) {
            e = launch_aggregate(c, *t, 2, d_y, int(n_refs), d_match, d_count, d_patches,
                                 d_weights, num, den, s);
            if (e == hipSuccess)
                e = launch_aggregate(c, *t, 3, d_y, int(n_refs), d_match, d_count, d_patches,
                                     d_weights, num, den, s);
        } else {
            e = launch_aggregate(c, *t, 1, d_y, int(n_refs), d_match, d_count, d_patches,
                                 d_weights, num, den, s);
        }
    }
    if (e == hipSuccess) e = launch_normalize(c, num, den, d_out, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "aggregation kernels");
    return BMND_OK;
}

}  // extern "C"

namespace bmnd {

// host part: configurations, reference counts and the workspace layout
bmnd_status plan_denoise_host(const bmnd_geometry* geom, const bmnd_noise* noise,
                              const bmnd_params* params, DenoisePlan* pl)
{
    if (!params) return fail(BMND_E_ARG, "params is NULL");
    bmnd_status st = make_stage(geom, noise, &params->ht, BMND_STAGE_HT, pl->c1);
    if (st != BMND_OK) return st;
    if ((st = make_stage(geom, noise, &params->wiener, BMND_STAGE_WIENER, pl->c2)) != BMND_OK)
        return st;
    if (!noise) return fail(BMND_E_ARG, "noise is NULL");
    bmnd_geometry one = *geom;
    one.batch = 1;
    pl->n1 = int64_t(host_origins_cached(one, params->ht)->size());
    pl->n2 = int64_t(host_origins_cached(one, params->wiener)->size());
    pl->nd1 = stage_uses_nd(pl->c1) && nd_blocks_fit(host_blocks_cached(one, params->ht, pl->c1.g)->blk);
    pl->nd2 = stage_uses_nd(pl->c2) &&
              nd_blocks_fit(host_blocks_cached(one, params->wiener, pl->c2.g)->blk);
    return denoise_layout(geom, params, pl->n1, pl->n2, pl->offs, &pl->total);
}

bmnd_status plan_denoise(const bmnd_geometry* geom, const bmnd_noise* noise,
                         const bmnd_params* params, DenoisePlan* pl, hipStream_t s)
{
    if (!params) return fail(BMND_E_ARG, "params is NULL");
    bmnd_status st = make_stage(geom, noise, &params->ht, BMND_STAGE_HT, pl->c1);
    if (st != BMND_OK) return st;
    if ((st = make_stage(geom, noise, &params->wiener, BMND_STAGE_WIENER, pl->c2)) != BMND_OK)
        return st;
    if (!noise) return fail(BMND_E_ARG, "noise is NULL");
    std::string err;
    bmnd_geometry one = *geom;
    one.batch = 1;
    pl->nd1 = stage_uses_nd(pl->c1) && nd_blocks_fit(host_blocks_cached(one, params->ht, pl->c1.g)->blk);
    pl->nd2 = stage_uses_nd(pl->c2) &&
              nd_blocks_fit(host_blocks_cached(one, params->wiener, pl->c2.g)->blk);
    auto l1 = device_list(one, params->ht, pl->c1.g, pl->nd1, s, err);
    auto l2 = l1 ? device_list(one, params->wiener, pl->c2.g, pl->nd2, s, err) : nullptr;
    if (!l1 || !l2) return fail(BMND_E_NOMEM, err);
    pl->r1 = l1->refs;
    pl->n1 = l1->n;
    pl->r2 = l2->refs;
    pl->n2 = l2->n;
    if (pl->nd1) pl->blk1 = l1->blk;
    if (pl->nd2) pl->blk2 = l2->blk;
    pl->keep[0] = l1;
    pl->keep[1] = l2;
    pl->ready[0] = l1->ready;
    pl->ready[1] = l2->ready;
    pl->t1 = device_tables(pl->c1, err);
    pl->t2 = pl->t1 ? device_tables(pl->c2, err) : nullptr;
    if (!pl->t1 || !pl->t2) return fail(BMND_E_NOMEM, err);
    if (pl->c1.metric != BMND_METRIC_SSD && !(pl->m1 = device_moments(pl->c1.metric, err)))
        return fail(BMND_E_NOMEM, err);
    return denoise_layout(geom, params, pl->n1, pl->n2, pl->offs, &pl->total);
}

// The two stages of one denoise on stream s (workspace ws of pl.total bytes).
hipError_t enqueue_denoise(const DenoisePlan& pl, const float* d_y, float* d_out,
                           float* d_pilot, char* ws, hipStream_t s, bool spans, bool from_pilot)
{
    int* match = reinterpret_cast<int*>(ws + pl.offs[0]);
    int* count = reinterpret_cast<int*>(ws + pl.offs[1]);
    int* kappa = reinterpret_cast<int*>(ws + pl.offs[2]);
    int* psum = reinterpret_cast<int*>(ws + pl.offs[3]);
    void* num = ws + pl.offs[4];
    void* den = ws + pl.offs[5];
    float* pilot = d_pilot ? d_pilot : reinterpret_cast<float*>(ws + pl.offs[6]);
    double* wf = reinterpret_cast<double*>(ws + pl.offs[7]);
    double* rden = reinterpret_cast<double*>(ws + pl.offs[8]);
    void* hstate = ws + pl.offs[9];
    const size_t vox = size_t(pl.c1.g.batch) * pl.c1.g.V;
    {
        // the origin lists' uploads, if another stream queued them
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        (void)hipStreamIsCapturing(s, &cs);
        for (hipEvent_t ev : pl.ready)
            if (ev && cs == hipStreamCaptureStatusNone) {
                const hipError_t e = hipStreamWaitEvent(s, ev, 0);
                if (e != hipSuccess) return e;
            }
    }
    const int no_span = -1;

    auto run_stage = [&](const StageCfg& c, const DevTables& t, const int64_t* refs, int64_t nr,
                         const float* src, const float* pil, float* out) -> hipError_t {
        const bool ht = c.stage == BMND_STAGE_HT;
        const bool nd = ht ? pl.nd1 : pl.nd2;
        const NdBlocks* blk = ht ? &pl.blk1 : &pl.blk2;
        hipError_t e = hipSuccess;
        {
            KernelSpan k(spans ? (ht ? BMND_KID_MATCH_HT : BMND_KID_MATCH_WIENER) : no_span, s);
            e = launch_match(c, src, kappa, psum, refs, int(nr), match, count, s,
                             ht ? pl.m1 : nullptr, nd ? blk : nullptr);
        }
        if (e == hipSuccess) {
            KernelSpan k(spans ? BMND_KID_ZERO : no_span, s);
            e = launch_zero(num, vox * sizeof(double), s);
            if (e == hipSuccess) e = launch_zero(nd ? wf : den, vox * sizeof(double), s);
        }
        if (e != hipSuccess) return e;
        {
            KernelSpan k(spans ? (ht ? BMND_KID_FILTER_HT : BMND_KID_FILTER_WIENER) : no_span, s);
            if (nd) {
                // per-origin weights W, eta = W * window, numerator in boxes
                if (c.mc) {
                    // sweep 2 reads 1 / eta (into the reciprocal region)
                    void* st = ht ? hstate : nullptr;
                    e = launch_filter_blocked(c, t, 2, d_y, pil, int(nr), match, count, num, den,
                                              wf, blk, st, s);
                    if (e == hipSuccess)
                        e = launch_window_conv(c.g, t, wf, static_cast<double*>(den), rden, s);
                    if (e == hipSuccess)
                        e = launch_filter_blocked(c, t, 3, d_y, pil, int(nr), match, count, num,
                                                  rden, wf, blk, st, s);
                } else {
                    e = launch_filter_blocked(c, t, 1, d_y, pil, int(nr), match, count, num, den,
                                              wf, blk, nullptr, s);
                    if (e == hipSuccess)
                        e = launch_window_conv(c.g, t, wf, static_cast<double*>(den), nullptr, s);
                }
            } else if (c.mc) {
                e = launch_filter(c, t, 2, d_y, pil, int(nr), match, count, nullptr, nullptr, num,
                                  den, s);
                if (e == hipSuccess)
                    e = launch_filter(c, t, 3, d_y, pil, int(nr), match, count, nullptr, nullptr,
                                      num, den, s);
            } else {
                e = launch_filter(c, t, 1, d_y, pil, int(nr), match, count, nullptr, nullptr, num,
                                  den, s);
            }
        }
        if (e == hipSuccess) {
            KernelSpan k(spans ? BMND_KID_NORMALIZE : no_span, s);
            e = launch_normalize(c, num, den, out, nullptr, s);
        }
        return e;
    };
    if (!from_pilot) {
        hipError_t e = run_stage(pl.c1, *pl.t1, pl.r1, pl.n1, d_y, nullptr, pilot);
        if (e != hipSuccess) return e;
    }
    return run_stage(pl.c2, *pl.t2, pl.r2, pl.n2, pilot, pilot, d_out);
}

}  // namespace bmnd

namespace {

// ------------------------------------------------------------- batches

constexpr int kBatchStreams = 4;  // concurrent streams (the device's hardware queues)

// Library streams and events of one device for batches; calls of
// bmnd_denoise_batch are serialized per process.
struct BatchPool {
    hipStream_t work[kBatchStreams] = {};
    hipStream_t capture = nullptr;
    hipEvent_t fork = nullptr, in = nullptr, out = nullptr;
    hipEvent_t join[kBatchStreams] = {};
    std::map<std::string, hipGraphExec_t> graphs;  // launch sequences by job table
    // the device lists each cached graph reads (kept while it may replay)
    std::map<std::string, std::vector<std::shared_ptr<const void>>> graph_keep;
    std::vector<std::string> order;                // insertion order (eviction)
};
std::mutex g_batch_mu;
std::map<int, BatchPool> g_pools;
constexpr size_t kMaxGraphs = 16;

hipError_t pool_for_device(BatchPool** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    auto it = g_pools.find(dev);
    if (it != g_pools.end()) {
        *out = &it->second;
        return hipSuccess;
    }
    BatchPool p;
    for (int i = 0; i < kBatchStreams && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&p.work[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p.capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p.in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p.out, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    *out = &(g_pools[dev] = p);
    return hipSuccess;
}

// Work estimate of a job (candidate patch-samples of both stages).
double job_work(const DenoisePlan& pl)
{
    double cand = 1.0;
    for (int d = 0; d < kAx; ++d) cand *= pl.c1.g.W[d];
    return double(pl.c1.g.batch) * double(pl.n1 + pl.n2) * cand * pl.c1.g.P + 1.0;
}

// Jobs go to streams longest first, each to the least loaded stream; jobs
// on one stream run one after another and share that stream's workspace.
struct BatchLayout {
    std::vector<DenoisePlan> plans;
    std::vector<int> stream_of;
    std::vector<size_t> ws_off;  // per stream
    size_t total = 0;
};

bmnd_status layout_batch(int32_t n_jobs, const bmnd_job* jobs, BatchLayout* L, bool device,
                         hipStream_t s = nullptr)
{
    if (n_jobs < 0) return fail(BMND_E_ARG, "n_jobs < 0");
    if (n_jobs > 0 && !jobs) return fail(BMND_E_ARG, "jobs is NULL");
    L->plans.assign(size_t(n_jobs), DenoisePlan{});
    std::vector<int> idx(static_cast<size_t>(n_jobs));
    std::vector<double> work(static_cast<size_t>(n_jobs));
    for (int i = 0; i < n_jobs; ++i) {
        DenoisePlan* pl = &L->plans[size_t(i)];
        const bmnd_status st = device ? plan_denoise(&jobs[i].geom, &jobs[i].noise, &jobs[i].params, pl, s)
                                      : plan_denoise_host(&jobs[i].geom, &jobs[i].noise, &jobs[i].params, pl);
        if (st != BMND_OK) {
            set_error("job " + std::to_string(i) + ": " + bmnd_last_error());
            return st;
        }
        idx[size_t(i)] = i;
        work[size_t(i)] = job_work(L->plans[size_t(i)]);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work[size_t(a)] > work[size_t(b)]; });
    double load[kBatchStreams] = {};
    size_t need[kBatchStreams] = {};
    L->stream_of.assign(size_t(n_jobs), 0);
    for (int i : idx) {
        int best = 0;
        for (int k = 1; k < kBatchStreams; ++k)
            if (load[k] < load[best]) best = k;
        load[best] += work[size_t(i)];
        need[best] = std::max(need[best], L->plans[size_t(i)].total);
        L->stream_of[size_t(i)] = best;
    }
    L->ws_off.assign(kBatchStreams, 0);
    size_t o = 0;
    for (int k = 0; k < kBatchStreams; ++k) {
        L->ws_off[size_t(k)] = o;
        o += align256(need[k]);
    }
    L->total = o;
    return BMND_OK;
}

// Fork from `from` onto the work streams, enqueue every job in stream
// order (longest first), join back into `from`.
hipError_t enqueue_batch(BatchPool& P, const BatchLayout& L, int32_t n_jobs, const bmnd_job* jobs,
                         char* ws, hipStream_t from)
{
    hipError_t e = hipEventRecord(P.fork, from);
    for (int k = 0; k < kBatchStreams && e == hipSuccess; ++k) e = hipStreamWaitEvent(P.work[k], P.fork, 0);
    std::vector<int> idx(static_cast<size_t>(n_jobs));
    for (int i = 0; i < n_jobs; ++i) idx[size_t(i)] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return job_work(L.plans[size_t(a)]) > job_work(L.plans[size_t(b)]);
    });
    for (int i : idx) {
        if (e != hipSuccess) break;
        const int k = L.stream_of[size_t(i)];
        e = enqueue_denoise(L.plans[size_t(i)], jobs[i].d_y, jobs[i].d_out, jobs[i].d_pilot,
                            ws + L.ws_off[size_t(k)], P.work[k], false);
    }
    for (int k = 0; k < kBatchStreams && e == hipSuccess; ++k) {
        e = hipEventRecord(P.join[k], P.work[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(from, P.join[k], 0);
    }
    return e;
}

}  // namespace

extern "C" {

bmnd_status bmnd_denoise(const float* d_y, const bmnd_geometry* geom,
                         const bmnd_noise* noise, const bmnd_params* params, float* d_out,
                         float* d_pilot, void* d_ws, size_t ws_bytes, void* stream)
{
    DenoisePlan pl;
    bmnd_status st = plan_denoise(geom, noise, params, &pl, static_cast<hipStream_t>(stream));
    if (st != BMND_OK) return st;
    if (!d_y || !d_out) return fail(BMND_E_ARG, "NULL device pointer");
    if (!d_ws || ws_bytes < pl.total)
        return fail(BMND_E_WORKSPACE, "workspace missing or smaller than bmnd_workspace_size");
    hipError_t e = enqueue_denoise(pl, d_y, d_out, d_pilot, static_cast<char*>(d_ws),
                                   static_cast<hipStream_t>(stream), true);
    if (e != hipSuccess) return hip_fail(e, "denoise");
    return BMND_OK;
}

bmnd_status bmnd_denoise_from_pilot(const float* d_y, const float* d_pilot,
                                    const bmnd_geometry* geom, const bmnd_noise* noise,
                                    const bmnd_params* params, float* d_out, void* d_ws,
                                    size_t ws_bytes, void* stream)
{
    DenoisePlan pl;
    bmnd_status st = plan_denoise(geom, noise, params, &pl, static_cast<hipStream_t>(stream));
    if (st != BMND_OK) return st;
    if (!d_y || !d_pilot || !d_out) return fail(BMND_E_ARG, "NULL device pointer");
    if (!d_ws || ws_bytes < pl.total)
        return fail(BMND_E_WORKSPACE, "workspace missing or smaller than bmnd_workspace_size");
    // the Wiener stage only reads the pilot (matching, gathers, gains)
    hipError_t e = enqueue_denoise(pl, d_y, d_out, const_cast<float*>(d_pilot),
                                   static_cast<char*>(d_ws), static_cast<hipStream_t>(stream),
                                   true, true);
    if (e != hipSuccess) return hip_fail(e, "denoise from pilot");
    return BMND_OK;
}

static_assert(kNumBlockRules == BMND_BLOCK_RULES, "block rules and the C ABI disagree");

bmnd_status bmnd_autotune(const float* d_y, const bmnd_geometry* geom, const bmnd_noise* noise,
                          const bmnd_params* params, float* d_out, void* d_ws, size_t ws_bytes,
                          void* stream, int32_t* chosen, double* ms)
{
    if (chosen) *chosen = -1;
    DenoisePlan pl;
    bmnd_status st = plan_denoise(geom, noise, params, &pl, static_cast<hipStream_t>(stream));
    if (st != BMND_OK) return st;
    if (!d_y || !d_out) return fail(BMND_E_ARG, "NULL device pointer");
    if (!d_ws || ws_bytes < pl.total)
        return fail(BMND_E_WORKSPACE, "workspace missing or smaller than bmnd_workspace_size");
    if (ms)
        for (int r = 0; r < kNumBlockRules; ++r) ms[r] = -1.0;
    if (!pl.nd1 && !pl.nd2) return BMND_OK;   // no spatial blocks: nothing to tune
    bmnd_geometry one = *geom;
    one.batch = 1;
    const TuneKey k1 = tune_key(one, params->ht), k2 = tune_key(one, params->wiener);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(BMND_E_HIP, "event creation failed");
    auto set_rule = [&](int r) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_block_rule[k1] = r;
        g_block_rule[k2] = r;
    };
    int best = 0;
    float best_ms = 0.f;
    hipError_t e = hipSuccess;
    for (int r = 0; r < kNumBlockRules && e == hipSuccess; ++r) {
        set_rule(r);
        DenoisePlan q;
        if (plan_denoise(geom, noise, params, &q, s) != BMND_OK) continue;
        // a candidate whose boxes do not fit keeps the older kernels: skipped
        if (q.nd1 != pl.nd1 || q.nd2 != pl.nd2) continue;
        float t = 0.f;
        e = enqueue_denoise(q, d_y, d_out, nullptr, static_cast<char*>(d_ws), s, false);
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            if (e == hipSuccess) e = hipEventRecord(a, s);
            if (e == hipSuccess) e = enqueue_denoise(q, d_y, d_out, nullptr, static_cast<char*>(d_ws), s, false);
            if (e == hipSuccess) e = hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float m = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&m, a, b);
            t = rep == 0 ? m : std::min(t, m);
        }
        if (e != hipSuccess) break;
        if (ms) ms[r] = double(t);
        // another rule replaces rule 0 (and a later rule an earlier one) only
        // when at least 3 % faster, so timing noise does not flip the choice
        if (r == 0 || t < 0.97f * best_ms) {
            best = r;
            best_ms = t;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    set_rule(best);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    // the output of the chosen rule
    DenoisePlan q;
    if ((st = plan_denoise(geom, noise, params, &q, s)) != BMND_OK) return st;
    e = enqueue_denoise(q, d_y, d_out, nullptr, static_cast<char*>(d_ws), s, false);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (chosen) *chosen = best;
    return BMND_OK;
}

bmnd_status bmnd_batch_workspace_size(int32_t n_jobs, const bmnd_job* jobs, size_t* bytes)
{
    if (!bytes) return fail(BMND_E_ARG, "bytes is NULL");
    BatchLayout L;
    bmnd_status st = layout_batch(n_jobs, jobs, &L, false);
    if (st != BMND_OK) return st;
    *bytes = L.total;
    return BMND_OK;
}

bmnd_status bmnd_denoise_batch(int32_t n_jobs, const bmnd_job* jobs, void* d_ws, size_t ws_bytes,
                               int32_t flags, void* stream)
{
    BatchLayout L;
    bmnd_status st = layout_batch(n_jobs, jobs, &L, true, static_cast<hipStream_t>(stream));
    if (st != BMND_OK) return st;
    if (n_jobs == 0) return BMND_OK;
    for (int i = 0; i < n_jobs; ++i)
        if (!jobs[i].d_y || !jobs[i].d_out) return fail(BMND_E_ARG, "NULL device pointer in a job");
    if (!d_ws || ws_bytes < L.total)
        return fail(BMND_E_WORKSPACE, "workspace missing or smaller than bmnd_batch_workspace_size");
    if (flags & ~BMND_BATCH_GRAPH) return fail(BMND_E_ARG, "unknown batch flags");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(d_ws);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchPool* P = nullptr;
    hipError_t e = pool_for_device(&P);
    if (e != hipSuccess) return hip_fail(e, "batch streams");
    if (!(flags & BMND_BATCH_GRAPH)) {
        e = enqueue_batch(*P, L, n_jobs, jobs, ws, s);
        if (e != hipSuccess) return hip_fail(e, "batch");
        return BMND_OK;
    }
    // graph: keyed by the job table and the workspace (the launch sequence
    // depends on nothing else); captured on the library's capture stream
    std::string key(reinterpret_cast<const char*>(jobs), sizeof(bmnd_job) * size_t(n_jobs));
    key.append(reinterpret_cast<const char*>(&d_ws), sizeof(d_ws));
    hipGraphExec_t exec = nullptr;
    auto it = P->graphs.find(key);
    if (it != P->graphs.end()) exec = it->second;
    e = hipEventRecord(P->in, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(P->capture, P->in, 0);
    if (e == hipSuccess && !exec) {
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(P->capture, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = enqueue_batch(*P, L, n_jobs, jobs, ws, P->capture);
            e = hipStreamEndCapture(P->capture, &graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e == hipSuccess) {
            if (P->order.size() >= kMaxGraphs) {
                auto old = P->graphs.find(P->order.front());
                if (old != P->graphs.end()) {
                    (void)hipGraphExecDestroy(old->second);
                    P->graphs.erase(old);
                }
                P->graph_keep.erase(P->order.front());
                P->order.erase(P->order.begin());
            }
            P->graphs[key] = exec;
            P->order.push_back(key);
            auto& keep = P->graph_keep[key];
            for (const DenoisePlan& pl : L.plans) {
                keep.push_back(pl.keep[0]);
                keep.push_back(pl.keep[1]);
            }
        }
    }
    if (e == hipSuccess) e = hipGraphLaunch(exec, P->capture);
    if (e == hipSuccess) e = hipEventRecord(P->out, P->capture);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, P->out, 0);
    if (e != hipSuccess) return hip_fail(e, "batch graph");
    return BMND_OK;
}

bmnd_status bmnd_profile_begin(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    g_prof_on = true;
    return BMND_OK;
}

bmnd_status bmnd_profile_end(double* ms, int64_t* launches, int32_t n_ids)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = false;
    for (int i = 0; i < n_ids; ++i) {
        if (ms) ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    bmnd_status st = BMND_OK;
    for (auto& r : g_prof) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) st = hip_fail(e, "profile events");
        if (r.id < n_ids) {
            if (ms) ms[r.id] += t;
            if (launches) launches[r.id] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    return st;
}

bmnd_status bmnd_stream_status(void* stream)
{
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "stream");
    int flag = 0;
    e = read_and_clear_range_flag(&flag);
    if (e != hipSuccess) return hip_fail(e, "range flag");
    if (flag) return fail(BMND_E_RANGE, "counts outside the exact int32 scoring range");
    return BMND_OK;
}

}  // extern "C"
