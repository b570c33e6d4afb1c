// Exact finite-count moments of the Poisson matching metrics (subsection
// Exact Finite-Count Moment Calibration, Prop. universal finite-count
// moments): given the pooled count n, the reference count of a pair is
// Bin(n, 1/2) under the equal-rate null (Lemma conditional Poisson
// splitting), so mu(n) and v(n) are binomial averages of the per-entry
// contribution phi(x, n - x) and of its square.  Host code, FP64; device
// copies are library-owned and built once per metric and device.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "bmnd_internal.h"

namespace bmnd {

namespace {

// phi(x, n - x) for the pair (x, n - x) of integral counts, from tables of
// ln k: deviance 2 sum a ln(2a / n), Pearson (n - 2x)^2 / n, Anscombe
// (A(n - x) - A(x))^2 / 2 with A(k) = 2 sqrt(k + 3/8)
double phi_pair(int metric, int x, int n, const std::vector<double>& lnk)
{
    const int y = n - x;
    if (metric == BMND_METRIC_DEVIANCE) {
        if (n == 0) return 0.0;
        const double l2n = std::log(2.0) - lnk[size_t(n)];
        double v = 0.0;
        if (x > 0) v += x * (lnk[size_t(x)] + l2n);
        if (y > 0) v += y * (lnk[size_t(y)] + l2n);
        return 2.0 * v;
    }
    if (metric == BMND_METRIC_PEARSON) {
        if (n == 0) return 0.0;
        const double d = double(y - x);
        return d * d / n;
    }
    const double d = 2.0 * std::sqrt(y + 0.375) - 2.0 * std::sqrt(x + 0.375);
    return 0.5 * d * d;
}

struct MomKey {
    int dev, metric;
    bool operator<(const MomKey& o) const
    {
        return dev != o.dev ? dev < o.dev : metric < o.metric;
    }
};
std::mutex g_mom_mu;
std::map<MomKey, MomentTables> g_mom;

}  // namespace

void count_moments_host(int metric, int nmax, std::vector<double>& mu, std::vector<double>& v)
{
    mu.assign(size_t(nmax) + 1, 0.0);
    v.assign(size_t(nmax) + 1, 0.0);
    std::vector<double> lnk(size_t(nmax) + 1, 0.0);
    for (int k = 1; k <= nmax; ++k) lnk[size_t(k)] = std::log(double(k));
    const double ln2 = std::log(2.0);
    for (int n = 1; n <= nmax; ++n) {
        // log of C(n, x) 2^-n by the ratio C(n, x + 1) / C(n, x) = (n - x) / (x + 1)
        double lw = -n * ln2, m1 = 0.0, m2 = 0.0;
        for (int x = 0; x <= n; ++x) {
            if (lw > -745.0) {
                const double w = std::exp(lw);
                const double f = phi_pair(metric, x, n, lnk);
                m1 += w * f;
                m2 += w * f * f;
            }
            if (x < n) lw += lnk[size_t(n - x)] - lnk[size_t(x) + 1];
        }
        mu[size_t(n)] = m1;
        v[size_t(n)] = std::max(m2 - m1 * m1, 0.0);
    }
}

const MomentTables* device_moments(int metric, std::string& err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mom_mu);
    auto it = g_mom.find(MomKey{dev, metric});
    if (it != g_mom.end()) return &it->second;
    const int nmax = BMND_MOMENT_MAX_COUNT;
    std::vector<double> mu, v;
    count_moments_host(metric, nmax, mu, v);
    const size_t n = size_t(nmax) + 1;
    std::vector<float> f(2 * n);
    for (size_t i = 0; i < n; ++i) {
        f[i] = float(mu[i]);
        f[n + i] = float(v[i]);
    }
    std::vector<double> d(2 * n);
    for (size_t i = 0; i < n; ++i) {
        d[i] = mu[i];
        d[n + i] = v[i];
    }
    float* df = nullptr;
    double* dd = nullptr;
    if (hipMalloc(&df, f.size() * sizeof(float)) != hipSuccess ||
        hipMalloc(&dd, d.size() * sizeof(double)) != hipSuccess ||
        hipMemcpy(df, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dd, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        err = "upload of the finite-count moment tables failed";
        return nullptr;
    }
    MomentTables t;
    t.mu = df;
    t.v = df + n;
    t.mu64 = dd;
    t.v64 = dd + n;
    t.nmax = nmax;
    return &g_mom.emplace(MomKey{dev, metric}, t).first->second;
}

}  // namespace bmnd
