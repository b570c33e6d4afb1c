// Transform matrices and aggregation window (Appendix A: Haar group
// transform, bior1.5 spatial transform in the HT stage, DCT in the Wiener
// stage, Kaiser window with beta = 2).
//
// bior1.5: the synthesis lowpass is the order-1 B-spline filter
// (1, 1)/sqrt(2).  Its 10-tap dual (analysis) lowpass is obtained here as
// the solution of the linear conditions that define it: biorthogonality
// sum_n lo[n] lo~[n + 2k] = delta_k for |k| <= 2, and five
// vanishing moments of the synthesis highpass hi[t] = (-1)^t lo~[1 - t]
// (equivalently a fifth-order zero of lo~ at the Nyquist frequency).  The
// periodised multilevel synthesis operator U is assembled from (lo, hi)
// and the analysis operator is T = U^-1, inverted in double precision.
#include <algorithm>
#include <cmath>
#include <utility>

#include "bmnd_internal.h"

namespace bmnd {

namespace {

// Solve A x = b (n x n, row-major) by Gauss-Jordan with partial pivoting.
bool solve(std::vector<double> A, std::vector<double>& b, int n)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[size_t(r * n + c)]) > std::fabs(A[size_t(piv * n + c)])) piv = r;
        if (std::fabs(A[size_t(piv * n + c)]) < 1e-300) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[size_t(c * n + k)], A[size_t(piv * n + k)]);
            std::swap(b[size_t(c)], b[size_t(piv)]);
        }
        const double inv = 1.0 / A[size_t(c * n + c)];
        for (int k = 0; k < n; ++k) A[size_t(c * n + k)] *= inv;
        b[size_t(c)] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[size_t(r * n + c)];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) A[size_t(r * n + k)] -= f * A[size_t(c * n + k)];
            b[size_t(r)] -= f * b[size_t(c)];
        }
    }
    return true;
}

// Inverse of an n x n matrix (columns solved one by one).
std::vector<double> inverse(const std::vector<double>& A, int n)
{
    std::vector<double> inv(size_t(n * n), 0.0);
    for (int c = 0; c < n; ++c) {
        std::vector<double> e(size_t(n), 0.0);
        e[size_t(c)] = 1.0;
        solve(A, e, n);
        for (int r = 0; r < n; ++r) inv[size_t(r * n + c)] = e[size_t(r)];
    }
    return inv;
}

// Dual lowpass taps lo~[t], t = -4 .. 5, of the bior1.5 pair.
std::vector<double> bior15_dual_lowpass()
{
    const int n = 10;  // unknowns lo~[-4..5]
    std::vector<double> A(size_t(n * n), 0.0), b(size_t(n), 0.0);
    const double lo0 = 1.0 / std::sqrt(2.0), lo1 = lo0;  // lo[0], lo[1]
    int row = 0;
    // biorthogonality: lo[0] lo~[2k] + lo[1] lo~[2k + 1] = delta_k, k = -2..2
    for (int k = -2; k <= 2; ++k, ++row) {
        A[size_t(row * n + (2 * k + 4))] += lo0;
        A[size_t(row * n + (2 * k + 1 + 4))] += lo1;
        b[size_t(row)] = (k == 0) ? 1.0 : 0.0;
    }
    // vanishing moments: sum_t (-1)^t lo~[t] t^p = 0, p = 0..4
    for (int p = 0; p <= 4; ++p, ++row) {
        for (int t = -4; t <= 5; ++t) {
            const double sgn = (((t % 2) + 2) % 2 == 0) ? 1.0 : -1.0;
            A[size_t(row * n + (t + 4))] = sgn * std::pow(double(t), double(p));
        }
        b[size_t(row)] = 0.0;
    }
    solve(A, b, n);
    return b;
}

// Periodised one-level synthesis operator on m points (m even): maps
// [a (m/2); d (m/2)] to x, x[s] = sum_k a[k] lo[s - 2k] + d[k] hi[s - 2k].
std::vector<double> synthesis_level(int m, const std::vector<double>& dual)
{
    std::vector<double> S(size_t(m * m), 0.0);
    const double r = 1.0 / std::sqrt(2.0);
    auto wrap = [m](int v) { return ((v % m) + m) % m; };
    for (int k = 0; k < m / 2; ++k) {
        S[size_t(wrap(2 * k) * m + k)] += r;       // lo[0]
        S[size_t(wrap(2 * k + 1) * m + k)] += r;   // lo[1]
        for (int t = -4; t <= 5; ++t) {             // hi[t] = (-1)^t lo~[1 - t]
            const int src = 1 - t;                   // lies in [-4, 5]
            const double sgn = (((t % 2) + 2) % 2 == 0) ? 1.0 : -1.0;
            S[size_t(wrap(2 * k + t) * m + (m / 2 + k))] += sgn * dual[size_t(src + 4)];
        }
    }
    return S;
}

std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n)
{
    std::vector<double> C(size_t(n * n), 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double a = A[size_t(i * n + k)];
            if (a == 0.0) continue;
            for (int j = 0; j < n; ++j) C[size_t(i * n + j)] += a * B[size_t(k * n + j)];
        }
    return C;
}

}  // namespace

void spatial_matrices(int kind, int n, std::vector<double>& T, std::vector<double>& U)
{
    T.assign(size_t(n * n), 0.0);
    U.assign(size_t(n * n), 0.0);
    if (kind == BMND_SPATIAL_DCT && n > 1) {
        const double pi = std::acos(-1.0);
        for (int k = 0; k < n; ++k)
            for (int s = 0; s < n; ++s) {
                const double scale = std::sqrt((k == 0 ? 1.0 : 2.0) / n);
                double v = scale * std::cos(pi * k * (2 * s + 1) / (2.0 * n));
                // odd multiples of pi/2 are exact zeros of the DCT-II matrix
                if (std::fabs(v) < 1e-12) v = 0.0;
                T[size_t(k * n + s)] = v;
                U[size_t(s * n + k)] = v;
            }
        return;
    }
    for (int i = 0; i < n; ++i) U[size_t(i * n + i)] = 1.0;
    if (kind == BMND_SPATIAL_BIOR15 && n > 1) {
        const std::vector<double> dual = bior15_dual_lowpass();
        // U = S_1 * blockdiag(S_2, I) * blockdiag(S_3, I) * ...
        int m = n;
        while (m % 2 == 0 && m >= 2) {
            std::vector<double> lvl(size_t(n * n), 0.0);
            for (int i = 0; i < n; ++i) lvl[size_t(i * n + i)] = 1.0;
            const std::vector<double> S = synthesis_level(m, dual);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) lvl[size_t(i * n + j)] = S[size_t(i * m + j)];
            U = matmul(U, lvl, n);
            m /= 2;
        }
    }
    T = inverse(U, n);
    // Both multilevel operators have exact zeros (their nonzero entries are
    // >= 1e-4 in magnitude up to n = 32); the solved dual taps and the
    // inversion leave round-off of order 1e-16 there, which would turn
    // zero-variance coefficients of dark groups into spurious nonzero ones.
    // Restore the exact zeros.
    for (double& v : T)
        if (std::fabs(v) < 1e-12) v = 0.0;
    for (double& v : U)
        if (std::fabs(v) < 1e-12) v = 0.0;
}

// Orthonormal multilevel Haar, rows: scaling, then detail rows with support
// K, K/2, ..., 2 (row l in [2^t, 2^(t+1)) covers members
// [(l - 2^t) K/2^t, (l - 2^t + 1) K/2^t), + on the first half, - on the second).
void haar_matrix(int K, std::vector<double>& H)
{
    H.assign(size_t(K * K), 0.0);
    for (int j = 0; j < K; ++j) H[size_t(j)] = 1.0 / std::sqrt(double(K));
    for (int l = 1; l < K; ++l) {
        int t = 0;
        while ((2 << t) <= l) ++t;
        const int support = K >> t;
        const int first = (l - (1 << t)) * support;
        const double v = 1.0 / std::sqrt(double(support));
        for (int j = 0; j < support; ++j)
            H[size_t(l * K + first + j)] = (j < support / 2) ? v : -v;
    }
}

std::vector<double> kaiser_window(int n, double beta)
{
    std::vector<double> w(size_t(n), 1.0);
    if (n == 1) return w;
    const double den = std::cyl_bessel_i(0.0, beta);
    for (int m = 0; m < n; ++m) {
        const double r = (2.0 * m - (n - 1)) / double(n - 1);
        const double arg = beta * std::sqrt(std::max(0.0, 1.0 - r * r));
        w[size_t(m)] = std::cyl_bessel_i(0.0, arg) / den;
    }
    return w;
}

}  // namespace bmnd
