// quadrature.cpp -- collocation rules of the stochastic collocation step
// (arXiv 2508.18202, Sec. 2.3, Eq. coef_discrete and Eq. quad_moments: nodes
// Z^(j) and weights a_j) for inputs xi ~ U(-1, 1)^d or z ~ N(0, 1)^d,
// probability weights, and the Hermite chaos basis of the gPC expansion.
//
//   Gauss-Hermite   Golub-Welsch on the orthonormal probabilists' Hermite
//                   recurrence (off-diagonal sqrt(k)), tensor product over
//                   the dimensions (the paper's dense tensor-product rule).
//
//   Gauss-Legendre  Golub-Welsch: the nodes are the eigenvalues of the Jacobi
//                   matrix of the Legendre recurrence (off-diagonal
//                   k / sqrt(4k^2 - 1)), the weights the squared first
//                   components of its normalised eigenvectors.
//   Smolyak CC      nested Clenshaw-Curtis rules (1, 3, 5, 9, ... points,
//                   Chebyshev extrema) combined by the combination technique
//                   sum_{L-d+1 <= |l| <= L} (-1)^(L-|l|) C(d-1, L-|l|) Q_l1 x ... x Q_ld;
//                   each 1-D rule's weights solve the Chebyshev moment
//                   equations sum_j w_j T_k(x_j) = E[T_k(xi)].
#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "quadrature.h"

namespace lbmsc {

// Symmetric tridiagonal eigenproblem by implicit QL with Wilkinson shifts;
// d: diagonal (eigenvalues out), e: sub-diagonal (e[0..n-2]), z: first row of
// the eigenvector matrix (starts as e_1).
static bool tql_first_row(std::vector<double> &d, std::vector<double> e, std::vector<double> &z)
{
    const int n = (int)d.size();
    e.push_back(0.0);
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-300 + 1e-17 * dd) break;
            }
            if (m == l) break;
            if (++iter > 200) return false;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            for (; i >= l; --i) {
                double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                f = z[i + 1];
                z[i + 1] = s * z[i] + c * f;
                z[i] = c * z[i] - s * f;
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

bool gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    if (n < 1) return false;
    std::vector<double> d(n, 0.0), e(n > 1 ? n - 1 : 0), z(n, 0.0);
    for (int k = 1; k < n; ++k) e[k - 1] = k / std::sqrt(4.0 * k * k - 1.0);
    z[0] = 1.0;
    if (!tql_first_row(d, e, z)) return false;
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        x[i] = d[idx[i]];
        w[i] = z[idx[i]] * z[idx[i]];  // mu_0 = 1 for the probability measure
    }
    // exact symmetry of the rule
    for (int i = 0; i < n / 2; ++i) {
        const double a = 0.5 * (x[n - 1 - i] - x[i]);
        x[i] = -a;
        x[n - 1 - i] = a;
        const double b = 0.5 * (w[i] + w[n - 1 - i]);
        w[i] = w[n - 1 - i] = b;
    }
    if (n & 1) x[n / 2] = 0.0;
    return true;
}

// Golub-Welsch for the standard normal: the orthonormal probabilists'
// Hermite recurrence has zero diagonal and off-diagonal sqrt(k).
bool gauss_hermite(int n, std::vector<double> &x, std::vector<double> &w)
{
    if (n < 1) return false;
    std::vector<double> d(n, 0.0), e(n > 1 ? n - 1 : 0), z(n, 0.0);
    for (int k = 1; k < n; ++k) e[k - 1] = std::sqrt((double)k);
    z[0] = 1.0;
    if (!tql_first_row(d, e, z)) return false;
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        x[i] = d[idx[i]];
        w[i] = z[idx[i]] * z[idx[i]];
    }
    for (int i = 0; i < n / 2; ++i) {
        const double a = 0.5 * (x[n - 1 - i] - x[i]);
        x[i] = -a;
        x[n - 1 - i] = a;
        const double b = 0.5 * (w[i] + w[n - 1 - i]);
        w[i] = w[n - 1 - i] = b;
    }
    if (n & 1) x[n / 2] = 0.0;
    double s = 0.0;
    for (double v : w) s += v;
    for (double &v : w) v /= s;
    return true;
}

bool tensor_gauss_hermite(int n, int dim, std::vector<double> &nodes, std::vector<double> &weights)
{
    if (dim < 1 || dim > 8) return false;
    std::vector<double> x, w;
    if (!gauss_hermite(n, x, w)) return false;
    long total = 1;
    for (int k = 0; k < dim; ++k) {
        total *= n;
        if (total > 65536) return false;
    }
    nodes.assign((size_t)total * dim, 0.0);
    weights.assign((size_t)total, 1.0);
    for (long j = 0; j < total; ++j) {
        long r = j;
        for (int k = dim - 1; k >= 0; --k) {
            const int i = (int)(r % n);
            r /= n;
            nodes[(size_t)j * dim + k] = x[i];
            weights[(size_t)j] *= w[i];
        }
    }
    return true;
}

static void multi_rec(int dim, int k, int left, std::vector<int> &cur, std::vector<int> &out)
{
    if (k == dim - 1) {
        cur[k] = left;
        out.insert(out.end(), cur.begin(), cur.end());
        return;
    }
    for (int a = left; a >= 0; --a) {
        cur[k] = a;
        multi_rec(dim, k + 1, left - a, cur, out);
    }
}

void gpc_multi_indices(int dim, int order, std::vector<int> &alpha)
{
    alpha.clear();
    std::vector<int> cur(dim, 0);
    for (int deg = 0; deg <= order; ++deg) multi_rec(dim, 0, deg, cur, alpha);
}

void gpc_basis(const double *nodes, int n_nodes, int dim, const std::vector<int> &alpha, std::vector<double> &phi)
{
    const int P = (int)alpha.size() / dim;
    int maxdeg = 0;
    for (int a : alpha) maxdeg = std::max(maxdeg, a);
    phi.assign((size_t)n_nodes * P, 1.0);
    std::vector<double> he(maxdeg + 1);
    std::vector<double> fact(maxdeg + 1, 1.0);
    for (int k = 1; k <= maxdeg; ++k) fact[k] = fact[k - 1] * k;
    for (int j = 0; j < n_nodes; ++j)
        for (int k = 0; k < dim; ++k) {
            const double z = nodes[(size_t)j * dim + k];
            he[0] = 1.0;
            if (maxdeg >= 1) he[1] = z;
            for (int m = 1; m < maxdeg; ++m) he[m + 1] = z * he[m] - m * he[m - 1];
            for (int p = 0; p < P; ++p) {
                const int a = alpha[(size_t)p * dim + k];
                phi[(size_t)j * P + p] *= he[a] / std::sqrt(fact[a]);
            }
        }
}

static bool solve(std::vector<double> A, std::vector<double> b, int n, std::vector<double> &y)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[p * n + k], A[c * n + k]);
            std::swap(b[p], b[c]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    y.assign(n, 0.0);
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * y[k];
        y[r] = s / A[r * n + r];
    }
    return true;
}

bool clenshaw_curtis(int m, std::vector<double> &x, std::vector<double> &w)
{
    if (m < 1) return false;
    if (m == 1) {
        x.assign(1, 0.0);
        w.assign(1, 1.0);
        return true;
    }
    const int n = m - 1;
    x.resize(m);
    for (int j = 0; j < m; ++j) x[j] = (2 * j == n) ? 0.0 : std::cos(M_PI * (double)(n - j) / n);
    // rows k = 0..m-1: sum_j w_j T_k(x_j) = E[T_k] = 1/(1-k^2) for even k, 0 for odd k
    std::vector<double> A((size_t)m * m), b(m);
    for (int k = 0; k < m; ++k) {
        for (int j = 0; j < m; ++j) A[(size_t)k * m + j] = std::cos(k * std::acos(std::max(-1.0, std::min(1.0, x[j]))));
        b[k] = (k % 2) ? 0.0 : 1.0 / (1.0 - (double)k * k);
    }
    return solve(A, b, m, w);
}

bool smolyak_cc(int level, int dim, std::vector<double> &nodes, std::vector<double> &weights)
{
    if (level < 0 || dim < 1 || level > 12 || dim > 8) return false;
    std::vector<std::vector<double>> rx(level + 1), rw(level + 1);
    for (int l = 0; l <= level; ++l) {
        const int m = l == 0 ? 1 : (1 << l) + 1;
        if (!clenshaw_curtis(m, rx[l], rw[l])) return false;
    }
    std::map<std::vector<long long>, std::pair<std::vector<double>, double>> acc;
    std::vector<int> l(dim, 0);
    for (;;) {
        int s = 0;
        for (int v : l) s += v;
        if (s <= level && s >= level - dim + 1) {
            const int k = level - s;
            double binom = 1.0;
            for (int t = 0; t < k; ++t) binom = binom * (dim - 1 - t) / (t + 1);
            const double coef = ((k & 1) ? -1.0 : 1.0) * binom;
            std::vector<int> j(dim, 0);
            for (;;) {
                std::vector<double> p(dim);
                std::vector<long long> key(dim);
                double wt = coef;
                for (int a = 0; a < dim; ++a) {
                    p[a] = rx[l[a]][j[a]];
                    wt *= rw[l[a]][j[a]];
                    key[a] = std::llround(p[a] * 1e12);
                }
                auto it = acc.find(key);
                if (it == acc.end()) acc.emplace(key, std::make_pair(p, wt));
                else it->second.second += wt;
                int a = 0;
                for (; a < dim; ++a) {
                    if (++j[a] < (int)rx[l[a]].size()) break;
                    j[a] = 0;
                }
                if (a == dim) break;
            }
        }
        int a = 0;
        for (; a < dim; ++a) {
            if (++l[a] <= level) break;
            l[a] = 0;
        }
        if (a == dim) break;
    }
    nodes.clear();
    weights.clear();
    for (auto &kv : acc) {
        if (std::fabs(kv.second.second) < 1e-15) continue;  // cancelled node
        for (double v : kv.second.first) nodes.push_back(v);
        weights.push_back(kv.second.second);
    }
    return true;
}

}  // namespace lbmsc
