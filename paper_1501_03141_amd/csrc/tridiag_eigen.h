// Eigen-decomposition of a real symmetric tridiagonal matrix by the implicit QL method
// with Wilkinson-type shifts and accumulated rotations (Bowdler, Martin, Reinsch and
// Wilkinson, "The QR and QL algorithms for symmetric matrices", Numer. Math. 11 (1968),
// published as procedure tql2).  Host code; O(n^2) per sweep plus the rotations of the
// eigenvector matrix.
#pragma once

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

namespace pdep {

// d: the n diagonal entries (in: T_ii, out: eigenvalues ascending); e: the n - 1
// off-diagonal entries T_i,i+1; Z: n x n row-major, out: Z[i * n + k] = component i of
// eigenvector k.  Returns false if an eigenvalue needed more than 60 iterations.
inline bool tridiag_eigen(int n, std::vector<double>& d, std::vector<double> e, std::vector<double>& Z) {
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    if (n <= 1) return true;
    e.resize(n);
    e[n - 1] = 0.0;
    const double eps = std::numeric_limits<double>::epsilon();
    double f = 0.0, tst1 = 0.0;
    bool ok = true;
    for (int l = 0; l < n; ++l) {
        // find a negligible off-diagonal entry at or below l
        tst1 = std::max(tst1, std::abs(d[l]) + std::abs(e[l]));
        int m = l;
        while (m < n - 1 && std::abs(e[m]) > eps * tst1) ++m;
        if (m > l) {
            int iter = 0;
            do {
                if (++iter > 60) {
                    ok = false;
                    break;
                }
                // shift from the leading 2 x 2 block
                double g = d[l];
                double p = (d[l + 1] - g) / (2.0 * e[l]);
                double r = std::hypot(p, 1.0);
                if (p < 0) r = -r;
                d[l] = e[l] / (p + r);
                d[l + 1] = e[l] * (p + r);
                const double dl1 = d[l + 1];
                double h = g - d[l];
                for (int i = l + 2; i < n; ++i) d[i] -= h;
                f += h;
                // implicit QL sweep from m up to l
                p = d[m];
                double c = 1.0, c2 = 1.0, c3 = 1.0, s = 0.0, s2 = 0.0;
                const double el1 = e[l + 1];
                for (int i = m - 1; i >= l; --i) {
                    c3 = c2;
                    c2 = c;
                    s2 = s;
                    g = c * e[i];
                    h = c * p;
                    r = std::hypot(p, e[i]);
                    e[i + 1] = s * r;
                    s = e[i] / r;
                    c = p / r;
                    p = c * d[i] - s * g;
                    d[i + 1] = h + s * (c * g + s * d[i]);
                    for (int k = 0; k < n; ++k) {
                        const double zk1 = Z[(size_t)k * n + i + 1], zk = Z[(size_t)k * n + i];
                        Z[(size_t)k * n + i + 1] = s * zk + c * zk1;
                        Z[(size_t)k * n + i] = c * zk - s * zk1;
                    }
                }
                p = -s * s2 * c3 * el1 * e[l] / dl1;
                e[l] = s * p;
                d[l] = c * p;
            } while (std::abs(e[l]) > eps * tst1);
        }
        d[l] += f;
        e[l] = 0.0;
    }
    // ascending order, columns of Z with them
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] < d[b]; });
    std::vector<double> d2(n), Z2((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        d2[k] = d[ord[k]];
        for (int i = 0; i < n; ++i) Z2[(size_t)i * n + k] = Z[(size_t)i * n + ord[k]];
    }
    d.swap(d2);
    Z.swap(Z2);
    return ok;
}

}  // namespace pdep
