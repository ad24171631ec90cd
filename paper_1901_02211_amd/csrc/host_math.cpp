// Host-side FP64 scalar set-up: Jacobi elliptic functions, Zolotarev coefficients
// (section 1, Eq. 4), symmetric tridiagonal extreme eigenvalues (Lanczos bounds),
// the SplitMix64 counter generator and the probing colourings (section 2.2).
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace smpq {

// Complete elliptic integral of the first kind K(m), parameter m = k^2, through the
// arithmetic-geometric mean: K = pi / (2 AGM(1, sqrt(1 - m)))  (Abramowitz & Stegun 17.6).
double elliptic_k(double m) {
    double a = 1.0, b = std::sqrt(1.0 - m);
    for (int i = 0; i < 64 && std::fabs(a - b) > 1e-17 * a; ++i) {
        double an = 0.5 * (a + b);
        b = std::sqrt(a * b);
        a = an;
    }
    return M_PI / (2.0 * a);
}

// Jacobi sn, cn, dn of argument u and parameter m by the AGM / descending Landen
// scheme (Abramowitz & Stegun 16.4): run the AGM to a_N, set phi_N = 2^N a_N u,
// recurse phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2, then
// sn = sin phi_0, cn = cos phi_0 and dn = sqrt(1 - m sn^2) (the quotient form
// cos phi_0 / cos(phi_1 - phi_0) is 0/0 at u = K).
void elliptic_j(double u, double m, double *sn, double *cn, double *dn) {
    double a[40], c[40];
    a[0] = 1.0;
    double b = std::sqrt(1.0 - m);
    c[0] = std::sqrt(m);
    int n = 0;
    while (std::fabs(c[n]) > 1e-17 && n < 38) {
        a[n + 1] = 0.5 * (a[n] + b);
        c[n + 1] = 0.5 * (a[n] - b);
        b = std::sqrt(a[n] * b);
        ++n;
    }
    double phi = std::ldexp(1.0, n) * a[n] * u;
    for (int i = n; i > 0; --i) phi = 0.5 * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
    *sn = std::sin(phi);
    *cn = std::cos(phi);
    *dn = std::sqrt(1.0 - m * (*sn) * (*sn));
}

// x R(x^2)/d with R(x^2) = d prod_l (x^2 + a_{2l}) / (x^2 + a_{2l-1});  a[0] = a_1.
static double zolo_unnormalised(double x, const std::vector<double> &a) {
    double x2 = x * x, r = x;
    for (size_t l = 0; l + 1 < a.size(); l += 2) r *= (x2 + a[l + 1]) / (x2 + a[l]);
    return r;
}

// Zolotarev's optimal rational approximation of sign on [k, 1]:
//   a_l = k^2 sn^2(l K'/(2n+1); k') / cn^2(l K'/(2n+1); k'),  l = 1..2n,  k' = sqrt(1 - k^2);
// the error alternates at x_j = k / dn(j K'/(2n+1); k'), j = 0..2n+1, so the symmetric
// normalisation is d = 2/(min + max) of x R(x^2)/d over those points and
// delta = (max - min)/(max + min).  Partial fractions b_0 = d,
//   b_l = d prod_j (a_{2j} - a_{2l-1}) / prod_{j != l} (a_{2j-1} - a_{2l-1}),
// and for |H| in [lam_min, lam_max]: c_0 = b_0/lam_max, c_l = b_l lam_max,
// q_l = a_{2l-1} lam_max^2.
Zolo zolotarev(int n, double lam_min, double lam_max) {
    if (n < 1 || !(lam_min > 0.0) || !(lam_max > lam_min) || !std::isfinite(lam_max))
        throw std::invalid_argument("zolotarev: need n >= 1 and 0 < lam_min < lam_max");
    const double k = lam_min / lam_max;
    const double mp = 1.0 - k * k;            // parameter of modulus k'
    const double Kp = elliptic_k(mp);
    std::vector<double> a(2 * n);
    for (int l = 1; l <= 2 * n; ++l) {
        double sn, cn, dn;
        elliptic_j(l * Kp / (2 * n + 1), mp, &sn, &cn, &dn);
        a[l - 1] = k * k * sn * sn / (cn * cn);
    }
    double fmin = INFINITY, fmax = -INFINITY;
    for (int j = 0; j <= 2 * n + 1; ++j) {
        double sn, cn, dn;
        elliptic_j(j * Kp / (2 * n + 1), mp, &sn, &cn, &dn);
        double f = zolo_unnormalised(k / dn, a);
        fmin = std::min(fmin, f);
        fmax = std::max(fmax, f);
    }
    const double d = 2.0 / (fmin + fmax);
    Zolo z;
    z.n = n;
    z.lam_min = lam_min;
    z.lam_max = lam_max;
    z.delta = (fmax - fmin) / (fmax + fmin);
    z.c0 = d / lam_max;
    std::vector<std::pair<double, double>> qc(n);
    for (int l = 0; l < n; ++l) {
        double den_l = a[2 * l];
        double num = 1.0, den = 1.0;
        for (int j = 0; j < n; ++j) {
            num *= a[2 * j + 1] - den_l;
            if (j != l) den *= a[2 * j] - den_l;
        }
        qc[l] = {den_l * lam_max * lam_max, d * num / den * lam_max};
    }
    std::sort(qc.begin(), qc.end());
    for (auto &p : qc) {
        z.q.push_back(p.first);
        z.c.push_back(p.second);
        if (!(p.first > 0.0) || !(p.second > 0.0) || !std::isfinite(p.second))
            throw std::runtime_error("zolotarev: non-positive or non-finite coefficient");
    }
    if (!(z.delta >= 0.0 && z.delta < 1.0) || !(z.c0 > 0.0))
        throw std::runtime_error("zolotarev: normalisation failed");
    return z;
}

// Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x, from the
// signs of the pivots of T - x = L D L^T (Sturm sequence count).
static int sturm_count(const std::vector<double> &al, const std::vector<double> &be, double x) {
    int cnt = 0;
    double d = 1.0;
    for (size_t i = 0; i < al.size(); ++i) {
        double b2 = (i == 0) ? 0.0 : be[i - 1] * be[i - 1];
        d = al[i] - x - (i == 0 ? 0.0 : b2 / d);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

// Smallest and largest eigenvalue of a symmetric tridiagonal matrix by bisection on the
// Sturm count, starting from the Gershgorin interval.
void tridiag_extremes(const std::vector<double> &alpha, const std::vector<double> &beta,
                      double *lo, double *hi) {
    const size_t n = alpha.size();
    double gl = INFINITY, gh = -INFINITY;
    for (size_t i = 0; i < n; ++i) {
        double r = (i > 0 ? std::fabs(beta[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(beta[i]) : 0.0);
        gl = std::min(gl, alpha[i] - r);
        gh = std::max(gh, alpha[i] + r);
    }
    auto bisect = [&](int k) {   // k-th smallest eigenvalue, k = 0..n-1
        double a = gl, b = gh;
        for (int it = 0; it < 200 && b - a > 1e-16 * std::max(std::fabs(a), std::fabs(b)); ++it) {
            double m = 0.5 * (a + b);
            if (sturm_count(alpha, beta, m) > k) b = m; else a = m;
        }
        return 0.5 * (a + b);
    };
    *lo = bisect(0);
    *hi = bisect(static_cast<int>(n) - 1);
}

// All eigenpairs of the symmetric tridiagonal matrix with diagonal d (n) and off-diagonal e
// (n - 1) by the implicit QL iteration with Wilkinson shifts (Bowdler, Martin, Reinsch and
// Wilkinson, Numer. Math. 11 (1968)): plane rotations chase the bulge from the bottom of the
// unreduced block to its top, and their product, accumulated in z, gives the eigenvectors.
// On return evals is ascending and column j of z (n x n, column-major) is its eigenvector.
void tridiag_eigen(std::vector<double> d, std::vector<double> e, std::vector<double> &evals,
                   std::vector<double> &z) {
    const int n = static_cast<int>(d.size());
    e.resize(n, 0.0);
    z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {   // first negligible off-diagonal entry at or below l
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd) break;
            }
            if (m == l) break;
            if (iter == 100) throw std::runtime_error("tridiag_eigen: no convergence");
            // Wilkinson shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            for (; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {   // the rotation split the block: deflate and restart
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
                for (int k = 0; k < n; ++k) {   // rotate columns i and i+1 of z
                    const double zi = z[(size_t)i * n + k], zi1 = z[(size_t)(i + 1) * n + k];
                    z[(size_t)(i + 1) * n + k] = s * zi + c * zi1;
                    z[(size_t)i * n + k] = c * zi - s * zi1;
                }
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // ascending order
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
    evals.resize(n);
    std::vector<double> zs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        evals[j] = d[order[j]];
        std::copy(z.begin() + (size_t)order[j] * n, z.begin() + (size_t)(order[j] + 1) * n, zs.begin() + (size_t)j * n);
    }
    z.swap(zs);
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based stream: word i of stream
// `seed` is mix(seed + (i + 1) * 0x9e3779b97f4a7c15), mapped to [0, 1) by its top 53 bits.
double splitmix64_uniform(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return static_cast<double>(z >> 11) * 0x1.0p-53;
}

// Probing colourings (section 2.2).  Returns the class count; colour has V entries.
int make_colouring(const int dims[4], const int r[4], int mode, std::vector<int32_t> &colour,
                   std::string &err) {
    for (int mu = 0; mu < 4; ++mu) {
        if (r[mu] < 1 || dims[mu] % r[mu] != 0) {
            err = "gap r does not divide the lattice extent (Eq. 19)";
            return -1;
        }
    }
    if (mode == 1) {
        for (int mu = 0; mu < 4; ++mu)
            if ((dims[mu] / r[mu]) % 2 != 0) {
                err = "split mode needs an even number of class sites in every direction";
                return -1;
            }
    } else if (mode == 2) {
        for (int mu = 0; mu < 4; ++mu)
            if (r[mu] % 2 != 0) {
                err = "combine mode needs an even gap in all four directions";
                return -1;
            }
    } else if (mode != 0) {
        err = "mode must be 0 (normal), 1 (split) or 2 (combine)";
        return -1;
    }
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    colour.resize(V);
    const int nbase = r[0] * r[1] * r[2] * r[3];
    for (int64_t s = 0; s < V; ++s) {
        int64_t t = s;
        int x[4];
        for (int mu = 0; mu < 4; ++mu) {
            x[mu] = static_cast<int>(t % dims[mu]);
            t /= dims[mu];
        }
        int y[4];
        for (int mu = 0; mu < 4; ++mu) y[mu] = x[mu] % r[mu];
        if (mode == 2 && y[3] >= r[3] / 2)
            for (int mu = 0; mu < 4; ++mu) y[mu] = (y[mu] + r[mu] / 2) % r[mu];
        int lex = y[0] + r[0] * (y[1] + r[1] * (y[2] + r[2] * y[3]));
        if (mode == 1) {
            int par = (x[0] / r[0] + x[1] / r[1] + x[2] / r[2] + x[3] / r[3]) & 1;
            lex = 2 * lex + par;
        }
        colour[s] = lex;
    }
    return mode == 0 ? nbase : (mode == 1 ? 2 * nbase : nbase / 2);
}

}  // namespace smpq
