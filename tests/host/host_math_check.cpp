// Host-side checks of paper_1901_02211_amd/csrc/host_math.cpp, built with address and
// undefined-behaviour sanitizers by tests/test_host_sanitized.py.  Exit status 0 = all pass.
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1901_02211_amd/csrc/host_math.h"

static int failures = 0;
#define CHECK(cond, ...)                       \
    do {                                       \
        if (!(cond)) {                         \
            std::printf("FAIL %s: ", #cond);   \
            std::printf(__VA_ARGS__);          \
            std::printf("\n");                 \
            ++failures;                        \
        }                                      \
    } while (0)

int main() {
    using namespace smpq;
    // Jacobi elliptic identities sn^2 + cn^2 = 1, dn^2 + m sn^2 = 1; K(0) = pi/2
    for (double m : {0.0, 0.3, 0.9, 0.9999}) {
        for (double u : {0.0, 0.4, 1.3, 2.0}) {
            double sn, cn, dn;
            elliptic_j(u, m, &sn, &cn, &dn);
            CHECK(std::fabs(sn * sn + cn * cn - 1.0) < 1e-14, "m=%g u=%g", m, u);
            CHECK(std::fabs(dn * dn + m * sn * sn - 1.0) < 1e-14, "m=%g u=%g", m, u);
        }
    }
    CHECK(std::fabs(elliptic_k(0.0) - M_PI / 2) < 1e-15, "K(0)");
    // Zolotarev: positive coefficients, ascending shifts, small error for 14 poles
    for (double lo : {0.05, 0.15, 0.5}) {
        Zolo z = zolotarev(14, lo, 2.7);
        CHECK(z.delta > 0.0 && z.delta < 1e-9, "delta %g at lo=%g", z.delta, lo);
        CHECK(z.c0 > 0.0, "c0");
        for (int i = 0; i < 14; ++i) {
            CHECK(z.c[i] > 0.0 && z.q[i] > 0.0, "coefficient %d", i);
            if (i) CHECK(z.q[i] > z.q[i - 1], "ascending %d", i);
        }
    }
    bool threw = false;
    try {
        zolotarev(14, 2.0, 1.0);
    } catch (const std::exception &) {
        threw = true;
    }
    CHECK(threw, "lam_min > lam_max must throw");
    // implicit-QL tridiagonal eigensolver: residuals, orthonormality, order, split blocks
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    for (int n : {1, 2, 3, 17, 200}) {
        std::vector<double> d(n), e(n > 1 ? n - 1 : 0), ev, z;
        for (double &x : d) x = U(rng);
        for (size_t i = 0; i < e.size(); ++i) e[i] = (i % 9 == 4) ? 0.0 : U(rng);
        tridiag_eigen(d, e, ev, z);
        double res = 0.0, orth = 0.0;
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < n; ++i) {
                double t = d[i] * z[(size_t)j * n + i];
                if (i > 0) t += e[i - 1] * z[(size_t)j * n + i - 1];
                if (i < n - 1) t += e[i] * z[(size_t)j * n + i + 1];
                res = std::fmax(res, std::fabs(t - ev[j] * z[(size_t)j * n + i]));
            }
            for (int k = 0; k < n; ++k) {
                double sdot = 0.0;
                for (int i = 0; i < n; ++i) sdot += z[(size_t)j * n + i] * z[(size_t)k * n + i];
                orth = std::fmax(orth, std::fabs(sdot - (j == k ? 1.0 : 0.0)));
            }
            if (j) CHECK(ev[j] >= ev[j - 1], "order n=%d", n);
        }
        CHECK(res < 1e-13 && orth < 1e-13, "n=%d residual %g orthogonality %g", n, res, orth);
        // the extremes agree with the Sturm-bisection routine
        double lo, hi;
        tridiag_extremes(d, e, &lo, &hi);
        CHECK(std::fabs(lo - ev[0]) < 1e-12 && std::fabs(hi - ev[n - 1]) < 1e-12, "extremes n=%d", n);
    }
    // SplitMix64: first output of stream 0 is 0xe220a8397b1dcdaf (Steele, Lea, Flood 2014)
    CHECK(splitmix64_uniform(0, 0) == (double)(0xe220a8397b1dcdafull >> 11) * 0x1.0p-53, "splitmix64");
    // colourings: class counts of the three modes and the rejections
    const int dims[4] = {8, 8, 8, 8};
    std::vector<int32_t> col;
    std::string err;
    const int r2[4] = {2, 2, 2, 2}, r4[4] = {4, 4, 4, 4}, r3[4] = {3, 3, 3, 3};
    CHECK(make_colouring(dims, r2, 0, col, err) == 16 && col.size() == 4096u, "mode 0");
    CHECK(make_colouring(dims, r2, 1, col, err) == 32, "mode 1");
    CHECK(make_colouring(dims, r4, 2, col, err) == 128, "mode 2");
    CHECK(make_colouring(dims, r3, 0, col, err) == -1, "3 does not divide 8");
    const int r8[4] = {8, 8, 8, 8};
    CHECK(make_colouring(dims, r8, 1, col, err) == -1, "mode 1 with odd m");
    std::printf("%d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
