// Host-side FP64 scalar set-up shared by the C ABI: elliptic functions, Zolotarev
// coefficients, tridiagonal bisection, SplitMix64 and the probing colourings.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace smpq {

struct Zolo {
    int n = 0;
    double lam_min = 0, lam_max = 0, delta = 0, c0 = 0;
    std::vector<double> c, q;   // q ascending
};

double elliptic_k(double m);
void elliptic_j(double u, double m, double *sn, double *cn, double *dn);
Zolo zolotarev(int n, double lam_min, double lam_max);
void tridiag_extremes(const std::vector<double> &alpha, const std::vector<double> &beta,
                      double *lo, double *hi);
double splitmix64_uniform(uint64_t seed, uint64_t i);
// Eigenvalues (ascending) and eigenvectors (column-major n x n) of a symmetric tridiagonal
// matrix (diagonal d, off-diagonal e) by implicit QL.
void tridiag_eigen(std::vector<double> d, std::vector<double> e, std::vector<double> &evals,
                   std::vector<double> &z);
int make_colouring(const int dims[4], const int r[4], int mode, std::vector<int32_t> &colour,
                   std::string &err);

}  // namespace smpq
