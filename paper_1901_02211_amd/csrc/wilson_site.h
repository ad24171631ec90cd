// Per-site Wilson hopping term, written once for the GPU kernels and for host checks.
//
// hop(x) = sum_mu [ P(-s)_mu U_mu(x) psi(x + mu) + P(+s)_mu U_mu(x - mu)^dag psi(x - mu) ],
// with P(s)_mu = 1 - s gamma_mu, s = +1 for D_W and s = -1 for D_W^dag (the adjoint swaps
// the two projectors), so that D_W psi = psi - kappa hop (section 1, Eq. 3).
//
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_x = -i sigma_1,
// A_y = -i sigma_2, A_z = -i sigma_3, A_t = 1.  (1 - s gamma_mu) psi has upper half
// h = psi_up - s A_mu psi_dn and lower half -s A_mu^dag h, so each hop projects to a
// two-spinor, multiplies it by the link and rebuilds the lower half.
#pragma once
#include <hip/hip_runtime.h>

namespace smpq {

template <class T>
struct cpx {
    T re, im;
};

template <class T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
// i * a
template <class T>
__host__ __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.im, a.re}; }
// a * b
template <class T>
__host__ __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <class T>
__host__ __device__ __forceinline__ cpx<T> cjmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a * b + c with a single rounding
__host__ __device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// c + a * b and c + conj(a) * b as chains of fused multiply-adds: sums of complex products
// written this way take 4 instructions per term instead of 6 (the compiler does not
// reassociate a sum of products into such a chain by itself)
template <class T>
__host__ __device__ __forceinline__ cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> c) {
    return {fmadd(a.re, b.re, fmadd(-a.im, b.im, c.re)), fmadd(a.re, b.im, fmadd(a.im, b.re, c.im))};
}
template <class T>
__host__ __device__ __forceinline__ cpx<T> cjfma(cpx<T> a, cpx<T> b, cpx<T> c) {
    return {fmadd(a.re, b.re, fmadd(a.im, b.im, c.re)), fmadd(a.re, b.im, fmadd(-a.im, b.re, c.im))};
}

// Upper two spin rows of (1 - S gamma_MU) psi; psi[spin*3 + colour], h[spin*3 + colour].
template <int MU, int S, class T>
__host__ __device__ __forceinline__ void project(const cpx<T> p[12], cpx<T> h[6]) {
    constexpr T s = static_cast<T>(S);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<T> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
        if constexpr (MU == 0) {        // A = -i sigma_1:  A psi_dn = (-i p3, -i p2)
            h[a] = p0 + s * mul_i(p3);
            h[3 + a] = p1 + s * mul_i(p2);
        } else if constexpr (MU == 1) { // A = -i sigma_2 = [[0,-1],[1,0]]: A psi_dn = (-p3, p2)
            h[a] = p0 + s * p3;
            h[3 + a] = p1 - s * p2;
        } else if constexpr (MU == 2) { // A = -i sigma_3 = diag(-i, i): A psi_dn = (-i p2, i p3)
            h[a] = p0 + s * mul_i(p2);
            h[3 + a] = p1 - s * mul_i(p3);
        } else {                        // A = 1
            h[a] = p0 - s * p2;
            h[3 + a] = p1 - s * p3;
        }
    }
}

// acc += (1 - S gamma_MU) spinor whose upper half is g (lower half = -S A^dag g).
template <int MU, int S, class T>
__host__ __device__ __forceinline__ void accumulate(cpx<T> acc[12], const cpx<T> g[6]) {
    constexpr T s = static_cast<T>(S);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<T> g0 = g[a], g1 = g[3 + a];
        acc[a] = acc[a] + g0;
        acc[3 + a] = acc[3 + a] + g1;
        if constexpr (MU == 0) {        // A^dag = i sigma_1: A^dag g = (i g1, i g0)
            acc[6 + a] = acc[6 + a] - s * mul_i(g1);
            acc[9 + a] = acc[9 + a] - s * mul_i(g0);
        } else if constexpr (MU == 1) { // A^dag = [[0,1],[-1,0]]: A^dag g = (g1, -g0)
            acc[6 + a] = acc[6 + a] - s * g1;
            acc[9 + a] = acc[9 + a] + s * g0;
        } else if constexpr (MU == 2) { // A^dag = diag(i, -i): A^dag g = (i g0, -i g1)
            acc[6 + a] = acc[6 + a] - s * mul_i(g0);
            acc[9 + a] = acc[9 + a] + s * mul_i(g1);
        } else {
            acc[6 + a] = acc[6 + a] - s * g0;
            acc[9 + a] = acc[9 + a] - s * g1;
        }
    }
}

// g = U h for both spin rows (U row-major u[row*3 + col]).
template <class T>
__host__ __device__ __forceinline__ void su3_mul(const cpx<T> u[9], const cpx<T> h[6], cpx<T> g[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            g[3 * sp + a] = cfma(u[3 * a + 2], h[3 * sp + 2], cfma(u[3 * a + 1], h[3 * sp + 1], cmul(u[3 * a], h[3 * sp])));
}

// g = U^dag h.
template <class T>
__host__ __device__ __forceinline__ void su3_dag_mul(const cpx<T> u[9], const cpx<T> h[6], cpx<T> g[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            g[3 * sp + a] = cjfma(u[6 + a], h[3 * sp + 2], cjfma(u[3 + a], h[3 * sp + 1], cjmul(u[a], h[3 * sp])));
}

// Neighbour indices of site s on the periodic lattice (x fastest).
struct Nbr {
    int fwd[4], bwd[4];
};

__host__ __device__ __forceinline__ Nbr neighbours(int s, int nx, int ny, int nz, int nt) {
    Nbr n;
    const int sxy = nx * ny, sxyz = sxy * nz;
    const int x = s % nx, y = (s / nx) % ny, z = (s / sxy) % nz, t = s / sxyz;
    n.fwd[0] = (x == nx - 1) ? s - (nx - 1) : s + 1;
    n.bwd[0] = (x == 0) ? s + (nx - 1) : s - 1;
    n.fwd[1] = (y == ny - 1) ? s - (ny - 1) * nx : s + nx;
    n.bwd[1] = (y == 0) ? s + (ny - 1) * nx : s - nx;
    n.fwd[2] = (z == nz - 1) ? s - (nz - 1) * sxy : s + sxy;
    n.bwd[2] = (z == 0) ? s + (nz - 1) * sxy : s - sxy;
    n.fwd[3] = (t == nt - 1) ? s - (nt - 1) * sxyz : s + sxyz;
    n.bwd[3] = (t == 0) ? s + (nt - 1) * sxyz : s - sxyz;
    return n;
}

}  // namespace smpq
