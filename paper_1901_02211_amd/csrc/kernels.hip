// Device kernels of the overlap charge-density path on gfx950 (CDNA4, wave64).
//
//  k_dslash        Wilson stencil D_W / D_W^dag (section 1, Eq. 3) in FP64: R right-hand
//                  sides interleaved over the lanes of a block share each link fetch
//  k_dslash_f32    the FP32 stencil: one site per thread, its eight links held in registers
//                  for several right-hand sides (k_dslash_f32_plane: the same with one
//                  16x16 xy-plane per block staged in LDS, _xyl also its x and y links;
//                  k_dslash_f32_tile: xy-tiles of any width <= 64 with halo rows); all take an
//                  optional epilogue "+ sigma aux" with a fused <aux, out> partial for
//                  H^2 + sigma (Eq. 4).
//  k_cg_init ...   multi-shift CG for (D_W^dag D_W + q_i) x_i = b (Eqs. 6-8): the stencil
//                  epilogues sum <p, A p> = |D_W p|^2 + s0 |p|^2 in the first stencil and
//                  update the residual in place in the second; fused update of every active
//                  shift's search direction plus the
//                  running rational sum y = c_0 b + sum_i c_i x_i, scalar recurrences on the
//                  device (one wave per right-hand side), FP64 residual replacement.
//  k_contract      q(x) += 1/2 [gamma5 D_ov phi](x, alpha, a) on the probed sites (Eq. 16), or
//                  the probing estimate of tr D_W^-1 (x, x) from the unshifted solve.
//  k_multi_dot ... low-mode deflation: many dot products and linear combinations at once
//                  (Lanczos reorthogonalisation, Ritz vectors), deflated sources and terms.
//  k_block_mean_abs  locality of D_ov (Eq. 12): mean |D_ov(x, . ; y, .)| per site.
//
// Vectors that a kernel touches once (search directions, residuals, running sums, stencil
// outputs) use non-temporal loads and stores; stencil inputs and links stay cached, since
// neighbouring sites and right-hand-side groups reuse them through L2.
// Reductions are two-pass and fixed-order (per-block partials, then one wave per
// right-hand side), so every FP64 result is bitwise reproducible from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <type_traits>

#include "kernels.h"
#include "wilson_site.h"

namespace smpq {

// ------------------------------------------------------------------ storage traits
template <class T>
struct Store;

template <>
struct Store<double> {
    using vec = double2;
    using link = double2;
    static constexpr int units = 12;
    __device__ static __forceinline__ void load(const double2 *p, size_t vs, int s, cpx<double> v[12]) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 t = p[c * vs + s];
            v[c] = {t.x, t.y};
        }
    }
    __device__ static __forceinline__ void store(double2 *p, size_t vs, int s, const cpx<double> v[12]) {
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c * vs + s] = make_double2(v[c].re, v[c].im);
    }
    // a vector read once by the kernel (non-temporal)
    __device__ static __forceinline__ void load_stream(const double2 *p, size_t vs, int s, cpx<double> v[12]) {
        typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p + c * vs + s));
            v[c] = {t.x, t.y};
        }
    }
    // the stencil's output: written once, read by the next kernel (non-temporal)
    __device__ static __forceinline__ void store_stream(double2 *p, size_t vs, int s, const cpx<double> v[12]) {
        typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const d2 t = {v[c].re, v[c].im};
            __builtin_nontemporal_store(t, reinterpret_cast<d2 *>(p + c * vs + s));
        }
    }
};

template <>
struct Store<float> {
    using vec = float4;
    using link = float4;   // two rows of the SU(3) link: (u00,u01), (u02,u10), (u11,u12)
    static constexpr int units = 6;
    __device__ static __forceinline__ void load(const float4 *p, size_t vs, int s, cpx<float> v[12]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float4 t = p[k * vs + s];
            v[2 * k] = {t.x, t.y};
            v[2 * k + 1] = {t.z, t.w};
        }
    }
    __device__ static __forceinline__ void store(float4 *p, size_t vs, int s, const cpx<float> v[12]) {
#pragma unroll
        for (int k = 0; k < 6; ++k)
            p[k * vs + s] = make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im);
    }
    // a vector read once by the kernel (non-temporal)
    __device__ static __forceinline__ void load_stream(const float4 *p, size_t vs, int s, cpx<float> v[12]) {
        typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p + k * vs + s));
            v[2 * k] = {t.x, t.y};
            v[2 * k + 1] = {t.z, t.w};
        }
    }
    // the stencil's output: written once, read by the next kernel (non-temporal)
    __device__ static __forceinline__ void store_stream(float4 *p, size_t vs, int s, const cpx<float> v[12]) {
        typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const f4 t = {v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
            __builtin_nontemporal_store(t, reinterpret_cast<f4 *>(p + k * vs + s));
        }
    }
};

// FP64 links: all nine entries, [mu][row*3 + col][site] double2.
// FP32 links: the first two rows, [mu][3][site] float4; the third row is rebuilt as
// conj(row0 x row1), exact for a special unitary matrix.
__device__ __forceinline__ void unpack_rows(float4 a, float4 b, float4 c, cpx<float> u[9]) {
    u[0] = {a.x, a.y};
    u[1] = {a.z, a.w};
    u[2] = {b.x, b.y};
    u[3] = {b.z, b.w};
    u[4] = {c.x, c.y};
    u[5] = {c.z, c.w};
    const cpx<float> r0 = cfma(u[1], u[5], -1.0f * cmul(u[2], u[4]));
    const cpx<float> r1 = cfma(u[2], u[3], -1.0f * cmul(u[0], u[5]));
    const cpx<float> r2 = cfma(u[0], u[4], -1.0f * cmul(u[1], u[3]));
    u[6] = {r0.re, -r0.im};
    u[7] = {r1.re, -r1.im};
    u[8] = {r2.re, -r2.im};
}

template <class T>
__device__ __forceinline__ void load_link(const typename Store<T>::link *U, int V, int mu, int s, cpx<T> u[9]);

template <>
__device__ __forceinline__ void load_link<double>(const double2 *U, int V, int mu, int s, cpx<double> u[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 t = U[(size_t)(mu * 9 + k) * V + s];
        u[k] = {t.x, t.y};
    }
}

template <>
__device__ __forceinline__ void load_link<float>(const float4 *U, int V, int mu, int s, cpx<float> u[9]) {
    unpack_rows(U[(size_t)(mu * 3) * V + s], U[(size_t)(mu * 3 + 1) * V + s], U[(size_t)(mu * 3 + 2) * V + s], u);
}

// Hardware dispatches consecutive workgroups round-robin over the 8 XCDs; give each XCD
// a contiguous range of sites so that stencil neighbours share that XCD's L2.
__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, xcd = b & 7, k = b >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// Plane p of the block order -> (z, t) plane index z + nz t.  The planes are taken in bands of
// g.band consecutive z: t runs over the whole extent inside a band, so that the +-t
// neighbours of a plane were staged g.band blocks earlier (still in L2) rather than nz.
__device__ __forceinline__ int plane_order(int p, const Geom &g) {
    if (g.band == 1) return p;
    const int per = g.band * g.nt, b = p / per, i = p % per;
    return b * g.band + i % g.band + g.nz * (i / g.band);
}

// Neighbours of site s = (x, y) of the (z, t) plane pl = z + nz t without per-thread integer
// divisions (the plane is uniform over a block, so the z and t offsets are too).  The tile
// kernels read the +x and +y neighbours from LDS: fwd[0] and fwd[1] are left at s.
__device__ __forceinline__ Nbr plane_neighbours(int s, int x, int y, int pl, int nx, int ny, int nz, int nt) {
    const int zc = pl % nz, tc = pl / nz;
    const int sxy = nx * ny, sxyz = sxy * nz;
    Nbr nb;
    nb.fwd[0] = nb.fwd[1] = s;
    nb.bwd[0] = x == 0 ? s + (nx - 1) : s - 1;
    nb.bwd[1] = y == 0 ? s + (ny - 1) * nx : s - nx;
    nb.fwd[2] = s + (zc == nz - 1 ? -(nz - 1) * sxy : sxy);
    nb.bwd[2] = s + (zc == 0 ? (nz - 1) * sxy : -sxy);
    nb.fwd[3] = s + (tc == nt - 1 ? -(nt - 1) * sxyz : sxyz);
    nb.bwd[3] = s + (tc == 0 ? (nt - 1) * sxyz : -sxyz);
    return nb;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum of n partials in a fixed order by one wave (lane l takes l, l+64, ...).
__device__ __forceinline__ double wave_sum_partials(const double *p, int n) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) v += p[i];
    return wave_sum(v);
}

__device__ __forceinline__ int slot_of(const Slots &sl, int k) { return sl.list ? sl.list[k] : k; }
__device__ __forceinline__ int slot_count(const Slots &sl) { return sl.count ? *sl.count : sl.n; }

// One storage unit of a spinor: FP64 one complex (double2), FP32 two complexes (float4).
__device__ __forceinline__ void unit_load(const double2 *p, size_t vs, int k, int s, cpx<double> v[1]) {
    const double2 t = p[k * vs + s];
    v[0] = {t.x, t.y};
}
__device__ __forceinline__ void unit_load(const float4 *p, size_t vs, int k, int s, cpx<float> v[2]) {
    const float4 t = p[k * vs + s];
    v[0] = {t.x, t.y};
    v[1] = {t.z, t.w};
}
__device__ __forceinline__ void unit_load_stream(const double2 *p, size_t vs, int k, int s, cpx<double> v[1]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p + k * vs + s));
    v[0] = {t.x, t.y};
}
__device__ __forceinline__ void unit_load_stream(const float4 *p, size_t vs, int k, int s, cpx<float> v[2]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p + k * vs + s));
    v[0] = {t.x, t.y};
    v[1] = {t.z, t.w};
}
__device__ __forceinline__ void unit_store_stream(double2 *p, size_t vs, int k, int s, const cpx<double> v[1]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 t = {v[0].re, v[0].im};
    __builtin_nontemporal_store(t, reinterpret_cast<d2 *>(p + k * vs + s));
}
__device__ __forceinline__ void unit_store_stream(float4 *p, size_t vs, int k, int s, const cpx<float> v[2]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 t = {v[0].re, v[0].im, v[1].re, v[1].im};
    __builtin_nontemporal_store(t, reinterpret_cast<f4 *>(p + k * vs + s));
}

// ------------------------------------------------------------------ stencil epilogues
// At one site, d = [D in](s) (D_W, or D_W^dag) and self = in(s):
//   EPI 0  out = d
//   EPI 1  out = d + sigma aux;                         returns Re <aux, out>(s)
//   EPI 3  out = d;                                     returns |d|^2 + sigma |self|^2
//   EPI 2  a = d + sigma aux, not stored; out, which holds the residual r, becomes r - alpha a;
//          returns |r - alpha a|^2 (a slot whose status is not OK keeps r: alpha is taken as 0)
// In a CG iteration on H^2 + sigma (D_W^dag D_W + sigma) the first stencil D_W p with EPI 3
// yields <p, (H^2 + sigma) p> = |D_W p|^2 + sigma |p|^2, so alpha is known before the second
// stencil, which with EPI 2 updates r directly and never writes (H^2 + sigma) p.  The vectors
// are read and written one storage unit at a time, so that few extra registers are live.
template <class T, int EPI>
__device__ __forceinline__ double stencil_epilogue(cpx<T> d[12], const cpx<T> self[12],
                                                   const typename Store<T>::vec *aux,
                                                   typename Store<T>::vec *out, size_t vs, int s, T sigma,
                                                   T alpha, bool ok) {
    constexpr int UN = Store<T>::units, CU = 12 / UN;   // units per spinor, complexes per unit
    double acc = 0.0;
    if constexpr (EPI == 2) {
        if (!ok) alpha = T(0);   // a broken-down slot keeps its residual (written back unchanged)
    }
#pragma unroll
    for (int k = 0; k < UN; ++k) {
        cpx<T> *dk = d + k * CU;
        if constexpr (EPI == 1 || EPI == 2) {
            cpx<T> a[CU];
            unit_load(aux, vs, k, s, a);
#pragma unroll
            for (int j = 0; j < CU; ++j) {
                dk[j] = dk[j] + sigma * a[j];
                if constexpr (EPI == 1)
                    acc += (double)a[j].re * (double)dk[j].re + (double)a[j].im * (double)dk[j].im;
            }
        }
        if constexpr (EPI == 2) {
            cpx<T> r[CU];
            unit_load_stream(out, vs, k, s, r);
#pragma unroll
            for (int j = 0; j < CU; ++j) {
                r[j] = r[j] - alpha * dk[j];
                acc += (double)r[j].re * (double)r[j].re + (double)r[j].im * (double)r[j].im;
            }
            unit_store_stream(out, vs, k, s, r);
        } else {
            if constexpr (EPI == 3) {
#pragma unroll
                for (int j = 0; j < CU; ++j) {
                    const cpx<T> e = self[k * CU + j];
                    acc += (double)dk[j].re * (double)dk[j].re + (double)dk[j].im * (double)dk[j].im +
                           (double)sigma * ((double)e.re * (double)e.re + (double)e.im * (double)e.im);
                }
            }
            unit_store_stream(out, vs, k, s, dk);
        }
    }
    return acc;
}

// ------------------------------------------------------------------ Wilson stencil
// One right-hand side per thread.  A block of 256 threads covers 256/R consecutive sites
// times R right-hand sides, with the right-hand side in the low bits of the thread index:
// the R threads of one site load the same link addresses in the same wave, so a link is
// fetched once for R right-hand sides without holding R accumulators in registers.
template <int MU, int SF, class T>
__device__ __forceinline__ void hop_dir(const typename Store<T>::link *U, int V, size_t vs,
                                        const typename Store<T>::vec *in, int s, const Nbr &nb, cpx<T> acc[12]) {
    cpx<T> u[9], p[12], h[6], g[6];
    load_link<T>(U, V, MU, s, u);
    Store<T>::load(in, vs, nb.fwd[MU], p);
    project<MU, SF>(p, h);
    su3_mul(u, h, g);
    accumulate<MU, SF>(acc, g);
    load_link<T>(U, V, MU, nb.bwd[MU], u);
    Store<T>::load(in, vs, nb.bwd[MU], p);
    project<MU, -SF>(p, h);
    su3_dag_mul(u, h, g);
    accumulate<MU, -SF>(acc, g);
}

template <class T, int SF>
__device__ __forceinline__ void hop_site(const typename Store<T>::link *U, const Geom &g,
                                         const typename Store<T>::vec *in, int s, cpx<T> acc[12]) {
    const Nbr nb = neighbours(s, g.nx, g.ny, g.nz, g.nt);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
    hop_dir<0, SF, T>(U, g.V, g.vs, in, s, nb, acc);
    hop_dir<1, SF, T>(U, g.V, g.vs, in, s, nb, acc);
    hop_dir<2, SF, T>(U, g.V, g.vs, in, s, nb, acc);
    hop_dir<3, SF, T>(U, g.V, g.vs, in, s, nb, acc);
}

template <class T, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) void k_dslash(const typename Store<T>::link *__restrict__ U,
                                                   const typename Store<T>::vec *__restrict__ in, size_t in_stride,
                                                   size_t in_extra, typename Store<T>::vec *__restrict__ out,
                                                   size_t out_stride, const typename Store<T>::vec *__restrict__ aux,
                                                   size_t aux_stride, size_t aux_extra, Geom g, T kappa, T sigma,
                                                   Slots sl, int lgR, int nsb, double *__restrict__ partial,
                                                   size_t pstride, const double *__restrict__ alpha,
                                                   const int *__restrict__ status) {
    const int R = 1 << lgR;
    const int L = xcd_swizzle(blockIdx.x, gridDim.x);
    const int sb = L % nsb, rg = L / nsb;
    const int cnt = slot_count(sl);
    if (rg * R >= cnt) return;  // uniform over the block
    const int rl = threadIdx.x & (R - 1);
    const int s = sb * (kBlock >> lgR) + (threadIdx.x >> lgR);
    const int k = rg * R + rl;
    const int slot = k < cnt ? slot_of(sl, k) : 0;
    double dot = 0.0;
    if (k < cnt && s < g.V) {
        const auto *src = in + slot * in_stride + in_extra;
        cpx<T> acc[12];
        hop_site<T, DAG ? -1 : 1>(U, g, src, s, acc);
        cpx<T> self[12], v[12];
        Store<T>::load(src, g.vs, s, self);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = self[c] - kappa * acc[c];
        dot = stencil_epilogue<T, EPI>(v, self, aux + slot * aux_stride + aux_extra, out + slot * out_stride, g.vs, s,
                                       sigma, EPI == 2 ? (T)alpha[slot] : T(0),
                                       EPI == 2 ? status[slot] == kStatusOK : true);
    }
    if constexpr (EPI != 0) {
        // lanes with equal (lane mod R) hold the same right-hand side
        for (int off = 32; off >= R; off >>= 1) dot += __shfl_xor(dot, off);
        __shared__ double lds[kBlock / 64][8];
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (lane < R) lds[w][lane] = dot;
        __syncthreads();
        if ((int)threadIdx.x < R) {
            const int kk = rg * R + threadIdx.x;
            if (kk < cnt) {
                double t = 0.0;
#pragma unroll
                for (int i = 0; i < kBlock / 64; ++i) t += lds[i][threadIdx.x];
                partial[(size_t)slot_of(sl, kk) * pstride + sb] = t;
            }
        }
    }
}

// FP32 stencil, one site per thread: the eight two-row links a site needs (U_mu(x) and
// U_mu(x - mu)) are loaded into registers once and applied to NR right-hand sides in turn,
// so link bytes are paid once per NR sides without sharing lanes.  Blocks are ordered
// site-fastest within each XCD's contiguous range.
template <int NR, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) void k_dslash_f32(const float4 *__restrict__ U, const float4 *__restrict__ in,
                                                       size_t in_stride, size_t in_extra, float4 *__restrict__ out,
                                                       size_t out_stride, const float4 *__restrict__ aux,
                                                       size_t aux_stride, size_t aux_extra, Geom g, float kappa,
                                                       float sigma, Slots sl, int nsb, double *__restrict__ partial,
                                                       size_t pstride, const double *__restrict__ alpha,
                                                       const int *__restrict__ status) {
    constexpr int SF = DAG ? -1 : 1;
    const int L = xcd_swizzle(blockIdx.x, gridDim.x);
    const int sb = L % nsb, rg = L / nsb;
    const int cnt = slot_count(sl);
    const int k0 = rg * NR;
    if (k0 >= cnt) return;  // uniform over the block
    const int s = sb * kBlock + threadIdx.x;
    const bool site_ok = s < g.V;
    const int sv = site_ok ? s : 0;
    const Nbr nb = neighbours(sv, g.nx, g.ny, g.nz, g.nt);
    float4 lf[4][3], lb[4][3];
    if (site_ok) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                lf[mu][j] = U[(size_t)(mu * 3 + j) * g.V + sv];
                lb[mu][j] = U[(size_t)(mu * 3 + j) * g.V + nb.bwd[mu]];
            }
    }
    double dot[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dot[r] = 0.0;
#pragma unroll 1
    for (int r = 0; r < NR; ++r) {
        const int k = k0 + r;
        if (k >= cnt) break;  // uniform over the block
        if (!site_ok) continue;
        const int slot = slot_of(sl, k);
        const float4 *src = in + slot * in_stride + in_extra;
        cpx<float> acc[12], u[9], p[12], h[6], w[6];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
#define SMPQ_HOP(MU)                                                                 \
        unpack_rows(lf[MU][0], lf[MU][1], lf[MU][2], u);                             \
        Store<float>::load(src, g.vs, nb.fwd[MU], p);                                \
        project<MU, SF>(p, h);                                                       \
        su3_mul(u, h, w);                                                            \
        accumulate<MU, SF>(acc, w);                                                  \
        unpack_rows(lb[MU][0], lb[MU][1], lb[MU][2], u);                             \
        Store<float>::load(src, g.vs, nb.bwd[MU], p);                                \
        project<MU, -SF>(p, h);                                                      \
        su3_dag_mul(u, h, w);                                                        \
        accumulate<MU, -SF>(acc, w);
        SMPQ_HOP(0)
        SMPQ_HOP(1)
        SMPQ_HOP(2)
        SMPQ_HOP(3)
#undef SMPQ_HOP
        cpx<float> v[12];
        Store<float>::load(src, g.vs, sv, p);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = p[c] - kappa * acc[c];
        dot[r] = stencil_epilogue<float, EPI>(v, p, aux + slot * aux_stride + aux_extra, out + slot * out_stride, g.vs,
                                              sv, sigma, EPI == 2 ? (float)alpha[slot] : 0.f,
                                              EPI == 2 ? status[slot] == kStatusOK : true);
    }
    if constexpr (EPI != 0) {
        __shared__ double lds[NR][kBlock / 64];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double t = wave_sum(dot[r]);
            if (lane == 0) lds[r][wv] = t;
        }
        __syncthreads();
        if ((int)threadIdx.x < NR && k0 + (int)threadIdx.x < cnt) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < kBlock / 64; ++i) t += lds[threadIdx.x][i];
            partial[(size_t)slot_of(sl, k0 + threadIdx.x) * pstride + sb] = t;
        }
    }
}

// FP32 stencil on xy-tiles: a block of nx * ty threads (ty = g.tile_y rows, a divisor of ny)
// covers rows y0 .. y0 + ty - 1 of one (z, t) plane, one site per thread.  For each
// right-hand side the block stages those rows plus one halo row on each side (periodic in y)
// in LDS, so the +-x and +-y neighbours come from LDS and only +-z and +-t from global memory
// (their rows are the tiles of the neighbouring planes).  Links as in k_dslash_f32.
template <int NR, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) void k_dslash_f32_tile(const float4 *__restrict__ U, const float4 *__restrict__ in,
                                                            size_t in_stride, size_t in_extra,
                                                            float4 *__restrict__ out, size_t out_stride,
                                                            const float4 *__restrict__ aux, size_t aux_stride,
                                                            size_t aux_extra, Geom g, float kappa, float sigma,
                                                            Slots sl, int nsb, double *__restrict__ partial,
                                                            size_t pstride, const double *__restrict__ alpha,
                                                            const int *__restrict__ status) {
    constexpr int SF = DAG ? -1 : 1;
    constexpr int kTileSites = kBlock + 2 * 64;
    __shared__ float4 tile[6][kTileSites];
    const int L = xcd_swizzle(blockIdx.x, gridDim.x);
    const int sb = L % nsb, rg = L / nsb;
    const int cnt = slot_count(sl);
    const int k0 = rg * NR;
    if (k0 >= cnt) return;  // uniform over the block
    const int nx = g.nx, ny = g.ny, ty = g.tile_y;
    const int tiles_per_plane = ny / ty;
    const int pl = plane_order(sb / tiles_per_plane, g), y0 = (sb % tiles_per_plane) * ty;
    const int x = threadIdx.x % nx, yl = threadIdx.x / nx;
    const int plane0 = pl * nx * ny;
    const int s = plane0 + (y0 + yl) * nx + x;   // every site is valid: V is a multiple of the tile
    const Nbr nb = plane_neighbours(s, x, y0 + yl, pl, nx, ny, g.nz, g.nt);
    // halo loads: threads 0 .. 2nx-1 also fetch row y0 - 1 (first nx) or y0 + ty (next nx)
    const bool halo = (int)threadIdx.x < 2 * nx;
    const int hrow = threadIdx.x < (unsigned)nx ? 0 : ty + 1;
    const int hy = threadIdx.x < (unsigned)nx ? (y0 + ny - 1) % ny : (y0 + ty) % ny;
    const int hsite = plane0 + hy * nx + x;
    const int hl = hrow * nx + x;
    float4 lf[4][3], lb[4][3];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            lf[mu][j] = U[(size_t)(mu * 3 + j) * g.V + s];
            lb[mu][j] = U[(size_t)(mu * 3 + j) * g.V + nb.bwd[mu]];
        }
    const int me = (yl + 1) * nx + x;
    const int xf = (yl + 1) * nx + (x == nx - 1 ? 0 : x + 1);
    const int xb = (yl + 1) * nx + (x == 0 ? nx - 1 : x - 1);
    const int yf = me + nx, yb = me - nx;
    double dot[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dot[r] = 0.0;
#pragma unroll 1
    for (int r = 0; r < NR; ++r) {
        const int k = k0 + r;
        if (k >= cnt) break;  // uniform over the block
        const int slot = slot_of(sl, k);
        const float4 *src = in + slot * in_stride + in_extra;
        __syncthreads();  // the previous right-hand side is done with the tile
#pragma unroll
        for (int j = 0; j < 6; ++j) tile[j][me] = src[j * g.vs + s];
        if (halo) {
#pragma unroll
            for (int j = 0; j < 6; ++j) tile[j][hl] = src[j * g.vs + hsite];
        }
        cpx<float> acc[12], u[9], p[12], h[6], w[6];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
#define SMPQ_GLOBAL_HOP(MU)                                                          \
        unpack_rows(lf[MU][0], lf[MU][1], lf[MU][2], u);                             \
        Store<float>::load(src, g.vs, nb.fwd[MU], p);                                \
        project<MU, SF>(p, h);                                                       \
        su3_mul(u, h, w);                                                            \
        accumulate<MU, SF>(acc, w);                                                  \
        unpack_rows(lb[MU][0], lb[MU][1], lb[MU][2], u);                             \
        Store<float>::load(src, g.vs, nb.bwd[MU], p);                                \
        project<MU, -SF>(p, h);                                                      \
        su3_dag_mul(u, h, w);                                                        \
        accumulate<MU, -SF>(acc, w);
        SMPQ_GLOBAL_HOP(2)
        SMPQ_GLOBAL_HOP(3)
#undef SMPQ_GLOBAL_HOP
        __syncthreads();  // the tile is complete
#define SMPQ_TILE_LOAD(L, P)                                                         \
        _Pragma("unroll") for (int j = 0; j < 6; ++j) {                              \
            const float4 t_ = tile[j][L];                                            \
            P[2 * j] = {t_.x, t_.y};                                                 \
            P[2 * j + 1] = {t_.z, t_.w};                                             \
        }
#define SMPQ_TILE_HOP(MU, LF, LB)                                                    \
        unpack_rows(lf[MU][0], lf[MU][1], lf[MU][2], u);                             \
        SMPQ_TILE_LOAD(LF, p)                                                        \
        project<MU, SF>(p, h);                                                       \
        su3_mul(u, h, w);                                                            \
        accumulate<MU, SF>(acc, w);                                                  \
        unpack_rows(lb[MU][0], lb[MU][1], lb[MU][2], u);                             \
        SMPQ_TILE_LOAD(LB, p)                                                        \
        project<MU, -SF>(p, h);                                                      \
        su3_dag_mul(u, h, w);                                                        \
        accumulate<MU, -SF>(acc, w);
        SMPQ_TILE_HOP(0, xf, xb)
        SMPQ_TILE_HOP(1, yf, yb)
#undef SMPQ_TILE_HOP
        cpx<float> v[12];
        SMPQ_TILE_LOAD(me, p)
#undef SMPQ_TILE_LOAD
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = p[c] - kappa * acc[c];
        dot[r] = stencil_epilogue<float, EPI>(v, p, aux + slot * aux_stride + aux_extra, out + slot * out_stride, g.vs,
                                              s, sigma, EPI == 2 ? (float)alpha[slot] : 0.f,
                                              EPI == 2 ? status[slot] == kStatusOK : true);
    }
    if constexpr (EPI != 0) {
        __shared__ double lds[NR][kBlock / 64];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int nw = blockDim.x >> 6;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double t = wave_sum(dot[r]);
            if (lane == 0) lds[r][wv] = t;
        }
        __syncthreads();
        if ((int)threadIdx.x < NR && k0 + (int)threadIdx.x < cnt) {
            double t = 0.0;
            for (int i = 0; i < nw; ++i) t += lds[threadIdx.x][i];
            partial[(size_t)slot_of(sl, k0 + threadIdx.x) * pstride + sb] = t;
        }
    }
}

template <int NR, bool DAG, int EPI, bool XYL>
__device__ __forceinline__ void dslash_f32_plane_body(const float4 *__restrict__ U, const float4 *__restrict__ in,
                                                             size_t in_stride, size_t in_extra,
                                                             float4 *__restrict__ out, size_t out_stride,
                                                             const float4 *__restrict__ aux, size_t aux_stride,
                                                             size_t aux_extra, Geom g, float kappa, float sigma,
                                                             Slots sl, int nsb, double *__restrict__ partial,
                                                             size_t pstride, const double *__restrict__ alpha,
                                                             const int *__restrict__ status) {
    constexpr int SF = DAG ? -1 : 1;
    __shared__ float4 tile[6][kBlock];
    // XYL: the plane's x and y links in LDS (the backward ones are the neighbours' forward
    // links within the plane), so that fewer registers per thread hold links
    __shared__ float4 lxy[XYL ? 2 : 1][3][XYL ? kBlock : 1];
    const int L = xcd_swizzle(blockIdx.x, gridDim.x);
    const int sb = L % nsb, rg = L / nsb;
    const int cnt = slot_count(sl);
    const int k0 = rg * NR;
    if (k0 >= cnt) return;  // uniform over the block
    const int base = plane_order(sb, g) * kBlock;
    const int s = base + threadIdx.x;  // every site is valid: V is a multiple of the plane
    const Nbr nb = neighbours(s, g.nx, g.ny, g.nz, g.nt);
    float4 lf[4][3], lb[4][3];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (XYL && mu < 2) {
                if constexpr (XYL) lxy[mu][j][threadIdx.x] = U[(size_t)(mu * 3 + j) * g.V + s];
                continue;   // visible after the first barrier of the loop below
            }
            lf[mu][j] = U[(size_t)(mu * 3 + j) * g.V + s];
            lb[mu][j] = U[(size_t)(mu * 3 + j) * g.V + nb.bwd[mu]];
        }
    const int xf = nb.fwd[0] - base, xb = nb.bwd[0] - base, yf = nb.fwd[1] - base, yb = nb.bwd[1] - base;
    // EPI 1: per right-hand side, the block's <aux, out> is summed per wave at once and the
    // wave sums kept in LDS (no accumulators held across the loop)
    __shared__ double ldsdot[EPI != 0 ? NR : 1][kBlock / 64];
    [[maybe_unused]] const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll 1
    for (int r = 0; r < NR; ++r) {
        const int k = k0 + r;
        if (k >= cnt) break;  // uniform over the block
        const int slot = slot_of(sl, k);
        const float4 *src = in + slot * in_stride + in_extra;
        __syncthreads();  // the previous right-hand side is done with the tile
#pragma unroll
        for (int j = 0; j < 6; ++j) tile[j][threadIdx.x] = src[j * g.vs + s];
        cpx<float> acc[12], u[9], p[12], h[6], w[6];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
#define SMPQ_GLOBAL_HOP(MU)                                                          \
        unpack_rows(lf[MU][0], lf[MU][1], lf[MU][2], u);                             \
        Store<float>::load(src, g.vs, nb.fwd[MU], p);                                \
        project<MU, SF>(p, h);                                                       \
        su3_mul(u, h, w);                                                            \
        accumulate<MU, SF>(acc, w);                                                  \
        unpack_rows(lb[MU][0], lb[MU][1], lb[MU][2], u);                             \
        Store<float>::load(src, g.vs, nb.bwd[MU], p);                                \
        project<MU, -SF>(p, h);                                                      \
        su3_dag_mul(u, h, w);                                                        \
        accumulate<MU, -SF>(acc, w);
        SMPQ_GLOBAL_HOP(2)
        SMPQ_GLOBAL_HOP(3)
#undef SMPQ_GLOBAL_HOP
        __syncthreads();  // the tile is complete
#define SMPQ_TILE_LOAD(L, P)                                                         \
        _Pragma("unroll") for (int j = 0; j < 6; ++j) {                              \
            const float4 t_ = tile[j][L];                                            \
            P[2 * j] = {t_.x, t_.y};                                                 \
            P[2 * j + 1] = {t_.z, t_.w};                                             \
        }
#define SMPQ_TILE_HOP(MU, LF, LB)                                                    \
        if constexpr (XYL) unpack_rows(lxy[MU][0][threadIdx.x], lxy[MU][1][threadIdx.x],  \
                                       lxy[MU][2][threadIdx.x], u);                  \
        else unpack_rows(lf[MU][0], lf[MU][1], lf[MU][2], u);                        \
        SMPQ_TILE_LOAD(LF, p)                                                        \
        project<MU, SF>(p, h);                                                       \
        su3_mul(u, h, w);                                                            \
        accumulate<MU, SF>(acc, w);                                                  \
        if constexpr (XYL) unpack_rows(lxy[MU][0][LB], lxy[MU][1][LB], lxy[MU][2][LB], u); \
        else unpack_rows(lb[MU][0], lb[MU][1], lb[MU][2], u);                        \
        SMPQ_TILE_LOAD(LB, p)                                                        \
        project<MU, -SF>(p, h);                                                      \
        su3_dag_mul(u, h, w);                                                        \
        accumulate<MU, -SF>(acc, w);
        SMPQ_TILE_HOP(0, xf, xb)
        SMPQ_TILE_HOP(1, yf, yb)
#undef SMPQ_TILE_HOP
        cpx<float> v[12];
        SMPQ_TILE_LOAD(threadIdx.x, p)
#undef SMPQ_TILE_LOAD
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = p[c] - kappa * acc[c];
        double d = stencil_epilogue<float, EPI>(v, p, aux + slot * aux_stride + aux_extra, out + slot * out_stride,
                                                g.vs, s, sigma, EPI == 2 ? (float)alpha[slot] : 0.f,
                                                EPI == 2 ? status[slot] == kStatusOK : true);
        if constexpr (EPI != 0) {
            d = wave_sum(d);
            if (lane == 0) ldsdot[r][wv] = d;
        }
    }
    if constexpr (EPI != 0) {
        __syncthreads();
        if ((int)threadIdx.x < NR && k0 + (int)threadIdx.x < cnt) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < kBlock / 64; ++i) t += ldsdot[threadIdx.x][i];
            partial[(size_t)slot_of(sl, k0 + threadIdx.x) * pstride + sb] = t;
        }
    }
}


template <int NR, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) void k_dslash_f32_plane(const float4 *__restrict__ U, const float4 *__restrict__ in,
                                                             size_t in_stride, size_t in_extra,
                                                             float4 *__restrict__ out, size_t out_stride,
                                                             const float4 *__restrict__ aux, size_t aux_stride,
                                                             size_t aux_extra, Geom g, float kappa, float sigma,
                                                             Slots sl, int nsb, double *__restrict__ partial,
                                                             size_t pstride, const double *__restrict__ alpha,
                                                             const int *__restrict__ status) {
    dslash_f32_plane_body<NR, DAG, EPI, false>(U, in, in_stride, in_extra, out, out_stride, aux, aux_stride, aux_extra,
                                               g, kappa, sigma, sl, nsb, partial, pstride, alpha, status);
}

// The same with the x and y links in LDS, at 3 waves per SIMD.
template <int NR, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_dslash_f32_plane_xyl(
    const float4 *__restrict__ U, const float4 *__restrict__ in, size_t in_stride, size_t in_extra,
    float4 *__restrict__ out, size_t out_stride, const float4 *__restrict__ aux, size_t aux_stride, size_t aux_extra,
    Geom g, float kappa, float sigma, Slots sl, int nsb, double *__restrict__ partial, size_t pstride,
    const double *__restrict__ alpha, const int *__restrict__ status) {
    dslash_f32_plane_body<NR, DAG, EPI, true>(U, in, in_stride, in_extra, out, out_stride, aux, aux_stride, aux_extra,
                                              g, kappa, sigma, sl, nsb, partial, pstride, alpha, status);
}

// Stencil on xy-tiles with the links read for every right-hand side (FP64 kind 1, FP32 kind 4):
// a block of nx * ty threads (ty = g.tile_y rows of one (z, t) plane, one site per thread)
// stages, per right-hand side, its rows of the input in LDS (with one halo row on each side,
// unless the tile is the whole plane and y wraps inside it), so that the +-x and +-y neighbours
// come from LDS and only +-z and +-t from global memory.  Links: their first two rows (FP64
// 96 bytes, FP32 48), the third rebuilt as conj(row0 x row1) (exact for SU(3) up to rounding),
// read for every right-hand side from L2 rather than held in registers across them, which
// leaves registers for two (FP64) or more (FP32) waves per SIMD.
__device__ __forceinline__ void load_link64_rows(const double2 *U, int V, int mu, int s, cpx<double> u[9]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double2 t = U[(size_t)(mu * 9 + k) * V + s];
        u[k] = {t.x, t.y};
    }
    const cpx<double> r0 = cfma(u[1], u[5], -1.0 * cmul(u[2], u[4]));
    const cpx<double> r1 = cfma(u[2], u[3], -1.0 * cmul(u[0], u[5]));
    const cpx<double> r2 = cfma(u[0], u[4], -1.0 * cmul(u[1], u[3]));
    u[6] = {r0.re, -r0.im};
    u[7] = {r1.re, -r1.im};
    u[8] = {r2.re, -r2.im};
}
__device__ __forceinline__ void load_link_rows(const double2 *U, int V, int mu, int s, cpx<double> u[9]) {
    load_link64_rows(U, V, mu, s, u);
}
__device__ __forceinline__ void load_link_rows(const float4 *U, int V, int mu, int s, cpx<float> u[9]) {
    load_link<float>(U, V, mu, s, u);
}
// the spinor at LDS position l of a tile held as [unit][tsites]
__device__ __forceinline__ void tile_read(const double2 *tile, int tsites, int l, cpx<double> p[12]) {
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        const double2 t = tile[j * tsites + l];
        p[j] = {t.x, t.y};
    }
}
__device__ __forceinline__ void tile_read(const float4 *tile, int tsites, int l, cpx<float> p[12]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const float4 t = tile[j * tsites + l];
        p[2 * j] = {t.x, t.y};
        p[2 * j + 1] = {t.z, t.w};
    }
}

// Waves per SIMD the tile kernel is compiled for: the FP64 kernel with one right-hand side per
// block needs 164-171 VGPRs, just above the 168 that three waves allow.  The solver's two
// epilogues (3 and 2) fit 168 with at most two registers spilled and run the pair 9 % faster than
// at two waves; the plain D_W and the +sigma epilogue would spill 5-10 and keep two waves, as do
// all other instances.
template <class T, int NR, int EPI>
struct TileWaves {
    static constexpr int min = std::is_same<T, double>::value && NR == 1 && (EPI == 2 || EPI == 3) ? 3 : 1;
};

template <class T, int NR, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(TileWaves<T, NR, EPI>::min, 8))) void k_dslash_tile_rl(const typename Store<T>::link *__restrict__ U,
                                                           const typename Store<T>::vec *__restrict__ in,
                                                           size_t in_stride, size_t in_extra,
                                                           typename Store<T>::vec *__restrict__ out, size_t out_stride,
                                                           const typename Store<T>::vec *__restrict__ aux,
                                                           size_t aux_stride, size_t aux_extra, Geom g, T kappa,
                                                           T sigma, Slots sl, int nsb, double *__restrict__ partial,
                                                           size_t pstride, const double *__restrict__ alpha,
                                                           const int *__restrict__ status) {
    using vec = typename Store<T>::vec;
    using link = typename Store<T>::link;
    constexpr int SF = DAG ? -1 : 1;
    constexpr int UN = Store<T>::units;
    extern __shared__ __align__(16) unsigned char tile_raw[];
    vec *tile = reinterpret_cast<vec *>(tile_raw);   // [UN][tsites]
    const int L = xcd_swizzle(blockIdx.x, gridDim.x);
    // block order: groups of IL right-hand-side groups, tiles, then the IL groups of one tile
    // fastest (IL = 1: the tiles of one right-hand-side group in a row)
    const int IL = std::is_same<T, double>::value ? g.f64_il : g.f32_il;
    const int grp = L / (nsb * IL), rem = L - grp * nsb * IL;
    const int sb = rem / IL, rg = grp * IL + (rem - sb * IL);
    const int cnt = slot_count(sl);
    const int k0 = rg * NR;
    if (k0 >= cnt) return;  // uniform over the block
    const int nx = g.nx, ny = g.ny, ty = g.tile_y;
    const bool whole = ty == ny;             // the tile is the plane: y wraps inside it
    const int rows = whole ? ty : ty + 2;    // tile rows held in LDS
    const int tsites = rows * nx;
    const int tiles_per_plane = ny / ty;
    const int pl = plane_order(sb / tiles_per_plane, g), y0 = (sb % tiles_per_plane) * ty;
    const int x = threadIdx.x % nx, yl = threadIdx.x / nx;
    const int plane0 = pl * nx * ny;
    const int s = plane0 + (y0 + yl) * nx + x;   // every site is valid: V is a multiple of the tile
    const Nbr nb = plane_neighbours(s, x, y0 + yl, pl, nx, ny, g.nz, g.nt);
    // LDS row of tile row yl: shifted by the lower halo row when there is one
    const int off = whole ? 0 : 1;
    const int me = (yl + off) * nx + x;
    const int xf = (yl + off) * nx + (x == nx - 1 ? 0 : x + 1);
    const int xb = (yl + off) * nx + (x == 0 ? nx - 1 : x - 1);
    const int yf = whole ? ((yl + 1) % ty) * nx + x : me + nx;
    const int yb = whole ? ((yl + ty - 1) % ty) * nx + x : me - nx;
    const bool halo = !whole && (int)threadIdx.x < 2 * nx;
    const int hrow = threadIdx.x < (unsigned)nx ? 0 : ty + 1;
    const int hy = threadIdx.x < (unsigned)nx ? (y0 + ny - 1) % ny : (y0 + ty) % ny;
    const int hsite = plane0 + hy * nx + x;
    const int hl = hrow * nx + x;
    __shared__ double ldsdot[EPI != 0 ? NR : 1][kBlock / 64];
    [[maybe_unused]] const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll 1
    for (int r = 0; r < NR; ++r) {
        const int k = k0 + r;
        if (k >= cnt) break;  // uniform over the block
        const int slot = slot_of(sl, k);
        const vec *src = in + slot * in_stride + in_extra;
        // the links are re-read for every right-hand side: an empty asm makes the base pointer
        // opaque in each iteration, so that the compiler does not hoist all eight links out of
        // the loop into registers
        const link *Ur = U;
        asm volatile("" : "+s"(Ur));
        __syncthreads();  // the previous right-hand side is done with the tile
#pragma unroll
        for (int j = 0; j < UN; ++j) tile[j * tsites + me] = src[j * g.vs + s];
        if (halo) {
#pragma unroll
            for (int j = 0; j < UN; ++j) tile[j * tsites + hl] = src[j * g.vs + hsite];
        }
        __builtin_amdgcn_sched_barrier(0);   // the staging loads are not held across the hops
        cpx<T> acc[12], u[9], p[12], h[6], w[6];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
#define SMPQ_HOPT(MU, LOADF, LOADB)                                                  \
        load_link_rows(Ur, g.V, MU, s, u);                                           \
        LOADF                                                                        \
        project<MU, SF>(p, h);                                                       \
        su3_mul(u, h, w);                                                            \
        accumulate<MU, SF>(acc, w);                                                  \
        load_link_rows(Ur, g.V, MU, nb.bwd[MU], u);                                  \
        LOADB                                                                        \
        project<MU, -SF>(p, h);                                                      \
        su3_dag_mul(u, h, w);                                                        \
        accumulate<MU, -SF>(acc, w);
#define SMPQ_GT(S_) Store<T>::load(src, g.vs, S_, p);
#define SMPQ_TT(L_) tile_read(tile, tsites, L_, p);
        // one direction at a time: loads of later directions hoisted above earlier ones would hold
        // more links and spinors in registers than the occupancy target allows
        SMPQ_HOPT(2, SMPQ_GT(nb.fwd[2]), SMPQ_GT(nb.bwd[2]))
        __builtin_amdgcn_sched_barrier(0);
        SMPQ_HOPT(3, SMPQ_GT(nb.fwd[3]), SMPQ_GT(nb.bwd[3]))
        __syncthreads();  // the tile is complete
        SMPQ_HOPT(0, SMPQ_TT(xf), SMPQ_TT(xb))
        __builtin_amdgcn_sched_barrier(0);
        SMPQ_HOPT(1, SMPQ_TT(yf), SMPQ_TT(yb))
        cpx<T> v[12];
        SMPQ_TT(me)
#undef SMPQ_TT
#undef SMPQ_GT
#undef SMPQ_HOPT
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = p[c] - kappa * acc[c];
        double d = stencil_epilogue<T, EPI>(v, p, aux + slot * aux_stride + aux_extra, out + slot * out_stride, g.vs, s,
                                            sigma, EPI == 2 ? (T)alpha[slot] : T(0),
                                            EPI == 2 ? status[slot] == kStatusOK : true);
        if constexpr (EPI != 0) {
            d = wave_sum(d);
            if (lane == 0) ldsdot[r][wv] = d;
        }
    }
    if constexpr (EPI != 0) {
        __syncthreads();
        if ((int)threadIdx.x < NR && k0 + (int)threadIdx.x < cnt) {
            double t = 0.0;
            for (int i = 0; i < nw; ++i) t += ldsdot[threadIdx.x][i];
            partial[(size_t)slot_of(sl, k0 + threadIdx.x) * pstride + sb] = t;
        }
    }
}

__host__ __device__ int site_blocks(const Geom &g) { return (g.V + kBlock - 1) / kBlock; }
static int fp64_parts(const Geom &g) { return (g.V + (kBlock >> g.f64_lgr) - 1) / (kBlock >> g.f64_lgr); }
size_t partial_stride(const Geom &g) { return (size_t)12 * site_blocks(g); }
bool plane_tileable(const Geom &g) { return g.nx * g.ny == kBlock; }

int tile_rows(int nx, int ny) {
    if (nx > 64) return 0;
    for (int ty = kBlock / nx; ty >= 2; --ty)
        if (ny % ty == 0 && (nx * ty) % 64 == 0) return ty;
    return 0;
}

static int tile_blocks(const Geom &g) { return g.V / (g.nx * g.tile_y); }

// g with the FP32 variant of one direction in f32_kind, f32_nr and f32_il
static Geom for_direction(const Geom &g, int prec, bool dag) {
    Geom d = g;
    if (prec != 0 && dag) {
        d.f32_kind = g.f32_dag_kind;
        d.f32_nr = g.f32_dag_nr;
        d.f32_il = g.f32_dag_il;
    }
    return d;
}

int dslash_partials(int prec, const Geom &g, bool dag) {
    if (prec == 0) return g.f64_kind == 1 ? tile_blocks(g) : fp64_parts(g);
    const Geom d = for_direction(g, prec, dag);
    return d.f32_kind == 2 || d.f32_kind == 4 ? tile_blocks(d) : site_blocks(d);
}

static bool il_ok(int il) { return il == 1 || il == 2 || il == 4 || il == 8 || il == 16; }

static bool valid_f32(const Geom &g);

bool valid_tuning(int prec, const Geom &g) {
    if (prec != 0) return valid_f32(g) && valid_f32(for_direction(g, prec, true));
    if (g.f64_kind == 1)
        return g.tile_y > 0 && g.tile_y == tile_rows(g.nx, g.ny) && g.band >= 1 && g.nz % g.band == 0 &&
               (g.f64_nr == 1 || g.f64_nr == 2 || g.f64_nr == 4 || g.f64_nr == 8) && il_ok(g.f64_il);
    return g.f64_kind == 0 && g.f64_lgr >= 0 && g.f64_lgr <= 2 && g.f64_il == 1;
}

static bool valid_f32(const Geom &g) {
    if (g.f32_kind != 4 && g.f32_il != 1) return false;   // the interleave applies to kind 4 only
    const bool nr_tile = g.f32_nr == 4 || g.f32_nr == 8 || g.f32_nr == 16;
    if (g.f32_kind == 1 || g.f32_kind == 3) return plane_tileable(g) && nr_tile && g.band >= 1 && g.nz % g.band == 0;
    const bool tiled = g.tile_y > 0 && g.tile_y == tile_rows(g.nx, g.ny);
    const bool band_ok = g.band >= 1 && g.nz % g.band == 0;
    if (g.f32_kind == 2) return tiled && nr_tile && band_ok;
    if (g.f32_kind == 4)
        return tiled && band_ok && (g.f32_nr == 1 || g.f32_nr == 2 || g.f32_nr == 4 || g.f32_nr == 8) && il_ok(g.f32_il);
    return g.f32_kind == 0 && (g.f32_nr == 2 || g.f32_nr == 4 || g.f32_nr == 8);
}

template <class T, int NR, bool DAG, int EPI>
static void launch_tile_rl(const void *U, const void *in, size_t in_stride, size_t in_extra, void *out,
                           size_t out_stride, const void *aux, size_t aux_stride, size_t aux_extra, const Geom &g,
                           double kappa, double sigma, Slots sl, int max_slots, double *partial, const double *alpha,
                           const int *status, hipStream_t st) {
    using vec = typename Store<T>::vec;
    using link = typename Store<T>::link;
    const int nsb = tile_blocks(g);
    const int il = std::is_same<T, double>::value ? g.f64_il : g.f32_il;
    // right-hand-side groups, rounded up to whole interleave groups (the extra blocks exit)
    const int ngr = ((max_slots + NR - 1) / NR + il - 1) / il * il;
    const int rows = g.tile_y == g.ny ? g.tile_y : g.tile_y + 2;
    const size_t lds = (size_t)rows * g.nx * Store<T>::units * sizeof(vec);
    hipLaunchKernelGGL((k_dslash_tile_rl<T, NR, DAG, EPI>), dim3(nsb * ngr), dim3(g.nx * g.tile_y), lds, st,
                       (const link *)U, (const vec *)in, in_stride, in_extra, (vec *)out, out_stride, (const vec *)aux,
                       aux_stride, aux_extra, g, (T)kappa, (T)sigma, sl, nsb, partial, partial_stride(g), alpha,
                       status);
}

template <class T, bool DAG, int EPI>
static void launch_dslash_t(const void *U, const void *in, size_t in_stride, size_t in_extra, void *out,
                            size_t out_stride, const void *aux, size_t aux_stride, size_t aux_extra, const Geom &g,
                            double kappa, double sigma, Slots sl, int max_slots, double *partial, const double *alpha,
                            const int *status, hipStream_t st) {
    using vec = typename Store<T>::vec;
    using link = typename Store<T>::link;
    if constexpr (std::is_same<T, double>::value) {
        if (g.f64_kind == 1) {
#define SMPQ_F64T(NR)                                                                                             \
    launch_tile_rl<double, NR, DAG, EPI>(U, in, in_stride, in_extra, out, out_stride, aux, aux_stride, aux_extra, g, \
                                         kappa, sigma, sl, max_slots, partial, alpha, status, st)
            if (g.f64_nr == 1) SMPQ_F64T(1);
            else if (g.f64_nr == 2) SMPQ_F64T(2);
            else if (g.f64_nr == 8) SMPQ_F64T(8);
            else SMPQ_F64T(4);
#undef SMPQ_F64T
            return;
        }
    }
    const int lgR = g.f64_lgr;
    const int R = 1 << lgR;
    const int nsb = fp64_parts(g);
    const int ngr = (max_slots + R - 1) / R;
    hipLaunchKernelGGL((k_dslash<T, DAG, EPI>), dim3(nsb * ngr), dim3(kBlock), 0, st, (const link *)U,
                       (const vec *)in, in_stride, in_extra, (vec *)out, out_stride, (const vec *)aux, aux_stride,
                       aux_extra, g, (T)kappa, (T)sigma, sl, lgR, nsb, partial, partial_stride(g), alpha, status);
}

template <int NR, bool DAG, int EPI, int KIND>
static void launch_f32(const void *U, const void *in, size_t in_stride, size_t in_extra, void *out, size_t out_stride,
                       const void *aux, size_t aux_stride, size_t aux_extra, const Geom &g, double kappa, double sigma,
                       Slots sl, int max_slots, double *partial, const double *alpha, const int *status,
                       hipStream_t st) {
    const int nsb = KIND == 2 ? tile_blocks(g) : site_blocks(g);
    const int ngr = (max_slots + NR - 1) / NR;
    if constexpr (KIND == 2)
        hipLaunchKernelGGL((k_dslash_f32_tile<NR, DAG, EPI>), dim3(nsb * ngr), dim3(g.nx * g.tile_y), 0, st,
                           (const float4 *)U, (const float4 *)in, in_stride, in_extra, (float4 *)out, out_stride,
                           (const float4 *)aux, aux_stride, aux_extra, g, (float)kappa, (float)sigma, sl, nsb, partial,
                           partial_stride(g), alpha, status);
    else if constexpr (KIND == 3)
        hipLaunchKernelGGL((k_dslash_f32_plane_xyl<NR, DAG, EPI>), dim3(nsb * ngr), dim3(kBlock), 0, st,
                           (const float4 *)U, (const float4 *)in, in_stride, in_extra, (float4 *)out, out_stride,
                           (const float4 *)aux, aux_stride, aux_extra, g, (float)kappa, (float)sigma, sl, nsb, partial,
                           partial_stride(g), alpha, status);
    else if constexpr (KIND == 1)
        hipLaunchKernelGGL((k_dslash_f32_plane<NR, DAG, EPI>), dim3(nsb * ngr), dim3(kBlock), 0, st,
                           (const float4 *)U, (const float4 *)in, in_stride, in_extra, (float4 *)out, out_stride,
                           (const float4 *)aux, aux_stride, aux_extra, g, (float)kappa, (float)sigma, sl, nsb, partial,
                           partial_stride(g), alpha, status);
    else
        hipLaunchKernelGGL((k_dslash_f32<NR, DAG, EPI>), dim3(nsb * ngr), dim3(kBlock), 0, st, (const float4 *)U,
                           (const float4 *)in, in_stride, in_extra, (float4 *)out, out_stride, (const float4 *)aux,
                           aux_stride, aux_extra, g, (float)kappa, (float)sigma, sl, nsb, partial, partial_stride(g),
                           alpha, status);
}

template <bool DAG, int EPI>
static void launch_f32_tuned(const void *U, const void *in, size_t in_stride, size_t in_extra, void *out,
                             size_t out_stride, const void *aux, size_t aux_stride, size_t aux_extra, const Geom &g,
                             double kappa, double sigma, Slots sl, int max_slots, double *partial,
                             const double *alpha, const int *status, hipStream_t st) {
#define SMPQ_F32(NR, PL)                                                                                       \
    launch_f32<NR, DAG, EPI, PL>(U, in, in_stride, in_extra, out, out_stride, aux, aux_stride, aux_extra, g, kappa, \
                                 sigma, sl, max_slots, partial, alpha, status, st)
    if (g.f32_kind == 4) {
#define SMPQ_F32RL(NR)                                                                                            \
    launch_tile_rl<float, NR, DAG, EPI>(U, in, in_stride, in_extra, out, out_stride, aux, aux_stride, aux_extra, g, \
                                        kappa, sigma, sl, max_slots, partial, alpha, status, st)
        if (g.f32_nr == 1) SMPQ_F32RL(1);
        else if (g.f32_nr == 2) SMPQ_F32RL(2);
        else if (g.f32_nr == 8) SMPQ_F32RL(8);
        else SMPQ_F32RL(4);
#undef SMPQ_F32RL
    } else if (g.f32_kind == 2) {
        if (g.f32_nr == 4) SMPQ_F32(4, 2);
        else if (g.f32_nr == 16) SMPQ_F32(16, 2);
        else SMPQ_F32(8, 2);
    } else if (g.f32_kind == 1) {
        if (g.f32_nr == 4) SMPQ_F32(4, 1);
        else if (g.f32_nr == 16) SMPQ_F32(16, 1);
        else SMPQ_F32(8, 1);
    } else if (g.f32_kind == 3) {
        if (g.f32_nr == 4) SMPQ_F32(4, 3);
        else if (g.f32_nr == 16) SMPQ_F32(16, 3);
        else SMPQ_F32(8, 3);
    } else {
        if (g.f32_nr == 2) SMPQ_F32(2, 0);
        else if (g.f32_nr == 8) SMPQ_F32(8, 0);
        else SMPQ_F32(4, 0);
    }
#undef SMPQ_F32
}

void launch_dslash(int prec, bool dag, int epi, const void *U, const void *in, size_t in_stride, size_t in_extra,
                   void *out, size_t out_stride, const void *aux, size_t aux_stride, size_t aux_extra, const Geom &g,
                   double kappa, double sigma, Slots sl, int max_slots, double *partial, hipStream_t st,
                   const double *alpha, const int *status) {
    using Fn = void (*)(const void *, const void *, size_t, size_t, void *, size_t, const void *, size_t, size_t,
                        const Geom &, double, double, Slots, int, double *, const double *, const int *, hipStream_t);
    if (!valid_tuning(prec, g)) throw std::invalid_argument("stencil variant does not fit this lattice");
    if (epi < 0 || epi > 3) throw std::invalid_argument("unknown stencil epilogue");
    if (epi == 2 && (!alpha || !status)) throw std::invalid_argument("the residual epilogue needs alpha and status");
    // [precision][dagger][epilogue]; the FP32 stencil is built for the combinations the solver,
    // the autotuner and smpq_apply_dw use
    static const Fn table[2][2][4] = {
        {{launch_dslash_t<double, false, 0>, launch_dslash_t<double, false, 1>, launch_dslash_t<double, false, 2>,
          launch_dslash_t<double, false, 3>},
         {launch_dslash_t<double, true, 0>, launch_dslash_t<double, true, 1>, launch_dslash_t<double, true, 2>,
          launch_dslash_t<double, true, 3>}},
        {{launch_f32_tuned<false, 0>, nullptr, nullptr, launch_f32_tuned<false, 3>},
         {launch_f32_tuned<true, 0>, launch_f32_tuned<true, 1>, launch_f32_tuned<true, 2>, nullptr}}};
    const Fn f = table[prec == 0 ? 0 : 1][dag ? 1 : 0][epi];
    if (!f) throw std::invalid_argument("stencil epilogue not built for this precision and direction");
    f(U, in, in_stride, in_extra, out, out_stride, aux, aux_stride, aux_extra, for_direction(g, prec, dag), kappa,
      sigma, sl, max_slots, partial, alpha, status, st);
}

// ------------------------------------------------------------------ element-wise kernels
// Element-wise kernels work on one storage unit per thread: a float4 (two complex
// entries) in FP32 or a double2 (one complex entry) in FP64.  Block b of a slot covers
// unit u = b / nsb and sites (b % nsb)*256 + [0, 256), so a wave reads 64 consecutive
// units of one component plane.
template <class T>
struct Unit;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <>
struct Unit<float> {
    static constexpr int C = 2;
    __device__ static __forceinline__ void load(const float4 *p, size_t vs, int u, int s, cpx<float> v[2]) {
        const float4 t = p[u * vs + s];
        v[0] = {t.x, t.y};
        v[1] = {t.z, t.w};
    }
    __device__ static __forceinline__ void store(float4 *p, size_t vs, int u, int s, const cpx<float> v[2]) {
        p[u * vs + s] = make_float4(v[0].re, v[0].im, v[1].re, v[1].im);
    }
    // streamed (non-temporal) vector load/store: data touched once per kernel
    __device__ static __forceinline__ void load_stream(const float4 *p, size_t vs, int u, int s, cpx<float> v[2]) {
        const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p + u * vs + s));
        v[0] = {t.x, t.y};
        v[1] = {t.z, t.w};
    }
    __device__ static __forceinline__ void store_stream(float4 *p, size_t vs, int u, int s, const cpx<float> v[2]) {
        const f32x4 t = {v[0].re, v[0].im, v[1].re, v[1].im};
        __builtin_nontemporal_store(t, reinterpret_cast<f32x4 *>(p + u * vs + s));
    }
};

template <>
struct Unit<double> {
    static constexpr int C = 1;
    __device__ static __forceinline__ void load(const double2 *p, size_t vs, int u, int s, cpx<double> v[1]) {
        const double2 t = p[u * vs + s];
        v[0] = {t.x, t.y};
    }
    __device__ static __forceinline__ void store(double2 *p, size_t vs, int u, int s, const cpx<double> v[1]) {
        p[u * vs + s] = make_double2(v[0].re, v[0].im);
    }
    __device__ static __forceinline__ void load_stream(const double2 *p, size_t vs, int u, int s, cpx<double> v[1]) {
        const f64x2 t = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p + u * vs + s));
        v[0] = {t.x, t.y};
    }
    __device__ static __forceinline__ void store_stream(double2 *p, size_t vs, int u, int s, const cpx<double> v[1]) {
        const f64x2 t = {v[0].re, v[0].im};
        __builtin_nontemporal_store(t, reinterpret_cast<f64x2 *>(p + u * vs + s));
    }
};

// FP64 complex entry c of an FP64 spinor (double2 planes), streamed (non-temporal)
__device__ __forceinline__ cpx<double> ld64_stream(const double2 *p, size_t vs, int c, int s) {
    const f64x2 t = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p + c * vs + s));
    return {t.x, t.y};
}
__device__ __forceinline__ void st64_stream(double2 *p, size_t vs, int c, int s, cpx<double> v) {
    const f64x2 t = {v.re, v.im};
    __builtin_nontemporal_store(t, reinterpret_cast<f64x2 *>(p + c * vs + s));
}

// A shifted search direction in 16 bits: one FP32 unit (4 reals) in 8 bytes, holding p / scale.
// Conversions round to nearest even (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32 on gfx950).
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
template <int D>
struct Dir16;
template <>
struct Dir16<kDirF16> {
    using v = f16x4;
};
template <>
struct Dir16<kDirBF16> {
    using v = bf16x4;
};

template <int D>
__device__ __forceinline__ void load_dir16(const void *p, size_t vs, int u, int s, float scale, cpx<float> v[2]) {
    using h = typename Dir16<D>::v;
    const h t = __builtin_nontemporal_load(reinterpret_cast<const h *>(p) + u * vs + s);
    const f32x4 f = __builtin_convertvector(t, f32x4);
    v[0] = {f.x * scale, f.y * scale};
    v[1] = {f.z * scale, f.w * scale};
}
template <int D>
__device__ __forceinline__ void store_dir16(void *p, size_t vs, int u, int s, float inv_scale, const cpx<float> v[2]) {
    using h = typename Dir16<D>::v;
    const f32x4 f = {v[0].re * inv_scale, v[0].im * inv_scale, v[1].re * inv_scale, v[1].im * inv_scale};
    __builtin_nontemporal_store(__builtin_convertvector(f, h), reinterpret_cast<h *>(p) + u * vs + s);
}

// FP64 complex entry c of an FP64 spinor (double2 planes)
__device__ __forceinline__ cpx<double> ld64(const double2 *p, size_t vs, int c, int s) {
    const double2 t = p[c * vs + s];
    return {t.x, t.y};
}
__device__ __forceinline__ void st64(double2 *p, size_t vs, int c, int s, cpx<double> v) {
    p[c * vs + s] = make_double2(v.re, v.im);
}

__device__ __forceinline__ void block_partial(double v, double *partial, size_t idx) {
    __shared__ double lds[kBlock / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) t += lds[i];
        partial[idx] = t;
    }
}

// Entry c of the source of a slot at site s.
__device__ __forceinline__ cpx<double> source_entry(const Source &src, int slot, int c, int s, size_t vs) {
    cpx<double> v;
    if (src.b) {
        v = ld64(src.b + (size_t)slot * 12 * vs, vs, c, s);
    } else {
        const bool on = (src.colour[s] == src.slot_class[slot]) && (c == src.slot_comp[slot]);
        v = {on ? 1.0 : 0.0, 0.0};
    }
    // deflated modes projected out: b - sum_i <u_i, b> u_i
    for (int i = 0; i < src.dk; ++i) {
        const double2 a = src.dcoef[(size_t)slot * src.dk + i];
        const cpx<double> u = ld64(src.du + (size_t)i * 12 * vs, vs, c, s);
        v.re -= a.x * u.re - a.y * u.im;
        v.im -= a.x * u.im + a.y * u.re;
    }
    return v;
}

int unit_parts(int prec, const Geom &g) { return (prec == 0 ? 12 : 6) * site_blocks(g); }

// r = b, p_i = b for every shift, y = c0 b (FP64), running accumulators yacc = x0acc = 0 in the
// iteration precision (FP32 path only; the FP64 path accumulates into y directly and has no x0);
// partial = |b|^2 per block.
template <class T, int D>
__global__ __launch_bounds__(kBlock) void k_cg_init(Geom g, Source src, int NS, double c0,
                                                    typename Store<T>::vec *r, typename Store<T>::vec *p, double2 *y,
                                                    typename Store<T>::vec *yacc, double2 *x0,
                                                    typename Store<T>::vec *x0acc, double *partial, size_t pstride) {
    constexpr int C = Unit<T>::C;
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    const size_t rs = Store<T>::units * g.vs;
    double nrm = 0.0;
    if (s < g.V) {
        cpx<T> bt[C], z[C];
        double2 *ys = y + (size_t)slot * 12 * g.vs;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int c = u * C + i;
            const cpx<double> b = source_entry(src, slot, c, s, g.vs);
            bt[i] = {(T)b.re, (T)b.im};
            z[i] = {T(0), T(0)};
            nrm += (double)bt[i].re * bt[i].re + (double)bt[i].im * bt[i].im;
            st64(ys, g.vs, c, s, c0 * b);
            if (x0) st64(x0 + (size_t)slot * 12 * g.vs, g.vs, c, s, {0.0, 0.0});
        }
        Unit<T>::store(r + slot * rs, g.vs, u, s, bt);
        if constexpr (D == kDirF32) {
            for (int i = 0; i < NS; ++i) Unit<T>::store(p + ((size_t)slot * NS + i) * rs, g.vs, u, s, bt);
        } else {
            // the base direction; the 16-bit ones follow from r once |b| is known (k_dir16_init)
            Unit<T>::store(p + slot * rs, g.vs, u, s, bt);
        }
        if (yacc) Unit<T>::store(yacc + slot * rs, g.vs, u, s, z);
        if (x0acc) Unit<T>::store(x0acc + slot * rs, g.vs, u, s, z);
    }
    block_partial(nrm, partial, (size_t)slot * pstride + blockIdx.x);
}

void launch_cg_init(int prec, const Geom &g, const Source &src, int nslots, int NS, double c0, void *r, void *p,
                    double2 *y, void *yacc, double2 *x0, void *x0acc, double *partial, int dir, hipStream_t st) {
    dim3 grid(unit_parts(prec, g), nslots);
    if (prec == 0) {
        if (dir != kDirF32) throw std::invalid_argument("16-bit directions need the FP32 path");
        hipLaunchKernelGGL((k_cg_init<double, kDirF32>), grid, dim3(kBlock), 0, st, g, src, NS, c0, (double2 *)r,
                           (double2 *)p, y, (double2 *)yacc, x0, (double2 *)x0acc, partial, partial_stride(g));
        return;
    }
    if (dir == kDirF32)
        hipLaunchKernelGGL((k_cg_init<float, kDirF32>), grid, dim3(kBlock), 0, st, g, src, NS, c0, (float4 *)r,
                           (float4 *)p, y, (float4 *)yacc, x0, (float4 *)x0acc, partial, partial_stride(g));
    else   // only the base direction's layout depends on the 16-bit format
        hipLaunchKernelGGL((k_cg_init<float, kDirF16>), grid, dim3(kBlock), 0, st, g, src, NS, c0, (float4 *)r,
                           (float4 *)p, y, (float4 *)yacc, x0, (float4 *)x0acc, partial, partial_stride(g));
}

// 16-bit directions: p_i = b = r for every shift but the base, stored with the scale that
// k_scalars_init set from |b| (so that the entries of any source are near 1).
template <int D>
__global__ __launch_bounds__(kBlock) void k_dir16_init(Geom g, MSState S, const float4 *r, void *ph) {
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t rs = Store<float>::units * g.vs;
    cpx<float> v[2];
    Unit<float>::load(r + slot * rs, g.vs, u, s, v);
    for (int i = 0; i < S.NS; ++i)
        if (i != S.i0)
            store_dir16<D>(static_cast<typename Dir16<D>::v *>(ph) + ((size_t)slot * S.NS + i) * rs, g.vs, u, s,
                           (float)(1.0 / S.sh_scale[slot * S.NS + i]), v);
}

void launch_dir16_init(const Geom &g, const MSState &s, int nslots, const void *r, int dir, void *ph, hipStream_t st) {
    dim3 grid(unit_parts(1, g), nslots);
    if (dir == kDirF16)
        hipLaunchKernelGGL(k_dir16_init<kDirF16>, grid, dim3(kBlock), 0, st, g, s, (const float4 *)r, ph);
    else if (dir == kDirBF16)
        hipLaunchKernelGGL(k_dir16_init<kDirBF16>, grid, dim3(kBlock), 0, st, g, s, (const float4 *)r, ph);
    else
        throw std::invalid_argument("launch_dir16_init: not a 16-bit format");
}

// ------------------------------------------------------------------ CG scalars (one wave per slot)
// Slots >= nslots are not part of this batch and start finished.
__global__ void k_scalars_init(MSState S, int npart, int nslots) {
    const int slot = blockIdx.x;
    const double rr = slot < nslots ? wave_sum_partials(S.partial + (size_t)slot * S.pstride, npart) : 0.0;
    if (threadIdx.x != 0) return;
    S.rr[slot] = rr;
    S.bnorm[slot] = sqrt(rr);
    S.alpha_prev[slot] = 1.0;
    S.beta_prev[slot] = 0.0;
    S.alpha[slot] = 0.0;
    for (int i = 0; i < S.NS; ++i) {
        const int k = slot * S.NS + i;
        S.zeta[k] = 1.0;
        S.zeta_prev[k] = 1.0;
        S.zeta_new[k] = 1.0;
        S.sh_active[k] = rr > 0.0;
        S.sh_iters[k] = 0;
        S.sh_scale[k] = rr > 0.0 ? sqrt(rr) * S.dir_norm : 1.0;
    }
    S.done[slot] = !(rr > 0.0);
    S.iters[slot] = 0;
    S.status[slot] = kStatusOK;
    S.upd_n[slot] = 0;
    S.cnt_entries[slot] = 0;
    S.cnt_pupd[slot] = 0;
    S.cnt_active[slot] = 0;
    S.cnt_base_pupd[slot] = 0;
}

void launch_scalars_init(const MSState &s, int npart, int nslots, hipStream_t st) {
    hipLaunchKernelGGL(k_scalars_init, dim3(s.B), dim3(64), 0, st, s, npart, nslots);
}

// alpha_k = |r_k|^2 / <p_k, A p_k>; for each active shift the new zeta.
__global__ void k_scalars_alpha(MSState S, int npart) {
    if ((int)blockIdx.x >= *S.count) return;
    const int slot = S.list[blockIdx.x];
    const double pap = wave_sum_partials(S.partial + (size_t)slot * S.pstride, npart);
    if (threadIdx.x != 0) return;
    if (!(pap > 0.0) || !isfinite(pap)) {
        S.status[slot] = kStatusBreakdown;
        S.alpha[slot] = 0.0;
        return;
    }
    const double a = S.rr[slot] / pap;
    const double ap = S.alpha_prev[slot], bp = S.beta_prev[slot];
    S.alpha[slot] = a;
    for (int i = 0; i < S.NS; ++i) {
        const int k = slot * S.NS + i;
        if (!S.sh_active[k]) continue;
        const double z = S.zeta[k], zp = S.zeta_prev[k];
        S.zeta_new[k] = z * zp * ap / (a * bp * (zp - z) + zp * ap * (1.0 + S.delta[i] * a));
    }
}

void launch_scalars_alpha(const MSState &s, int npart, hipStream_t st) {
    hipLaunchKernelGGL(k_scalars_alpha, dim3(s.B), dim3(64), 0, st, s, npart);
}

// beta_k = |r_{k+1}|^2/|r_k|^2; per active shift: alpha^i, beta^i, convergence
// (zeta^i_{k+1} |r_{k+1}| <= tol |b|); build this iteration's update list.  The base
// shift's direction keeps being updated while any shift of the slot is active.
__global__ void k_scalars_beta(MSState S, int npart) {
    if ((int)blockIdx.x >= *S.count) return;
    const int slot = S.list[blockIdx.x];
    const double rrn = wave_sum_partials(S.partial + (size_t)slot * S.pstride, npart);
    if (threadIdx.x != 0) return;
    if (S.status[slot] != kStatusOK) {
        S.done[slot] = 1;
        S.upd_n[slot] = 0;
        return;
    }
    const double a = S.alpha[slot];
    const double b = rrn / S.rr[slot];
    const double rn = sqrt(rrn);
    const double lim = S.tol * S.bnorm[slot];
    const int it = S.iters[slot];
    int n = 0, still = 0, npupd = 0;
    for (int i = 0; i < S.NS; ++i) {
        const int k = slot * S.NS + i;
        const int u = slot * S.NS + n;
        if (S.sh_active[k]) {
            const double z = S.zeta[k], zn = S.zeta_new[k];
            const double ratio = zn / z;
            const bool conv = zn * rn <= lim;
            S.upd_idx[u] = i;
            S.upd_cy[u] = S.c[i] * a * ratio;
            S.upd_ax[u] = a * ratio;
            S.upd_zeta[u] = zn;
            S.upd_beta[u] = b * ratio * ratio;
            S.upd_pupd[u] = (!conv || i == S.i0) ? 1 : 0;
            ++n;
            if (conv) {
                S.sh_active[k] = 0;
                S.sh_iters[k] = it + 1;
            } else {
                ++still;
            }
            S.zeta_prev[k] = z;
            S.zeta[k] = zn;
        } else if (i == S.i0) {
            S.upd_idx[u] = i;
            S.upd_cy[u] = 0.0;
            S.upd_ax[u] = 0.0;
            S.upd_zeta[u] = 1.0;
            S.upd_beta[u] = b;
            S.upd_pupd[u] = 1;
            ++n;
        }
    }
    if (still == 0) {  // slot finished: no direction needs updating any more
        for (int e = 0; e < n; ++e) S.upd_pupd[slot * S.NS + e] = 0;
        S.done[slot] = 1;
    }
    // 16-bit directions: the stored p_i is decoded with its current scale and the new one is
    // stored divided by zeta^i_{k+1} |r_{k+1}| dir_norm, which keeps its entries near 1
    for (int e = 0; e < n; ++e) {
        const int u = slot * S.NS + e;
        const int k = slot * S.NS + S.upd_idx[u];
        S.upd_sold[u] = S.sh_scale[k];
        if (S.upd_pupd[u]) {
            double sc = S.upd_zeta[u] * rn * S.dir_norm;
            if (!(sc > 0.0) || !isfinite(sc)) sc = S.sh_scale[k];
            S.sh_scale[k] = sc;
            S.upd_snew[u] = 1.0 / sc;
            npupd++;
            if (S.upd_idx[u] == S.i0) S.cnt_base_pupd[slot] += 1;
        } else {
            S.upd_snew[u] = 1.0;
        }
    }
    S.upd_n[slot] = n;
    S.cnt_entries[slot] += n;
    S.cnt_pupd[slot] += npupd;
    S.cnt_active[slot] += 1;
    S.alpha_prev[slot] = a;
    S.beta_prev[slot] = b;
    S.rr[slot] = rrn;
    S.iters[slot] = it + 1;
}

void launch_scalars_beta(const MSState &s, int npart, hipStream_t st) {
    hipLaunchKernelGGL(k_scalars_beta, dim3(s.B), dim3(64), 0, st, s, npart);
}

// For every entry of the slot's update list: y += c_i alpha^i p_i (old p_i), then
// p_i = zeta^i r + beta^i p_i; x0 += alpha p_base where an x0 target is given (FP32 path).
// The sums go either straight into the FP64 vectors (Y64 / X64) or into running sums in the
// storage precision of p, which k_fold adds to FP64 every few iterations.  The FP64 path
// always accumulates into y directly.  D: storage of the shifted directions (kDirF32: all NS
// directions in p; 16-bit: the base in p, slot stride one vector, the others scaled in ph).
// XS: also x_i += alpha^i p_i in FP64 for every listed shift (xs [slot][NS][12][vs]).
template <class T, bool Y64, bool X64, int D, bool XS>
__global__ __launch_bounds__(kBlock) void k_shift_update(Geom g, MSState S, const typename Store<T>::vec *r,
                                                         typename Store<T>::vec *p, void *yt, void *xt, void *ph,
                                                         double2 *xs) {
    using vec = typename Store<T>::vec;
    constexpr int C = Unit<T>::C;
    if ((int)blockIdx.y >= *S.count) return;
    const int slot = S.list[blockIdx.y];
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const int n = S.upd_n[slot];
    if (n == 0) return;
    const size_t rs = Store<T>::units * g.vs, r64 = 12 * g.vs;
    cpx<T> rv[C];
    Unit<T>::load_stream(r + slot * rs, g.vs, u, s, rv);
    cpx<double> y64[C], x64[C];
    cpx<T> yl[C], xl[C];
    if constexpr (Y64) {
#pragma unroll
        for (int j = 0; j < C; ++j) y64[j] = ld64_stream((double2 *)yt + slot * r64, g.vs, u * C + j, s);
    } else {
        Unit<T>::load_stream((vec *)yt + slot * rs, g.vs, u, s, yl);
    }
    bool x_touched = false;
#pragma unroll 1
    for (int e = 0; e < n; ++e) {
        const int k = slot * S.NS + e;
        const int i = S.upd_idx[k];
        const double cy = S.upd_cy[k];
        const bool full = D == kDirF32 || i == S.i0;   // this direction is stored in T
        vec *pp = D == kDirF32 ? p + ((size_t)slot * S.NS + i) * rs : p + slot * rs;
        cpx<T> pv[C];
        if constexpr (D == kDirF32) {
            Unit<T>::load_stream(pp, g.vs, u, s, pv);
        } else {
            if (full) Unit<T>::load_stream(pp, g.vs, u, s, pv);
            else load_dir16<D>(static_cast<typename Dir16<D>::v *>(ph) + ((size_t)slot * S.NS + i) * rs, g.vs, u, s,
                               (float)S.upd_sold[k], pv);
        }
        if constexpr (XS) {
            const double ax = S.upd_ax[k];
            if (ax != 0.0) {
                double2 *xp = xs + ((size_t)slot * S.NS + i) * r64;
#pragma unroll
                for (int j = 0; j < C; ++j)
                    st64_stream(xp, g.vs, u * C + j, s,
                                ld64_stream(xp, g.vs, u * C + j, s) + ax * cpx<double>{(double)pv[j].re, (double)pv[j].im});
            }
        }
        if (cy != 0.0) {
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if constexpr (Y64) y64[j] = y64[j] + cy * cpx<double>{(double)pv[j].re, (double)pv[j].im};
                else yl[j] = yl[j] + (T)cy * pv[j];
            }
            if (xt && i == S.i0) {
                const double a = S.alpha[slot];
                x_touched = true;
                if constexpr (X64) {
#pragma unroll
                    for (int j = 0; j < C; ++j)
                        x64[j] = ld64_stream((double2 *)xt + slot * r64, g.vs, u * C + j, s) +
                                 a * cpx<double>{(double)pv[j].re, (double)pv[j].im};
                } else {
                    Unit<T>::load_stream((vec *)xt + slot * rs, g.vs, u, s, xl);
#pragma unroll
                    for (int j = 0; j < C; ++j) xl[j] = xl[j] + (T)a * pv[j];
                }
            }
        }
        if (S.upd_pupd[k]) {
            const T zn = (T)S.upd_zeta[k], bi = (T)S.upd_beta[k];
#pragma unroll
            for (int j = 0; j < C; ++j) pv[j] = zn * rv[j] + bi * pv[j];
            if constexpr (D == kDirF32) {
                Unit<T>::store_stream(pp, g.vs, u, s, pv);
            } else {
                if (full) Unit<T>::store_stream(pp, g.vs, u, s, pv);
                else store_dir16<D>(static_cast<typename Dir16<D>::v *>(ph) + ((size_t)slot * S.NS + i) * rs, g.vs,
                                    u, s, (float)S.upd_snew[k], pv);
            }
        }
    }
    if constexpr (Y64) {
#pragma unroll
        for (int j = 0; j < C; ++j) st64_stream((double2 *)yt + slot * r64, g.vs, u * C + j, s, y64[j]);
    } else {
        Unit<T>::store_stream((vec *)yt + slot * rs, g.vs, u, s, yl);
    }
    if (x_touched) {
        if constexpr (X64) {
#pragma unroll
            for (int j = 0; j < C; ++j) st64_stream((double2 *)xt + slot * r64, g.vs, u * C + j, s, x64[j]);
        } else {
            Unit<T>::store_stream((vec *)xt + slot * rs, g.vs, u, s, xl);
        }
    }
}

void launch_shift_update(int prec, const Geom &g, const MSState &s, const void *r, void *p, void *yt, bool y64,
                         void *xt, bool x64, int dir, void *ph, double2 *xs, hipStream_t st) {
    dim3 grid(unit_parts(prec, g), s.B);
    if (xs && dir != kDirF32) throw std::invalid_argument("the per-shift check needs FP32 or FP64 directions");
    if (prec == 0) {
        if (dir != kDirF32) throw std::invalid_argument("16-bit directions need the FP32 path");
        if (xs)
            hipLaunchKernelGGL((k_shift_update<double, true, true, kDirF32, true>), grid, dim3(kBlock), 0, st, g, s,
                               (const double2 *)r, (double2 *)p, yt, xt, ph, xs);
        else
            hipLaunchKernelGGL((k_shift_update<double, true, true, kDirF32, false>), grid, dim3(kBlock), 0, st, g, s,
                               (const double2 *)r, (double2 *)p, yt, xt, ph, xs);
        return;
    }
#define SMPQ_SU(Y, X, D, XS)                                                                                      \
    hipLaunchKernelGGL((k_shift_update<float, Y, X, D, XS>), grid, dim3(kBlock), 0, st, g, s, (const float4 *)r,   \
                       (float4 *)p, yt, xt, ph, xs)
#define SMPQ_SU_D(D, XS)                         \
    if (y64 && x64) SMPQ_SU(true, true, D, XS);  \
    else if (y64) SMPQ_SU(true, false, D, XS);   \
    else if (x64) SMPQ_SU(false, true, D, XS);   \
    else SMPQ_SU(false, false, D, XS)
    if (dir == kDirF16) {
        SMPQ_SU_D(kDirF16, false);
    } else if (dir == kDirBF16) {
        SMPQ_SU_D(kDirBF16, false);
    } else if (xs) {
        SMPQ_SU_D(kDirF32, true);
    } else {
        SMPQ_SU_D(kDirF32, false);
    }
#undef SMPQ_SU_D
#undef SMPQ_SU
}

// FP32 path: y += yacc, yacc = 0 when y is given, and x0 += x0acc, x0acc = 0 when x0acc is
// given, for the listed slots, in FP64.
__global__ __launch_bounds__(kBlock) void k_fold(Geom g, Slots sl, double2 *y, float4 *yacc, double2 *x0,
                                                 float4 *x0acc) {
    if ((int)blockIdx.y >= slot_count(sl)) return;
    const int slot = slot_of(sl, blockIdx.y);
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t rs = 6 * g.vs, ys = 12 * g.vs;
    const cpx<float> z[2] = {{0.f, 0.f}, {0.f, 0.f}};
    cpx<float> a[2];
    if (y) {
        Unit<float>::load_stream(yacc + slot * rs, g.vs, u, s, a);
        double2 *yp = y + slot * ys;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            st64_stream(yp, g.vs, 2 * u + j, s,
                        ld64_stream(yp, g.vs, 2 * u + j, s) + cpx<double>{(double)a[j].re, (double)a[j].im});
        Unit<float>::store_stream(yacc + slot * rs, g.vs, u, s, z);
    }
    if (x0acc) {
        Unit<float>::load_stream(x0acc + slot * rs, g.vs, u, s, a);
        double2 *xp = x0 + slot * ys;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            st64_stream(xp, g.vs, 2 * u + j, s, ld64_stream(xp, g.vs, 2 * u + j, s) + cpx<double>{(double)a[j].re, (double)a[j].im});
        Unit<float>::store_stream(x0acc + slot * rs, g.vs, u, s, z);
    }
}

void launch_fold(const Geom &g, Slots sl, int max_slots, double2 *y, void *yacc, double2 *x0, void *x0acc,
                 hipStream_t st) {
    dim3 grid(unit_parts(1, g), max_slots);
    hipLaunchKernelGGL(k_fold, grid, dim3(kBlock), 0, st, g, sl, y, (float4 *)yacc, x0, (float4 *)x0acc);
}

// Evaluated precision: an FP32 vector of every listed slot rounded in place to what 16-bit
// storage would hold, FP16 after division by the slot's scale sqrt(|r|^2 / (24 V)) (entries of
// a vector of norm ~|r| then lie near 1) or BF16 (FP32's exponent range); round to nearest
// even.  Applied to the vectors the stencil reads (the base direction and D_W p) after the
// kernels that write them, so that those compute in FP32 and only storage is emulated.
__global__ __launch_bounds__(kBlock) void k_round16(Geom g, MSState S, float4 *v, size_t slot_stride, size_t extra,
                                                    int mode) {
    if ((int)blockIdx.y >= *S.count) return;
    const int slot = S.list[blockIdx.y];
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    float4 *p = v + slot * slot_stride + extra + (size_t)u * g.vs + s;
    const float scale = mode == 1 ? (float)sqrt(S.rr[slot] / (24.0 * (double)g.V)) : 1.f;
    const float sc = scale > 0.f ? scale : 1.f, inv = 1.f / sc;
    const float4 t = *p;
    float x[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = mode == 1 ? (float)(_Float16)(x[i] * inv) * sc : (float)(__bf16)x[i];
    *p = make_float4(x[0], x[1], x[2], x[3]);
}

void launch_round16(const Geom &g, const MSState &s, void *v, size_t slot_stride, size_t extra, int mode,
                    hipStream_t st) {
    dim3 grid(unit_parts(1, g), s.B);
    hipLaunchKernelGGL(k_round16, grid, dim3(kBlock), 0, st, g, s, (float4 *)v, slot_stride, extra, mode);
}

// Ordered list of the slots still iterating.
__global__ void k_compact(MSState S) {
    if (threadIdx.x != 0) return;
    int n = 0;
    for (int slot = 0; slot < S.B; ++slot)
        if (!S.done[slot]) S.list[n++] = slot;
    *S.count = n;
}

void launch_compact(const MSState &s, hipStream_t st) { hipLaunchKernelGGL(k_compact, dim3(1), dim3(64), 0, st, s); }

// Residual replacement: r = b - (H^2 + s) x0 evaluated in FP64 (ap64 holds (H^2 + s) x0),
// stored in the iteration precision; partial |r|^2 of the stored values.
template <class T>
__global__ __launch_bounds__(kBlock) void k_reliable(Geom g, MSState S, Source src, const double2 *ap64,
                                                     typename Store<T>::vec *r) {
    constexpr int C = Unit<T>::C;
    if ((int)blockIdx.y >= *S.count) return;
    const int slot = S.list[blockIdx.y];
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    const size_t rs = Store<T>::units * g.vs;
    double nrm = 0.0;
    if (s < g.V) {
        cpx<T> rv[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int c = u * C + i;
            const cpx<double> d = source_entry(src, slot, c, s, g.vs) - ld64(ap64 + (size_t)slot * 12 * g.vs, g.vs, c, s);
            rv[i] = {(T)d.re, (T)d.im};
            nrm += (double)rv[i].re * rv[i].re + (double)rv[i].im * rv[i].im;
        }
        Unit<T>::store(r + slot * rs, g.vs, u, s, rv);
    }
    block_partial(nrm, S.partial, (size_t)slot * S.pstride + blockIdx.x);
}

void launch_reliable(int prec, const Geom &g, const MSState &s, const Source &src, const double2 *ap64, void *r,
                     hipStream_t st) {
    dim3 grid(unit_parts(prec, g), s.B);
    if (prec == 0)
        hipLaunchKernelGGL(k_reliable<double>, grid, dim3(kBlock), 0, st, g, s, src, ap64, (double2 *)r);
    else
        hipLaunchKernelGGL(k_reliable<float>, grid, dim3(kBlock), 0, st, g, s, src, ap64, (float4 *)r);
}

__global__ void k_scalars_rr(MSState S, int npart) {
    if ((int)blockIdx.x >= *S.count) return;
    const int slot = S.list[blockIdx.x];
    const double rr = wave_sum_partials(S.partial + (size_t)slot * S.pstride, npart);
    if (threadIdx.x == 0) S.rr[slot] = rr;
}

void launch_scalars_rr(const MSState &s, int npart, hipStream_t st) {
    hipLaunchKernelGGL(k_scalars_rr, dim3(s.B), dim3(64), 0, st, s, npart);
}

// ------------------------------------------------------------------ per-shift check
// out = b - ap64 in FP64 for the first nslots slots; partial |out|^2 per block.
__global__ __launch_bounds__(kBlock) void k_resid64(Geom g, Source src, const double2 *ap64, double2 *out,
                                                    double *partial, size_t pstride) {
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    double nrm = 0.0;
    if (s < g.V) {
        const size_t o = (size_t)slot * 12 * g.vs;
        const cpx<double> d = source_entry(src, slot, u, s, g.vs) - ld64(ap64 + o, g.vs, u, s);
        st64(out + o, g.vs, u, s, d);
        nrm = d.re * d.re + d.im * d.im;
    }
    block_partial(nrm, partial, (size_t)slot * pstride + blockIdx.x);
}

void launch_resid64(const Geom &g, int nslots, const Source &src, const double2 *ap64, double2 *out,
                    double *partial, size_t pstride, hipStream_t st) {
    hipLaunchKernelGGL(k_resid64, dim3(unit_parts(0, g), nslots), dim3(kBlock), 0, st, g, src, ap64, out, partial,
                       pstride);
}

__global__ void k_slot_sums(const double *partial, size_t pstride, int npart, double *sums) {
    const double v = wave_sum_partials(partial + (size_t)blockIdx.x * pstride, npart);
    if (threadIdx.x == 0) sums[blockIdx.x] = v;
}

void launch_slot_sums(int nslots, const double *partial, size_t pstride, int npart, double *sums, hipStream_t st) {
    hipLaunchKernelGGL(k_slot_sums, dim3(nslots), dim3(64), 0, st, partial, pstride, npart, sums);
}

__global__ __launch_bounds__(kBlock) void k_zero_unflagged(Geom g, const int *flag, double2 *v) {
    const int slot = blockIdx.y;
    if (flag[slot]) return;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s < g.V) st64(v + (size_t)slot * 12 * g.vs, g.vs, u, s, {0.0, 0.0});
}

void launch_zero_unflagged(const Geom &g, int nslots, const int *flag, double2 *v, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_unflagged, dim3(unit_parts(0, g), nslots), dim3(kBlock), 0, st, g, flag, v);
}

__global__ __launch_bounds__(kBlock) void k_refine_acc(Geom g, const double2 *e, double c, double2 *ysave,
                                                       double2 *xsi, size_t xs_stride) {
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t o = (size_t)slot * 12 * g.vs;
    const cpx<double> ev = ld64(e + o, g.vs, u, s);
    st64(ysave + o, g.vs, u, s, ld64(ysave + o, g.vs, u, s) + c * ev);
    double2 *xp = xsi + (size_t)slot * xs_stride;
    st64(xp, g.vs, u, s, ld64(xp, g.vs, u, s) + ev);
}

void launch_refine_acc(const Geom &g, int nslots, const double2 *e, double c, double2 *ysave, double2 *xsi,
                       size_t xs_stride, hipStream_t st) {
    hipLaunchKernelGGL(k_refine_acc, dim3(unit_parts(0, g), nslots), dim3(kBlock), 0, st, g, e, c, ysave, xsi,
                       xs_stride);
}

// ------------------------------------------------------------------ contraction (Eq. 16)
// For each probed site x of class position ci and each component j (slot 12 ci + j):
//   q(x)  += 1/2 gamma5_jj (1 + Re[D_W y_slot](x, j)),   qi(x) += 1/2 gamma5_jj Im[D_W y_slot](x, j),
// since gamma5 D_ov phi = gamma5 (phi + D_W y) with eps phi = gamma5 D_W y.
// INV (trace of D_W^-1): y_slot = (D_W^dag D_W)^-1 phi and D_W^-1 phi = g_j gamma5 D_W y_slot
// (from D_W^-1 = D_W^dag (D_W D_W^dag)^-1, D_W D_W^dag = gamma5 D_W^dag D_W gamma5 and
// gamma5 phi = g_j phi), so component j of D_W^-1 phi at x is [D_W y_slot](x, j):
//   t(x) += [D_W y_slot](x, j)  (real part into qx, imaginary part into qxi).
// With deflated modes (dk > 0), eps phi gains sum_i c_i w_i (w_i = H u_i / sqrt(theta_i),
// c_i = <u_i, phi>), which adds 1/2 sum_i c_i w_i(x, j) to [gamma5 D_ov phi](x, j) / 2.
template <bool INV>
__global__ __launch_bounds__(kBlock) void k_contract(Geom g, const double2 *U64, const double2 *y, double kappa,
                                                     const int *batch_classes, const int *class_ptr,
                                                     const int *class_sites, double *qx, double *qxi,
                                                     const double2 *dw, const double2 *dcoef, int dk) {
    const int ci = blockIdx.y;
    const int cls = batch_classes[ci];
    const int beg = class_ptr[cls], end = class_ptr[cls + 1];
    const int k = beg + blockIdx.x * kBlock + threadIdx.x;
    if (k >= end) return;
    const int x = class_sites[k];
    double q = 0.0, qi = 0.0;
#pragma unroll 1
    for (int j = 0; j < 12; ++j) {
        const double2 *yv = y + (size_t)(12 * ci + j) * 12 * g.vs;
        cpx<double> acc[12];
        hop_site<double, 1>(U64, g, yv, x, acc);
        const cpx<double> self = ld64(yv, g.vs, j, x);
        const double dre = self.re - kappa * acc[j].re;
        const double dim = self.im - kappa * acc[j].im;
        if constexpr (INV) {
            q += dre;
            qi += dim;
        } else {
            const double g5 = (j < 6) ? 0.5 : -0.5;
            q += g5 * (1.0 + dre);
            qi += g5 * dim;
            const int slot = 12 * ci + j;
            for (int i = 0; i < dk; ++i) {
                const double2 a = dcoef[(size_t)slot * dk + i];
                const cpx<double> w = ld64(dw + (size_t)i * 12 * g.vs, g.vs, j, x);
                q += 0.5 * (a.x * w.re - a.y * w.im);
                qi += 0.5 * (a.x * w.im + a.y * w.re);
            }
        }
    }
    qx[x] = q;
    qxi[x] = qi;
}

void launch_contract(const Geom &g, const double2 *U64, const double2 *y, double kappa, const int *batch_classes,
                     int n_classes, int max_class_size, const int *class_ptr, const int *class_sites, double *qx,
                     double *qxi, bool inverse, const double2 *dw, const double2 *dcoef, int dk, hipStream_t st) {
    dim3 grid((max_class_size + kBlock - 1) / kBlock, n_classes);
    if (inverse)
        hipLaunchKernelGGL(k_contract<true>, grid, dim3(kBlock), 0, st, g, U64, y, kappa, batch_classes, class_ptr,
                           class_sites, qx, qxi, nullptr, nullptr, 0);
    else
        hipLaunchKernelGGL(k_contract<false>, grid, dim3(kBlock), 0, st, g, U64, y, kappa, batch_classes, class_ptr,
                           class_sites, qx, qxi, dw, dcoef, dk);
}

// ------------------------------------------------------------------ locality of D_ov (Eq. 12)
// d holds D_W y_j for the twelve point-source columns j of site `site` (slot stride 12 vs);
// column j of D_ov is e_{site,j} + d_j.  m(x) = (1/144) sum_{i,j} |D_ov(x i; site j)|.
__global__ __launch_bounds__(kBlock) void k_block_mean_abs(Geom g, const double2 *d, int site, double *m) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= g.V) return;
    double acc = 0.0;
#pragma unroll 1
    for (int j = 0; j < 12; ++j) {
        const double2 *col = d + (size_t)j * 12 * g.vs;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            cpx<double> v = ld64(col, g.vs, i, x);
            if (x == site && i == j) v.re += 1.0;
            acc += sqrt(v.re * v.re + v.im * v.im);
        }
    }
    m[x] = acc / 144.0;
}

void launch_block_mean_abs(const Geom &g, const double2 *d, int site, double *m, hipStream_t st) {
    hipLaunchKernelGGL(k_block_mean_abs, dim3((g.V + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g, d, site, m);
}

// ------------------------------------------------------------------ Lanczos helpers (FP64, one vector)
__global__ __launch_bounds__(kBlock) void k_lanczos_update(Geom g, double2 *w, const double2 *v, const double2 *vprev,
                                                           double alpha, double beta, double *partial) {
    const int nsb = site_blocks(g);
    const int c = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    double nrm = 0.0;
    if (s < g.V) {
        const size_t i = c * g.vs + s;
        double2 t = w[i];
        const double2 a = v[i], b = vprev[i];
        t.x -= alpha * a.x + beta * b.x;
        t.y -= alpha * a.y + beta * b.y;
        w[i] = t;
        nrm = t.x * t.x + t.y * t.y;
    }
    block_partial(nrm, partial, blockIdx.x);
}

void launch_lanczos_update(const Geom &g, double2 *w, const double2 *v, const double2 *vprev, double alpha,
                           double beta, double *partial, hipStream_t st) {
    hipLaunchKernelGGL(k_lanczos_update, dim3(unit_parts(0, g)), dim3(kBlock), 0, st, g, w, v, vprev, alpha, beta,
                       partial);
}

__global__ __launch_bounds__(kBlock) void k_scale(Geom g, double2 *dst, const double2 *src, double f) {
    const int nsb = site_blocks(g);
    const int c = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const double2 t = src[c * g.vs + s];
    dst[c * g.vs + s] = make_double2(f * t.x, f * t.y);
}

void launch_scale(const Geom &g, double2 *dst, const double2 *src, double f, hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(unit_parts(0, g)), dim3(kBlock), 0, st, g, dst, src, f);
}

// ------------------------------------------------------------------ low-mode deflation (FP64)
// Complex block sum of (re, im) written to partial[idx] and partial[idx + stride].
__device__ __forceinline__ void block_partial_c(double re, double im, double *partial, size_t idx, size_t stride) {
    __shared__ double lds[2][kBlock / 64];
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = re;
        lds[1][threadIdx.x >> 6] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) {
            a += lds[0][i];
            b += lds[1][i];
        }
        partial[idx] = a;
        partial[idx + stride] = b;
    }
}

// partial[(2 i + {0,1}) np + block] = Re, Im of the block's share of <q_i, w>, i < nq,
// q_i = Q + i qstride; grid (np = unit_parts(0, g), nq).
__global__ __launch_bounds__(kBlock) void k_multi_dot(Geom g, const double2 *Q, size_t qstride, const double2 *w,
                                                      double *partial) {
    const int nsb = site_blocks(g);
    const int np = gridDim.x;
    const int c = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    const int i = blockIdx.y;
    double re = 0.0, im = 0.0;
    if (s < g.V) {
        const double2 q = Q[(size_t)i * qstride + c * g.vs + s], x = w[c * g.vs + s];
        re = q.x * x.x + q.y * x.y;
        im = q.x * x.y - q.y * x.x;
    }
    block_partial_c(re, im, partial, (size_t)(2 * i) * np + blockIdx.x, np);
}

// out[i] = sum of the np partials of pair i, in a fixed order (one wave per i).
__global__ void k_reduce_pairs(const double *partial, int np, double2 *out) {
    const int i = blockIdx.x;
    const double re = wave_sum_partials(partial + (size_t)(2 * i) * np, np);
    const double im = wave_sum_partials(partial + (size_t)(2 * i + 1) * np, np);
    if (threadIdx.x == 0) out[i] = make_double2(re, im);
}

// w -= sum_{i < nq} h_i q_i, or w = sum_{i < nq} h_i q_i when overwrite is set.
__global__ __launch_bounds__(kBlock) void k_multi_axpy(Geom g, const double2 *Q, size_t qstride, int nq,
                                                       const double2 *h, double2 *w, int overwrite) {
    const int nsb = site_blocks(g);
    const int c = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t o = c * g.vs + s;
    double ar = 0.0, ai = 0.0;
#pragma unroll 4
    for (int i = 0; i < nq; ++i) {
        const double2 q = Q[(size_t)i * qstride + o], hh = h[i];
        ar += hh.x * q.x - hh.y * q.y;
        ai += hh.x * q.y + hh.y * q.x;
    }
    if (overwrite) {
        w[o] = make_double2(ar, ai);
    } else {
        const double2 t = w[o];
        w[o] = make_double2(t.x - ar, t.y - ai);
    }
}

// v = f gamma5 v (gamma5 = +1 on spins 0, 1 and -1 on spins 2, 3; component c = 3 spin + colour).
__global__ __launch_bounds__(kBlock) void k_g5_scale(Geom g, double2 *v, double f) {
    const int nsb = site_blocks(g);
    const int c = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const double ff = c < 6 ? f : -f;
    const double2 t = v[c * g.vs + s];
    v[c * g.vs + s] = make_double2(ff * t.x, ff * t.y);
}

// Deflation coefficients of probing sources: coef[slot k + i] = <u_i, phi_slot> = sum over the
// sites x of the slot's class of conj(u_i(x, comp)); grid (k, nslots).
__global__ __launch_bounds__(kBlock) void k_defl_coef_probe(Geom g, const double2 *u, int k, const int *slot_class,
                                                            const int *slot_comp, const int *class_ptr,
                                                            const int *class_sites, double2 *coef) {
    const int i = blockIdx.x, slot = blockIdx.y;
    const int cls = slot_class[slot], comp = slot_comp[slot];
    const double2 *ui = u + (size_t)i * 12 * g.vs + comp * g.vs;
    double re = 0.0, im = 0.0;
    for (int t = class_ptr[cls] + threadIdx.x; t < class_ptr[cls + 1]; t += kBlock) {
        const double2 v = ui[class_sites[t]];
        re += v.x;
        im -= v.y;
    }
    __shared__ double lds[2][kBlock / 64];
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = re;
        lds[1][threadIdx.x >> 6] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int j = 0; j < kBlock / 64; ++j) {
            a += lds[0][j];
            b += lds[1][j];
        }
        coef[(size_t)slot * k + i] = make_double2(a, b);
    }
}

// out_slot += gamma5 sum_i coef[slot k + i] w_i  (D_ov b of deflated modes), grid (units, nslots).
__global__ __launch_bounds__(kBlock) void k_add_defl(Geom g, double2 *out, const double2 *w, int k,
                                                     const double2 *coef) {
    const int nsb = site_blocks(g);
    const int c = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    const int slot = blockIdx.y;
    if (s >= g.V) return;
    double ar = 0.0, ai = 0.0;
    for (int i = 0; i < k; ++i) {
        const double2 a = coef[(size_t)slot * k + i], v = w[(size_t)i * 12 * g.vs + c * g.vs + s];
        ar += a.x * v.x - a.y * v.y;
        ai += a.x * v.y + a.y * v.x;
    }
    const double f = c < 6 ? 1.0 : -1.0;
    double2 &o = out[(size_t)slot * 12 * g.vs + c * g.vs + s];
    o = make_double2(o.x + f * ar, o.y + f * ai);
}

void launch_multi_dot(const Geom &g, const double2 *Q, size_t qstride, int nq, const double2 *w, double *partial,
                      double2 *out, hipStream_t st) {
    const int np = unit_parts(0, g);
    hipLaunchKernelGGL(k_multi_dot, dim3(np, nq), dim3(kBlock), 0, st, g, Q, qstride, w, partial);
    hipLaunchKernelGGL(k_reduce_pairs, dim3(nq), dim3(64), 0, st, partial, np, out);
}

void launch_multi_axpy(const Geom &g, const double2 *Q, size_t qstride, int nq, const double2 *h, double2 *w,
                       bool overwrite, hipStream_t st) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(unit_parts(0, g)), dim3(kBlock), 0, st, g, Q, qstride, nq, h, w,
                       overwrite ? 1 : 0);
}

void launch_g5_scale(const Geom &g, double2 *v, double f, hipStream_t st) {
    hipLaunchKernelGGL(k_g5_scale, dim3(unit_parts(0, g)), dim3(kBlock), 0, st, g, v, f);
}

void launch_defl_coef_probe(const Geom &g, const double2 *u, int k, const int *slot_class, const int *slot_comp,
                            const int *class_ptr, const int *class_sites, int nslots, double2 *coef, hipStream_t st) {
    hipLaunchKernelGGL(k_defl_coef_probe, dim3(k, nslots), dim3(kBlock), 0, st, g, u, k, slot_class, slot_comp,
                       class_ptr, class_sites, coef);
}

void launch_add_defl(const Geom &g, double2 *out, const double2 *w, int k, const double2 *coef, int nslots,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_add_defl, dim3(unit_parts(0, g), nslots), dim3(kBlock), 0, st, g, out, w, k, coef);
}

// ------------------------------------------------------------------ precision conversion
__global__ __launch_bounds__(kBlock) void k_to_f32(Geom g, const double2 *src, float4 *dst) {
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const double2 *sp = src + (size_t)slot * 12 * g.vs;
    const double2 a = sp[(2 * u) * g.vs + s], b = sp[(2 * u + 1) * g.vs + s];
    dst[(size_t)slot * 6 * g.vs + u * g.vs + s] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
}

__global__ __launch_bounds__(kBlock) void k_to_f64(Geom g, const float4 *src, double2 *dst) {
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const float4 t = src[(size_t)slot * 6 * g.vs + u * g.vs + s];
    double2 *dp = dst + (size_t)slot * 12 * g.vs;
    dp[(2 * u) * g.vs + s] = make_double2(t.x, t.y);
    dp[(2 * u + 1) * g.vs + s] = make_double2(t.z, t.w);
}

// Host spinor layout [rhs][site][spin*3 + colour] complex128 <-> device [rhs][unit][site] double2.
__global__ __launch_bounds__(kBlock) void k_aos_to_soa(Geom g, const double2 *aos, double2 *soa) {
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    soa[((size_t)slot * 12 + u) * g.vs + s] = aos[((size_t)slot * g.V + s) * 12 + u];
}

__global__ __launch_bounds__(kBlock) void k_soa_to_aos(Geom g, const double2 *soa, double2 *aos) {
    const int slot = blockIdx.y;
    const int nsb = site_blocks(g);
    const int u = blockIdx.x / nsb;
    const int s = (blockIdx.x % nsb) * kBlock + threadIdx.x;
    if (s >= g.V) return;
    aos[((size_t)slot * g.V + s) * 12 + u] = soa[((size_t)slot * 12 + u) * g.vs + s];
}

void launch_layout(bool to_soa, const Geom &g, const double2 *src, double2 *dst, int nslots, hipStream_t st) {
    dim3 grid(unit_parts(0, g), nslots);
    if (to_soa)
        hipLaunchKernelGGL(k_aos_to_soa, grid, dim3(kBlock), 0, st, g, src, dst);
    else
        hipLaunchKernelGGL(k_soa_to_aos, grid, dim3(kBlock), 0, st, g, src, dst);
}

void launch_convert(int to_prec, const Geom &g, const void *src, void *dst, int nslots, hipStream_t st) {
    dim3 grid(unit_parts(1, g), nslots);
    if (to_prec == 1)
        hipLaunchKernelGGL(k_to_f32, grid, dim3(kBlock), 0, st, g, (const double2 *)src, (float4 *)dst);
    else
        hipLaunchKernelGGL(k_to_f64, grid, dim3(kBlock), 0, st, g, (const float4 *)src, (double2 *)dst);
}

// ------------------------------------------------------------------ calibration
// dst = src over n float4 (grid-stride), with cached or non-temporal loads and stores: kernels of
// known size (n * 16 bytes read and written) for scaling hardware byte counters.
template <bool NT>
__global__ __launch_bounds__(kBlock) void k_stream_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                        size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        if constexpr (NT) {
            const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(src + i));
            __builtin_nontemporal_store(t, reinterpret_cast<f32x4 *>(dst + i));
        } else {
            dst[i] = src[i];
        }
    }
}

void launch_stream_copy(bool nontemporal, const void *src, void *dst, size_t n_float4, hipStream_t st) {
    const size_t blocks = std::min<size_t>((n_float4 + kBlock - 1) / kBlock, 8192);
    if (nontemporal)
        hipLaunchKernelGGL(k_stream_copy<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const float4 *)src,
                           (float4 *)dst, n_float4);
    else
        hipLaunchKernelGGL(k_stream_copy<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const float4 *)src,
                           (float4 *)dst, n_float4);
}

}  // namespace smpq
