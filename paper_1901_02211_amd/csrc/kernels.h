// Launch interface of the device kernels (kernels.hip) used by the C ABI (api.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace smpq {

constexpr int kBlock = 256;

// Geometry + storage strides.  A spinor of one right-hand side is stored as
// components [unit][site] with unit stride `vs` (the padded volume): FP64 uses 12
// double2 units (one complex each), FP32 uses 6 float4 units (two complexes each).
// FP64 links are [mu][row*3 + col][site] double2; FP32 links keep the first two rows,
// [mu][3][site] float4 holding (u00,u01), (u02,u10), (u11,u12).
struct Geom {
    int nx, ny, nz, nt, V;
    size_t vs;
    // stencil tuning (chosen per lattice, see smpq_autotune): FP32 kernel kind (0: one site per
    // thread, 1: 16x16 xy-plane per block in LDS, 2: xy-tile of tile_y rows with y-halos in
    // LDS), FP32 right-hand sides per thread, log2 of the right-hand sides interleaved over the
    // lanes of an FP64 block, and the z-band of the plane order of kinds 1 and 2;
    // tile_y = tile_rows(nx, ny) (0 when no tile fits); FP64 kernel kind (0: right-hand sides
    // interleaved over the lanes, 2^f64_lgr per block; 1: xy-tiles in LDS like the FP32 kind 2,
    // f64_nr right-hand sides per block, links read per right-hand side); f32_il / f64_il: in
    // the tile kernels (FP32 kind 4, FP64 kind 1) consecutive blocks take that many groups of
    // right-hand sides of one tile before the next tile, so that the tile's links are still in L2
    int f32_kind, f32_nr, f64_lgr, band, tile_y;
    int f64_kind, f64_nr;
    int f32_il, f64_il;
    // the FP32 variant of the D_W^dag launches (f32_kind, f32_nr and f32_il above apply to D_W):
    // the two stencils of a CG iteration have different epilogues and favour different variants
    int f32_dag_kind, f32_dag_nr, f32_dag_il;
};

// Right-hand-side addressing: slot k of a launch uses offset (slot * slot_stride + extra)
// units from the base pointer, where slot = list[k] (or k when list is null) and the
// number of slots is *count (or n when count is null).
struct Slots {
    const int *list;
    const int *count;
    int n;
};

// Per-batch multi-shift CG state (all device pointers; one entry per slot or slot*NS).
struct MSState {
    int B, NS, i0;
    double tol;
    double *rr, *bnorm, *alpha, *alpha_prev, *beta_prev;
    double *zeta, *zeta_prev, *zeta_new;
    int *sh_active, *sh_iters;
    int *done, *iters, *status;
    int *upd_n, *upd_idx, *upd_pupd;
    double *upd_cy, *upd_zeta, *upd_beta;
    double *upd_ax;      // alpha^i of each update-list entry (0 for a converged base entry)
    // 16-bit shifted directions: p_i is stored as p_i / sh_scale[slot NS + i]; per update-list
    // entry the scale that decodes the stored direction and the reciprocal of the new one
    double *sh_scale, *upd_sold, *upd_snew;
    double dir_norm;     // 1 / sqrt(24 V): a direction of norm n has entries of size ~ n dir_norm
    long long *cnt_entries, *cnt_pupd, *cnt_active, *cnt_base_pupd;
    const double *c, *delta;
    double *partial;     // per-block partial sums, slot stride pstride
    size_t pstride;
    int *list, *count;
};

// Source of the right-hand sides: probing (class, spin-colour component) or explicit FP64 vectors.
struct Source {
    const int *colour;      // probing: colour of each site
    const int *slot_class;  // probing: class of each slot
    const int *slot_comp;   // probing: component (spin*3 + colour) of each slot
    const double2 *b;       // explicit: FP64 vectors, slot stride 12*vs (null for probing)
    // deflation: the source is b - sum_{i < dk} dcoef[slot dk + i] u_i, u_i = du + i 12 vs
    const double2 *du = nullptr;
    const double2 *dcoef = nullptr;
    int dk = 0;
};

enum { kStatusOK = 0, kStatusBreakdown = 1 };

// With d = in - kappa * hop(in) (D_W in, or D_W^dag in when dag):
//   epi 0: out = d
//   epi 1: out = d + sigma * aux, partial[slot][block] = Re <aux, out>
//   epi 3: out = d, partial = |d|^2 + sigma |in|^2   (= <in, (H^2 + sigma) in> when dag = 0)
//   epi 2: out holds r; r -= alpha[slot] (d + sigma * aux) unless status[slot] is not OK;
//          partial = |r|^2 (the product d + sigma aux is not stored)
// prec: 0 = FP64, 1 = FP32 (FP32: epi 0 both ways, epi 3 with dag = 0, epi 1 and 2 with
// dag = 1).  The kernel variant comes from g's tuning fields; epilogues 1-3 write
// dslash_partials(prec, g) partials per slot.
void launch_dslash(int prec, bool dag, int epi, const void *U, const void *in, size_t in_stride,
                   size_t in_extra, void *out, size_t out_stride, const void *aux, size_t aux_stride,
                   size_t aux_extra, const Geom &g, double kappa, double sigma, Slots sl, int max_slots,
                   double *partial, hipStream_t st, const double *alpha = nullptr, const int *status = nullptr);
__host__ __device__ int site_blocks(const Geom &g);   // blocks of 256 sites
int dslash_partials(int prec, const Geom &g, bool dag);   // partials per slot of the stencil epilogue
bool plane_tileable(const Geom &g);
// Rows per xy-tile: the largest divisor ty >= 2 of ny with nx * ty <= 256 and a multiple of 64
// (nx <= 64); 0 when there is none.
int tile_rows(int nx, int ny);                    // the xy-plane has exactly 256 sites
bool valid_tuning(int prec, const Geom &g);            // g's tuning names an instantiated variant
int unit_parts(int prec, const Geom &g);        // partials per slot written by element-wise kernels
size_t partial_stride(const Geom &g);           // slot stride of the partial buffer (>= both)

// Storage of the shifted search directions p_i (i != base) in the FP32 path: FP32, or FP16 /
// BF16 scaled by a per-direction FP64 factor (the base direction, which the stencil reads,
// stays FP32).  With 16-bit storage, p holds only the base direction of each slot (slot
// stride one vector) and ph the NS directions in 16 bits (the base entry unused).
enum { kDirF32 = 0, kDirF16 = 1, kDirBF16 = 2 };

// r = p_i = b, y = c0 b; FP32 path: yacc = 0, x0 = 0, x0acc = 0 (pass null otherwise).  With
// 16-bit directions only r and the base direction are written; launch_dir16_init writes the
// others after launch_scalars_init has set their scales from |b|.
void launch_cg_init(int prec, const Geom &g, const Source &src, int nslots, int NS, double c0, void *r,
                    void *p, double2 *y, void *yacc, double2 *x0, void *x0acc, double *partial, int dir,
                    hipStream_t st);
void launch_dir16_init(const Geom &g, const MSState &s, int nslots, const void *r, int dir, void *ph, hipStream_t st);
void launch_scalars_init(const MSState &s, int npart, int nslots, hipStream_t st);
void launch_scalars_alpha(const MSState &s, int npart, hipStream_t st);
void launch_scalars_beta(const MSState &s, int npart, hipStream_t st);
// Shift update.  yt receives sum_i c_i alpha^i p_i: the FP64 y when y64, else a running sum in
// the storage precision of p.  xt (FP32 path only, else null) receives alpha p_base: the FP64
// x0 when x64, else a running sum.  The FP64 path always uses y64 (and no xt).  xs (null, or
// FP64 vectors [slot][NS][12][vs], FP32 directions only) receives every shift's own solution,
// x_i += alpha^i p_i, for the per-shift true-residual check.
void launch_shift_update(int prec, const Geom &g, const MSState &s, const void *r, void *p, void *yt, bool y64,
                         void *xt, bool x64, int dir, void *ph, double2 *xs, hipStream_t st);
// FP32 path: y += yacc, yacc = 0 (and x0 += x0acc, x0acc = 0 when x0acc is not null)
void launch_fold(const Geom &g, Slots sl, int max_slots, double2 *y, void *yacc, double2 *x0, void *x0acc,
                 hipStream_t st);
void launch_compact(const MSState &s, hipStream_t st);
// Evaluated precision: FP32 vectors of the listed slots (v + slot * slot_stride + extra, in
// float4 units) rounded in place to FP16 (mode 1, scaled by sqrt(|r|^2 / (24 V)) of the slot)
// or BF16 (mode 2).
void launch_round16(const Geom &g, const MSState &s, void *v, size_t slot_stride, size_t extra, int mode,
                    hipStream_t st);
void launch_reliable(int prec, const Geom &g, const MSState &s, const Source &src, const double2 *ap64,
                     void *r, hipStream_t st);
void launch_scalars_rr(const MSState &s, int npart, hipStream_t st);

// Per-shift check (FP64 vectors, slot stride 12 vs, the first nslots slots):
// resid64: out = b - ap64 (b from src), partial[slot][block] = |out|^2 (unit_parts(0, g) blocks);
// slot_sums: sums[slot] = sum of the slot's npart partials (fixed order);
// zero_unflagged: v[slot] = 0 where flag[slot] == 0;
// refine_acc: ysave[slot] += c e[slot], xsi[slot] += e[slot] (xsi slot stride xs_stride units).
void launch_resid64(const Geom &g, int nslots, const Source &src, const double2 *ap64, double2 *out,
                    double *partial, size_t pstride, hipStream_t st);
void launch_slot_sums(int nslots, const double *partial, size_t pstride, int npart, double *sums, hipStream_t st);
void launch_zero_unflagged(const Geom &g, int nslots, const int *flag, double2 *v, hipStream_t st);
void launch_refine_acc(const Geom &g, int nslots, const double2 *e, double c, double2 *ysave, double2 *xsi,
                       size_t xs_stride, hipStream_t st);

// Low-mode deflation helpers (FP64 vectors [12][vs]).  multi_dot: out[i] = <q_i, w> for
// q_i = Q + i qstride, i < nq (partial: 2 nq unit_parts doubles); multi_axpy: w -= sum h_i q_i,
// or w = sum h_i q_i with overwrite; g5_scale: v = f gamma5 v; defl_coef_probe: coef[slot k +
// i] = <u_i, phi_slot> for probing sources; add_defl: out_slot += gamma5 sum_i coef w_i.
void launch_multi_dot(const Geom &g, const double2 *Q, size_t qstride, int nq, const double2 *w, double *partial,
                      double2 *out, hipStream_t st);
void launch_multi_axpy(const Geom &g, const double2 *Q, size_t qstride, int nq, const double2 *h, double2 *w,
                       bool overwrite, hipStream_t st);
void launch_g5_scale(const Geom &g, double2 *v, double f, hipStream_t st);
void launch_defl_coef_probe(const Geom &g, const double2 *u, int k, const int *slot_class, const int *slot_comp,
                            const int *class_ptr, const int *class_sites, int nslots, double2 *coef, hipStream_t st);
void launch_add_defl(const Geom &g, double2 *out, const double2 *w, int k, const double2 *coef, int nslots,
                     hipStream_t st);

// m(x) = mean |D_ov(x i; site j)| over the 144 entries, from d_j = D_W y_j of the twelve
// point-source columns of `site` (Eq. 12).
void launch_block_mean_abs(const Geom &g, const double2 *d, int site, double *m, hipStream_t st);

// q(x) contraction (Eq. 16) for the classes of one batch; slot = 12*class_pos + comp.
// inverse: the trace density of D_W^-1 from y = (D_W^dag D_W)^-1 phi instead.  dk deflated
// modes add their exact-sign part from dw (H u_i / sqrt(theta_i)) and dcoef ([slot][dk]).
void launch_contract(const Geom &g, const double2 *U64, const double2 *y, double kappa, const int *batch_classes,
                     int n_classes, int max_class_size, const int *class_ptr, const int *class_sites, double *qx,
                     double *qxi, bool inverse, const double2 *dw, const double2 *dcoef, int dk, hipStream_t st);

// Lanczos helpers (single FP64 vector); the update writes unit_parts(0, g) partials
void launch_lanczos_update(const Geom &g, double2 *w, const double2 *v, const double2 *vprev, double alpha,
                           double beta, double *partial, hipStream_t st);
void launch_scale(const Geom &g, double2 *dst, const double2 *src, double f, hipStream_t st);
// dst = src over n float4 with cached (nontemporal = false) or non-temporal loads and stores:
// kernels of known size for scaling hardware byte counters
void launch_stream_copy(bool nontemporal, const void *src, void *dst, size_t n_float4, hipStream_t st);
// layout conversion between FP64 (double2 x 12) and FP32 (float4 x 6) spinors, n slots
void launch_convert(int to_prec, const Geom &g, const void *src, void *dst, int nslots, hipStream_t st);
// host spinor layout [slot][site][12] double2 (V sites per slot) <-> device [slot][12][vs]
void launch_layout(bool to_soa, const Geom &g, const double2 *src, double2 *dst, int nslots, hipStream_t st);

}  // namespace smpq
