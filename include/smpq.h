/*
 * smpq.h -- C ABI of libsmpq: the overlap topological charge density
 *           q(x) = 1/2 tr(gamma5 D_ov)(x, x) by symmetric multi-probing, on AMD MI355X.
 *
 * The calls follow the paper's statement of the problem (Xiong, Zhang, Zou,
 * arXiv:1901.02211): a gauge field on a lattice L(nx, ny, nz, nt) (section 2.1),
 * the hopping parameter kappa of the Wilson kernel (section 1, Eq. 3), a
 * Zolotarev rational approximation of the sign function with its spectral
 * interval (Eq. 4), a probing scheme P(m_x, m_y, m_z, m_t, mode) (section 2.2,
 * Eq. 15) and, as output, q(x) (Eq. 16) and Q = sum_x q(x).
 *
 * Conventions shared by every call
 *  - Lattice: dims = {nx, ny, nz, nt}; site index s = x + nx*(y + ny*(z + nz*t));
 *    periodic boundary conditions in all four directions.  V = nx*ny*nz*nt.
 *  - Gamma basis (chiral, Euclidean, hermitian): gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
 *    for k = x, y, z; gamma_t = [[0, 1], [1, 0]]; gamma5 = gamma_x gamma_y gamma_z gamma_t
 *    = diag(1, 1, -1, -1).
 *  - Wilson kernel (Eq. 3): D_W psi(x) = psi(x) - kappa sum_mu [(1 - gamma_mu) U_mu(x) psi(x + mu)
 *    + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)];  H_W = gamma5 D_W;  D_ov = 1 + gamma5 eps(H_W).
 *  - Host gauge field: complex128 U[site][mu][row][col], interleaved (re, im) doubles,
 *    72*V doubles in all.
 *  - Host spinors: complex128 psi[rhs][site][spin][colour], 24*V doubles per right-hand side.
 *  - Ownership: every host buffer belongs to the caller; the library copies it in or out
 *    inside the call and keeps no pointer to it.  Device memory belongs to the context.
 *  - Errors: every call returns a smpq_status; negative values are errors, and
 *    smpq_last_error() gives a message for the last failing call on that context.
 *    Nothing throws across this boundary.  A failing call leaves the context usable.
 *  - Threads: a context is used by one host thread at a time.  All device work of a
 *    context runs on its stream, in order.
 *  - device = -1 creates a host-only context: colouring, Zolotarev coefficients and
 *    argument checks work, every call that needs the GPU returns SMPQ_EDEVICE.
 */
#ifndef SMPQ_H
#define SMPQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMPQ_MAX_POLES 32
#define SMPQ_MAX_DEFLATED 256

typedef struct smpq_ctx smpq_ctx;

typedef enum {
    SMPQ_OK = 0,
    SMPQ_EINVAL = -1,    /* bad argument (null pointer, out-of-range value)        */
    SMPQ_EDIM = -2,      /* sizes that do not fit the lattice or the scheme         */
    SMPQ_ENOMEM = -3,    /* device or host allocation failed                        */
    SMPQ_EDEVICE = -4,   /* HIP error, or a GPU call on a host-only context         */
    SMPQ_ENOCONV = -5,   /* a CG solve reached max_iter                              */
    SMPQ_ESTATE = -6,    /* call out of order (e.g. q(x) before a gauge field)      */
    SMPQ_ENUMERIC = -7   /* NaN/Inf, non-unitary links, or a CG breakdown           */
} smpq_status;

typedef enum {
    SMPQ_FP64 = 0,       /* every vector, link and scalar in FP64                    */
    SMPQ_MIXED_FP32 = 1, /* D_W and the CG body in FP32; FP64 CG scalars, FP64 reliable
                            updates of the residual, FP64 solution accumulators and
                            FP64 contraction                                          */
    SMPQ_MIXED_FP16DIR = 2, /* SMPQ_MIXED_FP32 with the search directions of the shifted
                            systems (all but the base system, whose direction D_W reads)
                            stored in FP16, each divided by a per-direction FP64 scale
                            zeta_i |r| / sqrt(24 V) that keeps its entries near 1; arithmetic
                            stays FP32.  Halves the bytes of those directions, but the
                            rounding of the stored directions reaches q(x): errors of
                            1e-4 (FP16) to 1e-3 (BF16) against the FP64 oracle on small
                            maps, against 1e-7 for SMPQ_MIXED_FP32.  An evaluated option,
                            not a recommended one                                     */
    SMPQ_MIXED_BF16DIR = 3, /* the same with BF16 storage (8-bit significand)          */
    SMPQ_MIXED_FP16VEC = 4, /* SMPQ_MIXED_FP32 with the vectors the FP32 stencil reads, the
                            base search direction p and D_W p, rounded to FP16 where they are
                            stored (each divided by its right-hand side's scale
                            |r| / sqrt(24 V), which keeps the entries near 1), the rest of the
                            path unchanged.  An evaluation of 16-bit storage of the stencil's
                            inputs: the values carry exactly the rounding of 16-bit storage but
                            stay in FP32 words, so the bytes and the time are those of
                            SMPQ_MIXED_FP32                                              */
    SMPQ_MIXED_BF16VEC = 5  /* the same rounded to BF16 (no scale needed)                 */
} smpq_precision;

typedef struct {
    double lam_min, lam_max;     /* Zolotarev interval used for |H_W|                  */
    double zolo_delta;           /* max |sign(x) - eps_Z(x)| on that interval           */
    double t_bounds_s;           /* Lanczos + Zolotarev set-up (0 if the interval was given) */
    double t_solve_s;            /* multi-shift CG over all sources                      */
    double t_contract_s;         /* rational assembly, contraction and copy-out          */
    double sum_imag_q;           /* sum_x Im q(x): zero up to rounding                   */
    double max_abs_imag_q;       /* diagnostic of the probing off-diagonal terms         */
    int64_t n_sources;           /* right-hand sides solved                             */
    int64_t n_batches;           /* device batches they were grouped in                 */
    int64_t total_iters;         /* sum over sources of CG iterations                   */
    int64_t max_iters;           /* largest CG iteration count of one source            */
    int64_t n_reliable_updates;  /* FP64 residual replacements (mixed precision)         */
    int64_t shift_updates;       /* sum over sources and iterations of updated shifts    */
    /* live kernel timing (HIP events on the context stream); filled when enabled
       with smpq_set_timing().  Bytes are the algorithmic bytes each kernel must move. */
    double dslash_ms;            /* total duration of the Wilson stencil launches        */
    double dslash_bytes;         /* algorithmic bytes of those launches                  */
    int64_t dslash_launches;
    double update_ms;            /* total duration of the fused multi-shift update       */
    double update_bytes;
    int64_t update_launches;
    double max_true_resid;       /* mixed precision: largest FP64 true residual
                                    ||b - (H^2 + q_1) x_1|| / ||b|| of the base system over the
                                    sources, taken after the solve (0 in FP64)              */
    /* per-shift check (smpq_set_shift_check; 0 when off) */
    double max_shift_resid;      /* largest FP64 ||b - (H^2 + q_i) x_i|| / ||b|| over sources
                                    and shifts, after the multi-shift solve                 */
    double max_shift_resid_final;/* the same after the refinement solves                    */
    int64_t n_refined;           /* (source, shift) systems refined                         */
    int64_t refine_iters;        /* CG iterations of the refinement solves (sum over sources) */
} smpq_stats;

/* Environment: SMPQ_TRACE (any value) when a context is created makes it print one line per
 * device batch to stderr (sources, CG iterations, solve time). */

/* Create a context for a lattice dims[4] = {nx, ny, nz, nt} on HIP device `device`
 * (-1: host only).  kappa starts at 0.21 (section 1), the solver at FP64 with
 * tol 1e-12, max_iter 10000 and a reliable update every 50 iterations.
 * Errors: EINVAL (null), EDIM (an extent < 1, or V >= 2^31), EDEVICE, ENOMEM. */
smpq_status smpq_create(const int dims[4], int device, smpq_ctx **out);

/* Release the context and all its device memory.  NULL is accepted. */
void smpq_destroy(smpq_ctx *ctx);

const char *smpq_strerror(smpq_status status);
const char *smpq_last_error(const smpq_ctx *ctx);

/* Copy a gauge field (host layout above, n_doubles = 72*V) to the device, keeping an
 * FP64 and an FP32 copy.  Rejects non-finite entries and links with
 * max |U^dag U - 1| > 1e-10 or |det U - 1| > 1e-10 (ENUMERIC).  (section 2.1) */
smpq_status smpq_load_gauge(smpq_ctx *ctx, const double *U, size_t n_doubles);

/* Hopping parameter of the Wilson kernel, 0 < kappa < 0.25 (section 1). */
smpq_status smpq_set_kappa(smpq_ctx *ctx, double kappa);

/* Lanczos on H_W^2 = D_W^dag D_W (FP64, on the device) for `steps` steps from the
 * SplitMix64 start vector of stream `seed` (counter i gives mix(seed + (i+1)*0x9e3779b97f4a7c15);
 * real parts from even counters, imaginary parts from odd ones, order (site, spin, colour)).
 * Returns the extreme Ritz values of H_W^2.  The interval of Eq. 4 is implied, not
 * printed, by the paper.  Errors: EINVAL (steps < 2), ESTATE (no gauge field). */
smpq_status smpq_lanczos(smpq_ctx *ctx, int steps, uint64_t seed, double *theta_min, double *theta_max);

/* Zolotarev interval for |H_W|: [0.9 sqrt(theta_min), 1.02 sqrt(theta_max)] from
 * smpq_lanczos(ctx, steps, 0, ...). */
smpq_status smpq_estimate_bounds(smpq_ctx *ctx, int steps, double *lam_min, double *lam_max);

/* Zolotarev coefficients of eps(H) ~ H (c_0 + sum_i c_i / (H^2 + q_i)) (Eq. 4) with
 * n_poles poles (the paper uses 14) on |H| in [lam_min, lam_max], computed on the host
 * in FP64.  Errors: EINVAL (n_poles outside 1..SMPQ_MAX_POLES, lam_min <= 0,
 * lam_min >= lam_max). */
smpq_status smpq_set_zolotarev(smpq_ctx *ctx, int n_poles, double lam_min, double lam_max);

/* Copy out the coefficients: c[n_poles], q[n_poles] (q ascending), delta = max error of
 * the approximation on the interval.  Any output pointer may be NULL.  ESTATE if unset. */
smpq_status smpq_get_zolotarev(const smpq_ctx *ctx, int *n_poles, double *c0, double *c,
                               double *q, double *delta);

/* Solver settings: precision, relative residual tol per shift (a shift stops once
 * zeta_i |r| <= tol |b|), iteration limit (ENOCONV when reached) and the interval, in
 * iterations, of FP64 residual replacement in the mixed precisions (0: none).  The solver
 * runs in groups of 10 iterations and tests convergence after each group, so
 * reliable_interval must be 0 or a multiple of 10 (EINVAL otherwise); max_iter is reached
 * at the end of the group that crosses it.  (section 2.1, Eqs. 6-8) */
smpq_status smpq_set_solver(smpq_ctx *ctx, smpq_precision prec, double tol, int max_iter,
                            int reliable_interval);

/* What a result computed with this context depends on besides the scheme and the Zolotarev
 * coefficients (for checkpoints that must not mix configurations): kappa, the solver settings
 * and a hash of the gauge field. */
typedef struct {
    double kappa;
    int precision;              /* smpq_precision                                        */
    double tol;
    int max_iter, reliable_interval;
    uint64_t gauge_hash;        /* FNV-1a (64 bit) of the bytes of the host field passed to
                                   the last successful smpq_load_gauge; 0 before one       */
} smpq_settings;

smpq_status smpq_get_settings(const smpq_ctx *ctx, smpq_settings *out);

/* Per-shift check of the shifted solves (section 2.1, Eqs. 6-8: every shifted system
 * M_i v_i = b is solved, not only the base system that the reliable updates correct).  With
 * enable = 1 every multi-shift solve also accumulates each shift's own solution x_i in FP64
 * and, after the solve, evaluates r_i = b - (H^2 + q_i) x_i in FP64 for every source and
 * shift (smpq_stats.max_shift_resid = max ||r_i|| / ||b||).  Where ||r_i|| / ||b|| >
 * refine_tol > 0, one refinement solve (H^2 + q_i) e = r_i runs in the context's precision
 * (reliable updates included) until its residual is below refine_tol ||b|| / 2, and
 * x_i += e, y += c_i e (max_shift_resid_final, n_refined, refine_iters).  refine_tol <= 0
 * checks without refining.  Applies to q(x), D_ov and the trace of D_W^-1 solves, not to
 * the inner solves of smpq_deflate.  Costs (n_poles + 2) FP64 vectors of device memory per
 * right-hand side (batches shrink accordingly), FP64 x_i traffic in the update and two FP64
 * stencils per shift after each batch.  The 16-bit direction precisions are refused
 * (EINVAL when a solve starts).  Default: off.  EINVAL: enable not 0/1, refine_tol >= 1 or
 * not finite. */
smpq_status smpq_set_shift_check(smpq_ctx *ctx, int enable, double refine_tol);

/* Upper bound on the right-hand sides resident on the device at once (0: automatic,
 * from free device memory).  Rounded down to a multiple of 12 when >= 12. */
smpq_status smpq_set_batch(smpq_ctx *ctx, int max_rhs);

/* Probing scheme with gaps r[mu] = n_mu / m_mu (section 2.2, Eqs. 15-19):
 *   mode 0 normal:  colour = x mod r                                 (prod r classes)
 *   mode 1 split:   colour = (x mod r, sum_mu floor(x_mu / r_mu) mod 2) (2 prod r classes;
 *                   every n_mu / r_mu must be even)
 *   mode 2 combine: classes x mod r and x mod r + r/2 merged            (prod r / 2 classes;
 *                   every r_mu must be even)
 * Labels: mode 0 = lexicographic index of (x mod r), x fastest; mode 1 = 2*that + parity;
 * mode 2 = index of the representative whose t-offset is < r_t/2.
 * Outputs (nullable): n_classes, n_sources = 12 * n_classes.  EDIM when r does not divide
 * the lattice or the mode's condition fails. */
smpq_status smpq_set_scheme(smpq_ctx *ctx, const int r[4], int mode, int *n_classes,
                            int *n_sources);

/* Minimal Euclidean distance between two sites of one class of the current scheme (Eq. 18;
 * minimum image on the torus) and the number of same-class sites at that distance from a
 * site (section 3).  Every class of the three modes is a translate of one sublattice, so
 * both are the same for all classes.  Host only.  0 and 0 when classes hold one site. */
smpq_status smpq_get_scheme_rmin(const smpq_ctx *ctx, double *r_min, int *nearest);

/* Point sources (section 2.1, Eq. 5): every site is its own class (V classes). */
smpq_status smpq_set_point_scheme(smpq_ctx *ctx, int *n_classes, int *n_sources);

/* Copy out the colour of every site (int32[V]).  ESTATE if no scheme is set. */
smpq_status smpq_get_coloring(const smpq_ctx *ctx, int32_t *colour);

/* out = D_W in (dagger = 0) or D_W^dag in (dagger = 1) for n_rhs spinors (host layout),
 * in the given precision (FP32 rounds the input, links and result through float). */
smpq_status smpq_apply_dw(smpq_ctx *ctx, const double *in, double *out, int n_rhs, int dagger,
                          smpq_precision prec);

/* smpq_apply_dw on caller-owned device buffers: in_dev and out_dev hold n_rhs spinors in the
 * host layout above ([rhs][site][spin][colour] complex128, 24 V doubles each) on the context's
 * device; the layout is converted on the device and the stream is synchronised before return.
 * Same results and errors as smpq_apply_dw (the same kernels).  The buffers must be memory of the
 * HIP runtime this library is linked to (hipMalloc in the same process): a framework that ships
 * its own copy of the HIP runtime (as some PyTorch wheels do) holds addresses of another runtime
 * instance, which this library cannot use. */
smpq_status smpq_apply_dw_dev(smpq_ctx *ctx, const double *in_dev, double *out_dev, int n_rhs, int dagger,
                              smpq_precision prec);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): smpq_apply_dw without any allocation.  Same
 * arguments, results and errors as smpq_apply_dw (the same stencil kernels); the host layout
 * is converted on the device.  Device memory comes from one fixed scratch array of 256 MiB per
 * GPU in the library (taken when the first context on that GPU is created and held until the
 * process ends); a call needs n_rhs * (192 V + 384 V_pad) bytes of it in FP64 and
 * n_rhs * (192 V + 576 V_pad) in FP32 (V_pad = V rounded up to 256), and EDIM is returned,
 * before any device work, when that exceeds 256 MiB (16^3 x 32: 2 right-hand sides in FP32).
 * Every call on one GPU uses the same array and leaves it holding its data: calls that
 * overlap on one GPU (from several threads or contexts) race. */
smpq_status smpq_apply_dw_noalloc(smpq_ctx *ctx, const double *in, double *out, int n_rhs, int dagger,
                                  smpq_precision prec);

/* out = D_ov in = in + gamma5 eps_Z(H_W) in (Eq. 3) for n_rhs spinors, through the
 * multi-shift CG of the solver settings.  Needs a gauge field and Zolotarev coefficients. */
smpq_status smpq_apply_dov(smpq_ctx *ctx, const double *in, double *out, int n_rhs);

/* q(x) on every site from all classes of the scheme (Eq. 16): for each class S and
 * each (alpha, a), phi = sum_{y in S} e_{y,alpha,a}, and for x in S
 * q(x) += 1/2 [gamma5 D_ov phi](x, alpha, a).  qx[V] gets Re q, qx_imag[V] (nullable) the
 * imaginary part (a diagnostic), Q (nullable) = sum_x qx[x].  If no Zolotarev
 * coefficients are set, 14 poles on smpq_estimate_bounds(ctx, 300) are used.
 * st (nullable) receives statistics.  The argument order puts the two V-sized maps side by
 * side and the scalar Q after them (the planned (qx, Q, qx_imag, st) order was changed for
 * that). */
smpq_status smpq_compute_qx(smpq_ctx *ctx, double *qx, double *qx_imag, double *Q,
                            smpq_stats *st);

/* smpq_compute_qx with the map left on the device: qx_dev (and qx_imag_dev, nullable) are
 * caller-owned device buffers of V doubles on the context's device, memory of the HIP runtime
 * this library is linked to (as for smpq_apply_dw_dev), written with device-to-device copies on
 * the context's stream, which is synchronised before return.  Q and st as in smpq_compute_qx
 * (Q summed on the host in the same order).  The buffers must not overlap the library's memory;
 * the call does not check that they are device memory. */
smpq_status smpq_compute_qx_dev(smpq_ctx *ctx, double *qx_dev, double *qx_imag_dev, double *Q,
                                smpq_stats *st);

/* As smpq_compute_qx for the listed classes only (each 0 <= class < n_classes, no
 * duplicates); sites of other classes are set to 0 in qx and qx_imag. */
smpq_status smpq_compute_qx_classes(smpq_ctx *ctx, const int32_t *classes, int n_classes,
                                    double *qx, double *qx_imag, smpq_stats *st);

/* Probing estimate of the trace of D_W^-1, the application the Conclusion proposes for the
 * same probing vectors (Eqs. 15-16): for x in the listed classes of the current scheme,
 *   t(x) = sum_{alpha,a} [D_W^-1 phi_{c,alpha,a}](x, alpha, a)
 *        = tr_sc D_W^-1(x, x) + sum_{y in S_c, y != x} sum_j D_W^-1(x j; y j),
 * exact with the point scheme (then sum_x t(x) = Tr D_W^-1, and t(x) is real).  Each source
 * is one CG solve of D_W^dag D_W y = phi (multi-shift machinery with the single shift 0, the
 * context's precision, tolerance and reliable updates), and D_W^-1 phi = g gamma5 D_W y with
 * g = gamma5 of the source's spin.  Needs no Zolotarev coefficients.
 *   classes   NULL: every class; else n distinct class indices
 *   t_re      V doubles, Re t(x) (0 outside the listed classes); t_im NULL or V doubles */
smpq_status smpq_compute_trinv(smpq_ctx *ctx, const int32_t *classes, int n, double *t_re, double *t_im,
                               smpq_stats *st);

/* Locality of the overlap operator (section 2.2, Eq. 12 and Fig. 1): the twelve columns
 * D_ov e_{site,beta,b} of the point source at `site` (one batch of 12 solves with the current
 * coefficients and precision), reduced at every x to
 *   mean_abs[x] = (1/144) sum_{alpha,a,beta,b} |D_ov(x alpha a; site beta b)|   (V doubles).
 * Averaging over the sites at one distance and fitting the logarithm gives the decay rate
 * gamma of Eq. 12. */
smpq_status smpq_dov_locality(smpq_ctx *ctx, int64_t site, double *mean_abs, smpq_stats *st);

/* Low-mode deflation of eps(H_W) (the exact sign on the lowest modes, the Zolotarev function
 * on the rest; the usual companion of the Zolotarev approximation of Eq. 4 when a few
 * eigenvalues of |H_W| lie far below the others).  Computes the n_modes lowest eigenpairs
 * (theta_i, u_i) of H_W^2 = D_W^dag D_W by `steps` steps of shift-and-invert Lanczos: Lanczos
 * with full reorthogonalisation on (H_W^2)^-1, each application an FP64 CG solve to relative
 * residual 1e-14 (start vector from the SplitMix64 stream 1; every Lanczos vector, 192 V_pad
 * bytes, is held on the device during the call); theta_i = <u_i, H^2 u_i> of the Ritz
 * vectors.  It keeps u_i and w_i = H_W u_i / sqrt(theta_i).  From then on smpq_compute_qx,
 * _classes, _points, _multi and smpq_apply_dov use
 *     eps b = sum_i w_i <u_i, b> + eps_Z(H_W) (b - sum_i u_i <u_i, b>)
 * (eps(H) = H (H^2)^(-1/2) maps u_i to w_i exactly); smpq_compute_trinv is unaffected.
 * n_modes = 0 removes the deflation, and so do smpq_load_gauge and smpq_set_kappa (the modes
 * belong to the previous operator).  Outputs (nullable): theta[n_modes + 1] = the deflated
 * values of H^2 ascending followed by the next Ritz value (the bottom of what the Zolotarev
 * function must cover); theta_max = the largest eigenvalue of H^2 (300 plain Lanczos steps);
 * max_resid = max_i ||H^2 u_i - theta_i u_i|| / theta_max.  With no Zolotarev coefficients
 * set, the next q(x) computation takes [0.9 sqrt(theta[n_modes]), 1.02 sqrt(theta_max)].
 * Errors: EINVAL (n_modes outside 0..SMPQ_MAX_DEFLATED, steps <= n_modes), ENUMERIC (the
 * Lanczos process ended before n_modes + 1 steps), ENOCONV (a mode's relative residual is
 * above 1e-12 after `steps` steps: more steps are needed; no deflation is kept). */
smpq_status smpq_deflate(smpq_ctx *ctx, int n_modes, int steps, double *theta, double *theta_max,
                         double *max_resid);

/* Exact point-source density (Eq. 5) on n listed sites: qx[i] = q(sites[i]).  Does not
 * change the scheme set with smpq_set_scheme. */
smpq_status smpq_compute_qx_points(smpq_ctx *ctx, const int64_t *sites, int n, double *qx,
                                   smpq_stats *st);

/* Allocate the device workspace that smpq_compute_qx will use with the current scheme,
 * solver settings and Zolotarev order, without computing anything (compute_qx otherwise
 * allocates on first use).  ESTATE without a gauge field, scheme or coefficients. */
smpq_status smpq_prepare(smpq_ctx *ctx);

/* Use `stream` (a hipStream_t) for all device work of the context; NULL restores the
 * context's own stream.  The caller keeps ownership of the stream. */
smpq_status smpq_set_stream(smpq_ctx *ctx, void *stream);

/* Enable (1) or disable (0) per-kernel HIP-event timing of the stencil and update
 * kernels inside the solver; results appear in smpq_stats. */
smpq_status smpq_set_timing(smpq_ctx *ctx, int enable);

/* Run each group of 10 CG iterations as a captured HIP graph (1, the default) or as eager
 * launches (0).  With per-kernel timing (smpq_set_timing) the graphs carry event-record
 * nodes around the timed kernels; where the runtime cannot capture those, timed groups run
 * eagerly. */
smpq_status smpq_set_graphs(smpq_ctx *ctx, int enable);

/* Standalone timing of the Wilson stencil: `launches` applications of D_W in the
 * given precision to n_rhs right-hand sides, rotating through n_sets disjoint
 * input/output/link sets so that consecutive launches do not reuse cached data.
 * Returns the mean duration per launch (HIP events) and the algorithmic bytes per
 * launch (links once, every input and output spinor once).  The buffers take at most half
 * of the free device memory: n_rhs is lowered to fit (SMPQ_ENOMEM if one does not). */
smpq_status smpq_bench_dslash(smpq_ctx *ctx, smpq_precision prec, int n_rhs, int n_sets,
                              int launches, double *ms_per_launch, double *bytes_per_launch);

/* Cap the device memory (bytes) the right-hand-side workspace of this context may take; the
 * batch size follows from it.  0 (the default) means 80% of the free device memory. */
smpq_status smpq_set_memory_limit(smpq_ctx *ctx, size_t bytes);

/* q(x) for several contexts at once on one device (configurations of different volume, each
 * with its own scheme, coefficients and precision): the q(x) of Eq. 16 per context, as
 * smpq_compute_qx_classes.  Contexts are prepared one after another (bounds by Lanczos when
 * no coefficients were set); contexts without a memory limit then share 80% of the free
 * device memory: one batch of 12 right-hand sides each first, the rest in proportion to
 * V x (number of classes), never more than a context can use (the excess goes to the
 * others).  Every context solves on its own stream from its own host thread, so the batches
 * of different contexts overlap on the GPU.  This replaces a single persistent launch over all
 * configurations: lattices of different geometry need different grids and stencil variants,
 * and measured overlap of separate streams leaves no idle device time to recover.  Results equal
 * those of separate calls bit for bit (each source's solve is independent of the batch it runs
 * in).
 *   ctxs[n_ctx]      distinct contexts on one device, with distinct streams, gauge and scheme set
 *   classes, n_classes  per-context class lists (NULL, or classes[k] NULL: every class)
 *   qx[k]            V_k doubles, written in full (sites of unlisted classes are 0)
 *   qx_imag          NULL, or per context NULL or V_k doubles
 *   st               NULL or n_ctx records
 *   failed           NULL or set to the index of the first failing context (-1 on success)
 * Returns the status of the first failing context (its message in smpq_last_error). */
smpq_status smpq_compute_qx_multi(smpq_ctx *const *ctxs, int n_ctx, const int32_t *const *classes,
                                  const int *n_classes, double *const *qx, double *const *qx_imag,
                                  smpq_stats *st, int *failed);

/* Device-to-device copy of `bytes` bytes (hipMemcpyAsync between two buffers of the context's
 * device, alternating direction), mean duration per copy over `launches` copies: the practical
 * bandwidth ceiling (2 * bytes / time) beside the roofline figures. */
smpq_status smpq_bench_copy(smpq_ctx *ctx, size_t bytes, int launches, double *ms_per_copy);

/* A hand-written streaming copy of `bytes` bytes (rounded down to 16) between two buffers of the
 * device, alternating direction, with cached (nontemporal = 0) or non-temporal (1) loads and
 * stores; mean duration per copy over `launches`.  A kernel of known size (bytes read and bytes
 * written per launch) for scaling hardware byte counters, and a bandwidth ceiling beside
 * smpq_bench_copy's library copy. */
smpq_status smpq_bench_stream(smpq_ctx *ctx, size_t bytes, int launches, int nontemporal, double *ms_per_copy);

/* Stencil variants.  f32_kind: 0 = one site per thread (f32_nr = 2, 4 or 8 right-hand sides
 * per thread, links held in registers across them); 1 = one 16x16 xy-plane per block staged
 * in LDS (nx*ny = 256; f32_nr = 4, 8 or 16); 2 = xy-tiles of ty rows plus one halo row on
 * each side staged in LDS, ty the largest divisor of ny with nx*ty <= 256 and a multiple of 64
 * (nx <= 64; f32_nr = 4, 8 or 16); 3 = kind 1 with the plane's x and y links in LDS instead
 * of registers, at 3 waves per SIMD; 4 = kind 2's tiles with the links read for every
 * right-hand side instead of held in registers (f32_nr = 1, 2, 4 or 8; 3-4 waves per SIMD), the
 * tile without halo rows when it is the whole plane.  plane_band (kinds 1-4; 1, 2 or 4, dividing nz): the
 * blocks take the (z, t) planes in bands of that many z with t running inside a band, so the
 * +-t neighbours of a plane were read shortly before (1 = z fastest).  FP64 stencil:
 * f64_kind 0 interleaves 2^f64_lgr = 1, 2 or 4 right-hand sides over the lanes of a block;
 * f64_kind 1 stages xy-tiles in LDS as FP32 kind 2 does (one halo row on each side unless the
 * tile is the whole plane), f64_nr = 1, 2, 4 or 8 right-hand sides per block, the links read as
 * their first two rows with the third rebuilt (where a tile fits; plane_band applies too).
 * f32_interleave (FP32 kind 4) and f64_interleave (FP64 kind 1): 1, 2, 4, 8 or 16 blocks in a
 * row take successive groups of right-hand sides of the same tile before the blocks move on
 * to the next tile, so that the links a tile reads for each right-hand side come from L2;
 * 1 for every other kind.
 * f32_kind, f32_nr and f32_interleave apply to the D_W launches (the first stencil of each CG
 * iteration, D_W p with the partial sums of <p, (H^2 + s) p>); f32_dag_kind, f32_dag_nr and
 * f32_dag_interleave, with the same meanings and limits, to the D_W^dag launches (the second,
 * which also updates the residual), so that each can use the variant that suits its epilogue.
 * Results do not depend on the variant beyond the rounding order of sums. */
typedef struct {
    int f32_kind, f32_nr, f64_lgr, plane_band;
    int f64_kind, f64_nr;
    int f32_interleave, f64_interleave;
    int f32_dag_kind, f32_dag_nr, f32_dag_interleave;
} smpq_tuning;

/* Choose the variants for this lattice by timing each on n_rhs right-hand sides as the solver
 * uses it: FP32 D_W with its partial sums and D_W^dag with the +sigma term and the residual
 * update, each alone and chosen separately (the plane band shared: the band with the smallest
 * sum of the two); FP64 the pair (two rotating buffer sets, 10 launches, best of two runs; fewer
 * right-hand sides where they would take more than half of the free device memory).  n_rhs = 0 times the batch size that a whole q(x)
 * map of the current scheme, coefficients and precision would use (ESTATE without them):
 * the variants' order can change with the number of right-hand sides through L2 reuse.  The choice is kept by the context and written to
 * *chosen (may be NULL); on an error the previous choice is kept.  Without this call a
 * context uses kind 1 / 8 where the plane fits, else kind 2 / 8 where a tile fits, else kind
 * 0 / 4 (the same for D_W and D_W^dag), with plane_band 1, f64_kind 0, f64_lgr 1 and the
 * interleaves 1. */
smpq_status smpq_autotune(smpq_ctx *ctx, int n_rhs, smpq_tuning *chosen);

/* Select the variants explicitly.  SMPQ_EINVAL (previous choice kept) if a variant is not
 * built or does not fit the lattice. */
smpq_status smpq_set_tuning(smpq_ctx *ctx, const smpq_tuning *tuning);

/* The variants in use. */
smpq_status smpq_get_tuning(smpq_ctx *ctx, smpq_tuning *tuning);

#ifdef __cplusplus
}
#endif
#endif /* SMPQ_H */
