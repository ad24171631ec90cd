// C ABI of libsmpq (include/smpq.h): context, gauge residency, Lanczos bounds,
// Zolotarev set-up, probing schemes, and the batched multi-shift CG driver that turns
// probing sources into q(x) (Xiong, Zhang, Zou, arXiv:1901.02211, sections 1-2); around it
// the stencil autotuner, concurrent contexts, low-mode deflation, the locality diagnostic and
// the trace of D_W^-1 by the same probing (Conclusion).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/smpq.h"
#include "host_math.h"
#include "kernels.h"

using namespace smpq;

// Device scratch of smpq_apply_dw_noalloc: a fixed array in the library's code object, one copy
// per GPU, held until the process ends.  In host code its name is only a stand-in for the
// symbol; kernels get the device address that hipGetSymbolAddress returns, taken once per device
// when the first context on that device is created.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch (the device must be current); nullptr if it cannot be had.
void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_ptr[device] = p;
    }
    return scratch_ptr[device];
}

struct Fail {
    smpq_status st;
    std::string msg;
};

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw Fail{e_ == hipErrorOutOfMemory ? SMPQ_ENOMEM : SMPQ_EDEVICE,                    \
                       std::string(#expr) + ": " + hipGetErrorString(e_)};                        \
    } while (0)

void *dev_alloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) return nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Fail{SMPQ_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    return p;
}

struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t b) {
        if (b <= bytes) return;
        release();
        p = dev_alloc(b);
        bytes = b;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

// Device workspace of one batch of right-hand sides.
struct Workspace {
    int prec = -1, NS = 0, B = 0;
    bool check = false;   // laid out for the per-shift check (xs, rres, ysave)
    DevMem r, tmp, p, ph, y, x0, tmp64, ap64, yacc, x0acc;
    DevMem xs, rres, ysave, sums, flags;   // per-shift check: x_i, residuals, saved y
    DevMem st_d;   // doubles of the MSState
    DevMem st_i;   // ints of the MSState
    DevMem st_l;   // long longs of the MSState
    DevMem partial, list, count, slot_class, slot_comp, batch_classes, bexp;
    MSState S{};
};

struct EventTimer {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    ~EventTimer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipEvent_t next() {
        if (used == ev.size()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            ev.push_back(e);
        }
        return ev[used++];
    }
    // record the next event on the stream; inside a stream capture it becomes an event node
    // of the graph, recorded again at every replay
    void record(hipStream_t s, bool captured) {
        hipEvent_t e = next();
        HIPCHK(captured ? hipEventRecordWithFlags(e, s, hipEventRecordExternal) : hipEventRecord(e, s));
    }
    // sum of elapsed times of consecutive (start, stop) pairs; requires the stream synced
    double sum() const {
        double ms = 0.0;
        for (size_t i = 0; i + 1 < used; i += 2) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            ms += t;
        }
        return ms;
    }
};

// Event pools of one group of iterations; for a captured group they are fixed at capture
// and read after every replay.
struct GroupTimers {
    EventTimer dslash, update;
};

}  // namespace

struct smpq_ctx {
    int dims[4];
    int V = 0;
    size_t vs = 0;
    int device = -1;
    hipStream_t own = nullptr, stream = nullptr;
    std::string err;
    double kappa = 0.21;
    bool have_gauge = false;
    uint64_t gauge_hash = 0;   // FNV-1a of the bytes of the loaded host field
    DevMem U64, U32;
    bool have_zolo = false;
    Zolo zolo;
    DevMem zc, zdelta;   // device copies of c_i and q_i - q_min
    // coefficients of the current multi-shift solve: the Zolotarev set, or the single
    // unshifted system of D_W^dag D_W (c0 = 0, c = 1, q = 0) for the trace of D_W^-1
    struct Coef {
        int n = 0;
        double c0 = 0.0, s0 = 0.0;
        const double *c = nullptr, *delta = nullptr;
    };
    Coef coef_eps, coef_inv, coef_ref;   // coef_ref: one shift of a refinement solve
    const Coef *coef = &coef_eps;
    const Coef *graph_coef = nullptr;   // the set the captured graphs were built with
    DevMem inv_cd;                      // {1, 0}: c and delta of the unshifted system
    // low-mode deflation: k eigenvectors u_i of H^2, w_i = H u_i / sqrt(theta_i), and the
    // per-slot coefficients <u_i, b> of the current batch
    int defl_k = 0;
    std::vector<double> defl_theta;
    double defl_next = 0.0, defl_tmax = 0.0;
    DevMem defl_u, defl_w, defl_coef;
    smpq_precision prec = SMPQ_FP64;
    double tol = 1e-12;
    int max_iter = 10000;
    int reliable = 50;
    int max_rhs = 0;
    size_t mem_limit = 0;   // workspace bytes a batch may use (0: 80% of free device memory)
    size_t run_limit = 0;   // share assigned by a multi-context call while it runs
    bool have_scheme = false;
    std::vector<int32_t> colour;
    int n_classes = 0;
    std::vector<int32_t> cptr, csites;
    DevMem d_colour, d_cptr, d_csites;
    DevMem d_pcolour, d_pptr;   // point scheme (identity) on demand
    Workspace ws;
    DevMem qx, qxi, lz;
    bool timing = false;
    bool use_graphs = true;
    // per-shift FP64 true-residual check and mixed refinement (smpq_set_shift_check)
    bool shift_check = false;
    double refine_tol = 0.0;
    bool refining = false;          // inside a refinement solve, which has no check of its own
    double2 *cur_xs = nullptr;      // x_i accumulators of the solve in progress (check mode)
    bool trace = std::getenv("SMPQ_TRACE") != nullptr;   // one line per batch on stderr
    // captured groups of kGroup CG iterations, one per accumulation variant; rebuilt when
    // anything they capture (workspace, links, coefficients, solver settings) changes
    // [timed][variant]; the timed graphs carry event nodes around the stencil and update kernels
    hipGraphExec_t graphs[2][4] = {{nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr, nullptr}};
    long long graph_gen[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};
    GroupTimers graph_timers[4];
    GroupTimers eager_timers;
    bool graph_timing_ok = true;
    long long gen = 0;
    int *h_count = nullptr;     // pinned
    // stencil variant (see Geom); defaults: plane tile where the xy-plane has 256 sites
    int f32_kind = 0, f32_nr = 4, f64_lgr = 1, band = 1, f64_kind = 0, f64_nr = 4, f32_il = 1, f64_il = 1;
    int f32_dag_kind = 0, f32_dag_nr = 4, f32_dag_il = 1;   // the D_W^dag launches
    Geom geom() const {
        return Geom{dims[0], dims[1], dims[2], dims[3], V, vs, f32_kind, f32_nr, f64_lgr, band,
                    tile_rows(dims[0], dims[1]), f64_kind, f64_nr, f32_il, f64_il, f32_dag_kind, f32_dag_nr,
                    f32_dag_il};
    }
    smpq_tuning tuning() const {
        return smpq_tuning{f32_kind, f32_nr, f64_lgr, band, f64_kind, f64_nr, f32_il, f64_il,
                           f32_dag_kind, f32_dag_nr, f32_dag_il};
    }
    void set_tuning(const smpq_tuning &t) {
        f32_kind = t.f32_kind;
        f32_nr = t.f32_nr;
        f64_lgr = t.f64_lgr;
        band = t.plane_band;
        f64_kind = t.f64_kind;
        f64_nr = t.f64_nr;
        f32_il = t.f32_interleave;
        f64_il = t.f64_interleave;
        f32_dag_kind = t.f32_dag_kind;
        f32_dag_nr = t.f32_dag_nr;
        f32_dag_il = t.f32_dag_interleave;
    }
};

namespace {

void need_device(smpq_ctx *c) {
    if (c->device < 0) throw Fail{SMPQ_EDEVICE, "host-only context (device = -1)"};
    HIPCHK(hipSetDevice(c->device));
}

template <class F>
smpq_status guarded(smpq_ctx *c, F &&f) {
    if (!c) return SMPQ_EINVAL;
    try {
        f();
        c->err.clear();
        return SMPQ_OK;
    } catch (const Fail &e) {
        c->err = e.msg;
        return e.st;
    } catch (const std::exception &e) {
        c->err = e.what();
        return SMPQ_EINVAL;
    }
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// host spinor [rhs][site][spin][colour] complex128 <-> device [rhs][comp][site] double2
void spinor_to_device(const smpq_ctx *c, const double *h, int n, std::vector<double> &stage) {
    stage.assign((size_t)n * 24 * c->vs, 0.0);
    for (int r = 0; r < n; ++r)
        for (int s = 0; s < c->V; ++s)
            for (int k = 0; k < 12; ++k) {
                const double *src = h + ((size_t)r * c->V + s) * 24 + 2 * k;
                double *dst = stage.data() + 2 * (((size_t)r * 12 + k) * c->vs + s);
                dst[0] = src[0];
                dst[1] = src[1];
            }
}

void spinor_from_device(const smpq_ctx *c, const std::vector<double> &stage, int n, double *h) {
    for (int r = 0; r < n; ++r)
        for (int s = 0; s < c->V; ++s)
            for (int k = 0; k < 12; ++k) {
                const double *src = stage.data() + 2 * (((size_t)r * 12 + k) * c->vs + s);
                double *dst = h + ((size_t)r * c->V + s) * 24 + 2 * k;
                dst[0] = src[0];
                dst[1] = src[1];
            }
}


// The CG body runs in groups of kGroup iterations; the host reads the number of active
// right-hand sides after each group.  FP32 path: the first iterations build most of y and x0
// (the residual falls by ~10^3 in the first 50 iterations at these condition numbers), so they
// accumulate straight into FP64: y for the first kDirectY iterations, x0 until the first
// reliable update.  Later contributions go to FP32 running sums, folded into FP64 at the end
// of every group (y) and at every reliable update (x0).
constexpr int kGroup = 10;
constexpr int kDirectY = 30;   // a multiple of kGroup

// Internal precision codes follow smpq_precision: 0 FP64; 1 FP32 body; 2 / 3 FP32 body with
// the shifted search directions stored in FP16 / BF16.  vec_prec is the precision of the
// residual, the stencil and every other vector; dir_store the storage of the shifted directions.
inline int vec_prec(int prec) { return prec == 0 ? 0 : 1; }
// precisions 4 / 5: the stencil's input vectors rounded to FP16 / BF16 after they are written
inline int vec16_mode(int prec) { return prec == 4 ? 1 : prec == 5 ? 2 : 0; }
inline int dir_store(int prec) { return prec == 2 ? kDirF16 : prec == 3 ? kDirBF16 : kDirF32; }

size_t bytes_per_slot(const smpq_ctx *c, int prec, int NS) {
    const size_t v64 = 12 * 16 * c->vs, v32 = 6 * 16 * c->vs, v16 = v32 / 2;
    // per-shift check: x_i for every shift, the residual and the saved y (+ tmp64 and ap64 in FP64)
    const size_t check = c->shift_check ? (NS + 2) * v64 + (prec == 0 ? 2 * v64 : 0) : 0;
    // r, tmp, the NS directions and y (+ in the FP32 path the running sums of y and x0, and the
    // FP64 x0, tmp64 and ap64 of the reliable updates)
    if (prec == 0) return (2 + NS) * v64 + v64 + check;
    if (dir_store(prec) != kDirF32) return 5 * v32 + NS * v16 + 4 * v64 + check;
    return (4 + NS) * v32 + 4 * v64 + check;
}

// Device workspace for at least B right-hand sides of the given precision and shift count.
// Everything, including the per-RHS CG state, is sized and laid out for the capacity w.B, the
// slot range every launch covers; a new layout invalidates the captured graphs.
void ensure_workspace(smpq_ctx *c, int prec, int NS, int B) {
    Workspace &w = c->ws;
    const Geom g = c->geom();
    const size_t v64 = 12 * 16 * c->vs, v32 = 6 * 16 * c->vs;
    const size_t vt = prec == 0 ? v64 : v32;
    if (w.prec == prec && w.NS == NS && w.B >= B && w.check == c->shift_check && w.S.rr) return;
    c->gen++;
    w.r.release(); w.tmp.release(); w.p.release(); w.ph.release(); w.y.release();
    w.x0.release(); w.tmp64.release(); w.ap64.release(); w.yacc.release(); w.x0acc.release();
    w.xs.release(); w.rres.release(); w.ysave.release();
    w.prec = prec;
    w.NS = NS;
    w.B = B;
    w.check = c->shift_check;
    w.r.ensure(vt * B);
    w.tmp.ensure(vt * B);
    if (dir_store(prec) != kDirF32) {
        w.p.ensure(vt * B);              // base directions
        w.ph.ensure(v32 / 2 * B * NS);   // shifted directions, 16 bits
    } else {
        w.p.ensure(vt * B * NS);
    }
    w.y.ensure(v64 * B);
    if (prec >= 1) {
        w.x0.ensure(v64 * B);
        w.tmp64.ensure(v64 * B);
        w.ap64.ensure(v64 * B);
        w.yacc.ensure(v32 * B);
        w.x0acc.ensure(v32 * B);
    }
    if (w.check) {
        w.xs.ensure(v64 * B * NS);
        w.rres.ensure(v64 * B);
        w.ysave.ensure(v64 * B);
        w.tmp64.ensure(v64 * B);
        w.ap64.ensure(v64 * B);
        w.sums.ensure(sizeof(double) * B);
        w.flags.ensure(sizeof(int) * B);
    }
    const size_t pstride = partial_stride(g);
    w.st_d.ensure(sizeof(double) * ((size_t)B * (5 + 3 * NS + 4 * NS + 3 * NS)));
    w.st_i.ensure(sizeof(int) * ((size_t)B * (2 * NS + 4 + 2 * NS) + 16));
    w.st_l.ensure(sizeof(long long) * (size_t)B * 4);
    w.partial.ensure(sizeof(double) * (size_t)B * pstride);
    w.list.ensure(sizeof(int) * B);
    w.count.ensure(sizeof(int) * 4);
    w.slot_class.ensure(sizeof(int) * B);
    w.slot_comp.ensure(sizeof(int) * B);
    w.batch_classes.ensure(sizeof(int) * (B / 12 + 1));
    MSState &S = w.S;
    double *d = w.st_d.as<double>();
    S.rr = d; d += B;
    S.bnorm = d; d += B;
    S.alpha = d; d += B;
    S.alpha_prev = d; d += B;
    S.beta_prev = d; d += B;
    S.zeta = d; d += (size_t)B * NS;
    S.zeta_prev = d; d += (size_t)B * NS;
    S.zeta_new = d; d += (size_t)B * NS;
    S.upd_cy = d; d += (size_t)B * NS;
    S.upd_zeta = d; d += (size_t)B * NS;
    S.upd_beta = d; d += (size_t)B * NS;
    S.upd_ax = d; d += (size_t)B * NS;
    S.sh_scale = d; d += (size_t)B * NS;
    S.upd_sold = d; d += (size_t)B * NS;
    S.upd_snew = d; d += (size_t)B * NS;
    S.dir_norm = 1.0 / std::sqrt(24.0 * (double)c->V);
    int *ip = w.st_i.as<int>();
    S.sh_active = ip; ip += (size_t)B * NS;
    S.sh_iters = ip; ip += (size_t)B * NS;
    S.done = ip; ip += B;
    S.iters = ip; ip += B;
    S.status = ip; ip += B;
    S.upd_n = ip; ip += B;
    S.upd_idx = ip; ip += (size_t)B * NS;
    S.upd_pupd = ip; ip += (size_t)B * NS;
    long long *lp = w.st_l.as<long long>();
    S.cnt_entries = lp; lp += B;
    S.cnt_pupd = lp; lp += B;
    S.cnt_active = lp; lp += B;
    S.cnt_base_pupd = lp; lp += B;
    S.partial = w.partial.as<double>();
    S.pstride = pstride;
    S.list = w.list.as<int>();
    S.count = w.count.as<int>();
    S.NS = NS;
    S.B = B;
}

// Free the right-hand-side vectors of the workspace (the next ensure_workspace lays it out again).
void release_workspace(smpq_ctx *c) {
    Workspace &w = c->ws;
    w.r.release(); w.tmp.release(); w.p.release(); w.ph.release(); w.y.release();
    w.x0.release(); w.tmp64.release(); w.ap64.release(); w.yacc.release(); w.x0acc.release();
    w.xs.release(); w.rres.release(); w.ysave.release();
    w.prec = -1;
    w.B = 0;
    w.S.rr = nullptr;
    c->gen++;
}

size_t workspace_bytes(const smpq_ctx *c) {
    const Workspace &w = c->ws;
    return (size_t)w.r.bytes + w.tmp.bytes + w.p.bytes + w.ph.bytes + w.y.bytes + w.x0.bytes + w.tmp64.bytes +
           w.ap64.bytes + w.yacc.bytes + w.x0acc.bytes + w.xs.bytes + w.rres.bytes + w.ysave.bytes;
}

int choose_batch(smpq_ctx *c, int prec, int NS, int total_slots, bool multiple_of_12) {
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    // memory already held by a workspace of the same shape is reusable
    size_t held = 0;
    if (c->ws.prec == prec && c->ws.NS == NS) held = bytes_per_slot(c, prec, NS) * c->ws.B;
    else held = workspace_bytes(c);
    const size_t limit = c->run_limit > 0 ? c->run_limit : c->mem_limit;
    const double budget = limit > 0 ? (double)limit : 0.80 * (double)(freeb + held);
    long long B = (long long)(budget / (double)bytes_per_slot(c, prec, NS));
    if (c->max_rhs > 0) B = std::min<long long>(B, c->max_rhs);
    B = std::min<long long>(B, total_slots);
    const int q = multiple_of_12 ? 12 : 1;
    B = (B / q) * q;
    if (B < q) throw Fail{SMPQ_ENOMEM, "not enough device memory for one batch of right-hand sides"};
    // spread the right-hand sides evenly over the batches this limit implies
    const long long nb = (total_slots + B - 1) / B;
    const long long even = ((total_slots + nb - 1) / nb + q - 1) / q * q;
    return (int)std::min(B, even);
}

void require_gauge_zolo(smpq_ctx *c) {
    if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
    if (!c->have_zolo) throw Fail{SMPQ_ESTATE, "no Zolotarev coefficients set"};
}

void upload_zolo(smpq_ctx *c) {
    const int n = c->zolo.n;
    std::vector<double> dl(n);
    for (int i = 0; i < n; ++i) dl[i] = c->zolo.q[i] - c->zolo.q[0];
    c->zc.ensure(sizeof(double) * n);
    c->zdelta.ensure(sizeof(double) * n);
    HIPCHK(hipMemcpy(c->zc.p, c->zolo.c.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->zdelta.p, dl.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    c->coef_eps = smpq_ctx::Coef{n, c->zolo.c0, c->zolo.q[0], c->zc.as<double>(), c->zdelta.as<double>()};
}

// Select the coefficient set of the next solves (Zolotarev or the unshifted inverse).
void use_coef(smpq_ctx *c, bool inverse) {
    if (inverse && !c->inv_cd.p) {
        const double cd[2] = {1.0, 0.0};
        c->inv_cd.ensure(sizeof(cd));
        HIPCHK(hipMemcpy(c->inv_cd.p, cd, sizeof(cd), hipMemcpyHostToDevice));
        c->coef_inv = smpq_ctx::Coef{1, 0.0, 0.0, c->inv_cd.as<double>(), c->inv_cd.as<double>() + 1};
    }
    c->coef = inverse ? &c->coef_inv : &c->coef_eps;
}

struct BatchResult {
    long long iters_sum = 0, iters_max = 0, n_reliable = 0, entries = 0, pupd = 0, active = 0;
    double max_true_resid = 0.0;
};

// One CG iteration for every active slot of the batch (capacity-sized launches; inactive
// slots exit at once).  y64 / x64 select FP64 or FP32-running-sum accumulation (FP32 path).
// The first stencil, tmp = D_W p, also sums <p, (H^2 + s0) p> = |tmp|^2 + s0 |p|^2, so alpha is
// known before the second, which updates r -= alpha (D_W^dag tmp + s0 p) in place with the
// partials of |r|^2 (the product itself is never stored).  With timers, events bracket the two
// stencil launches and the update launch.
void enqueue_iteration(smpq_ctx *c, int prec, const MSState &S, bool y64, bool x64, GroupTimers *tm,
                       bool captured) {
    Workspace &w = c->ws;
    const Geom g = c->geom();
    hipStream_t s = c->stream;
    const int NS = S.NS, B = S.B;
    const int vp = vec_prec(prec), dir = dir_store(prec);
    const size_t rs = (vp == 0 ? 12 : 6) * c->vs;
    // the base direction: one of NS per slot, or (16-bit shifted directions) the only one
    const size_t pst = dir == kDirF32 ? NS * rs : rs, pofs = dir == kDirF32 ? S.i0 * rs : 0;
    const void *U = vp == 0 ? c->U64.p : c->U32.p;
    // partials per slot of the first (D_W p) and the second (D_W^dag) stencil
    const int np_ds = dslash_partials(vp, g, false), np_dag = dslash_partials(vp, g, true);
    const bool mixed = prec >= 1;
    const Slots act{S.list, S.count, 0};
    const double s0 = c->coef->s0;
    if (tm) tm->dslash.record(s, captured);
    launch_dslash(vp, false, 3, U, w.p.p, pst, pofs, w.tmp.p, rs, nullptr, 0, 0, g, c->kappa, s0, act, B, S.partial, s);
    if (tm) tm->dslash.record(s, captured);
    const int m16 = vec16_mode(prec);
    if (m16) launch_round16(g, S, w.tmp.p, rs, 0, m16, s);   // D_W p as 16-bit storage would hold it
    launch_scalars_alpha(S, np_ds, s);
    if (tm) tm->dslash.record(s, captured);
    launch_dslash(vp, true, 2, U, w.tmp.p, rs, 0, w.r.p, rs, w.p.p, pst, pofs, g, c->kappa, s0, act, B, S.partial, s,
                  S.alpha, S.status);
    if (tm) tm->dslash.record(s, captured);
    launch_scalars_beta(S, np_dag, s);
    if (tm) tm->update.record(s, captured);
    launch_shift_update(vp, g, S, w.r.p, w.p.p, y64 ? w.y.p : w.yacc.p, y64,
                        mixed ? (x64 ? w.x0.p : w.x0acc.p) : nullptr, x64, dir, w.ph.p, c->cur_xs, s);
    if (tm) tm->update.record(s, captured);
    if (m16) launch_round16(g, S, w.p.p, pst, pofs, m16, s);   // the new base direction
    launch_compact(S, s);
}

// One group of kGroup iterations starting at iteration it0, plus the fold of the FP32 running
// sum of y at its end when the group used it.
void enqueue_group(smpq_ctx *c, int prec, const MSState &S, int it0, GroupTimers *tm, bool captured) {
    const bool mixed = prec >= 1;
    const bool y64 = !mixed || it0 < kDirectY;
    const bool x64 = mixed && (c->reliable == 0 || it0 < c->reliable);
    for (int gi = 0; gi < kGroup; ++gi) enqueue_iteration(c, prec, S, y64, x64, tm, captured);
    if (mixed && !y64)
        launch_fold(c->geom(), Slots{S.list, S.count, 0}, S.B, c->ws.y.as<double2>(), c->ws.yacc.p, nullptr, nullptr,
                    c->stream);
}

// Graph variant of a group (0: FP64 path; 1-3: FP32 path with FP64 y and x0 / FP32 y and FP64 x0
// / FP32 y and x0); -1 when the group is launched eagerly.
int group_variant(const smpq_ctx *c, int prec, int it0) {
    if (prec == 0) return 0;
    if (c->reliable % kGroup != 0) return -1;   // x0 accumulation would switch inside a group
    const bool y64 = it0 < kDirectY;
    const bool x64 = c->reliable == 0 || it0 < c->reliable;
    return y64 ? (x64 ? 1 : -1) : (x64 ? 2 : 3);
}

// Launch one group, as a captured graph where possible.  Returns the timers to read after
// the stream has synchronised (null when not timing).
GroupTimers *launch_group(smpq_ctx *c, int prec, const MSState &S, int it0) {
    const bool timed = c->timing;
    const int v = (!c->use_graphs || (timed && !c->graph_timing_ok)) ? -1 : group_variant(c, prec, it0);
    if (v < 0) {
        GroupTimers *tm = timed ? &c->eager_timers : nullptr;
        if (tm) tm->dslash.used = tm->update.used = 0;
        enqueue_group(c, prec, S, it0, tm, false);
        return tm;
    }
    if (c->graph_coef != c->coef) {   // the graphs hold the coefficients of the other set
        c->gen++;
        c->graph_coef = c->coef;
    }
    const int t = timed ? 1 : 0;
    GroupTimers *tm = timed ? &c->graph_timers[v] : nullptr;
    if (!c->graphs[t][v] || c->graph_gen[t][v] != c->gen) {
        if (c->graphs[t][v]) HIPCHK(hipGraphExecDestroy(c->graphs[t][v]));
        c->graphs[t][v] = nullptr;
        if (tm) tm->dslash.used = tm->update.used = 0;
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_group(c, prec, S, it0, tm, true);
        } catch (const Fail &) {
            (void)hipStreamEndCapture(c->stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            if (!timed) throw;
            c->graph_timing_ok = false;   // no event nodes in graphs: time eagerly from now on
            return launch_group(c, prec, S, it0);
        }
        HIPCHK(hipStreamEndCapture(c->stream, &graph));
        const hipError_t e = hipGraphInstantiateWithFlags(&c->graphs[t][v], graph, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(e);
        c->graph_gen[t][v] = c->gen;
    }
    HIPCHK(hipGraphLaunch(c->graphs[t][v], c->stream));
    return tm;
}

// Multi-shift CG for the first nslots slots of the workspace, sources from src.
// On return y[slot] = c_0 b + sum_i c_i x_i (Eq. 4 without the leading H).
void check_shifts(smpq_ctx *c, int prec, int nslots, const Source &src, smpq_stats *st);

BatchResult run_batch(smpq_ctx *c, int prec, int nslots, const Source &src, smpq_stats *st) {
    Workspace &w = c->ws;
    MSState S = w.S;
    S.B = w.B;           // launches are sized for the workspace capacity; slots >= nslots start done
    // a solve may use fewer shifts than the workspace holds (a refinement solves one)
    if (c->coef->n > w.NS) throw Fail{SMPQ_ESTATE, "workspace laid out for fewer shifts than the solve"};
    S.NS = c->coef->n;
    S.i0 = 0;            // q ascending: the smallest shift is the base system
    S.tol = c->tol;
    S.c = c->coef->c;
    S.delta = c->coef->delta;
    const int NS = S.NS;
    const Geom g = c->geom();
    hipStream_t s = c->stream;
    const double s0 = c->coef->s0;
    const size_t rs64 = 12 * c->vs;
    const int vp = vec_prec(prec), dir = dir_store(prec);
    const int np_unit = unit_parts(vp, g);
    const Slots act{S.list, S.count, 0};
    const bool mixed = prec >= 1;

    const bool check = c->shift_check && !c->refining;
    if (check && !w.check) throw Fail{SMPQ_ESTATE, "workspace laid out without the per-shift check"};
    if (check && dir != kDirF32)
        throw Fail{SMPQ_EINVAL, "the per-shift check needs SMPQ_FP64 or SMPQ_MIXED_FP32"};
    if (check) HIPCHK(hipMemsetAsync(w.xs.p, 0, (size_t)nslots * NS * rs64 * sizeof(double2), s));
    // the graphs capture this pointer: a change of check mode or refinement bumps c->gen
    c->cur_xs = check ? w.xs.as<double2>() : nullptr;
    launch_cg_init(vp, g, src, nslots, NS, c->coef->c0, w.r.p, w.p.p, w.y.as<double2>(), mixed ? w.yacc.p : nullptr,
                   mixed ? w.x0.as<double2>() : nullptr, mixed ? w.x0acc.p : nullptr, S.partial, dir, s);
    launch_scalars_init(S, np_unit, nslots, s);
    if (dir != kDirF32) launch_dir16_init(g, S, nslots, w.r.p, dir, w.ph.p, s);
    launch_compact(S, s);
    if (vec16_mode(prec))   // the first base direction, b, with the scale |b|
        launch_round16(g, S, w.p.p, dir == kDirF32 ? NS * rs64 / 2 : rs64 / 2, 0, vec16_mode(prec), s);
    HIPCHK(hipGetLastError());

    BatchResult res;
    int iter = 0;
    for (;;) {
        GroupTimers *tm = launch_group(c, prec, S, iter);
        iter += kGroup;
        if (mixed && c->reliable > 0 && iter % c->reliable == 0) {
            // residual replacement: fold the running base solution, r = b - (H^2 + s0) x0 in FP64
            // the running sum of y was folded at the end of the group (or is still zero before
            // the first FP32-summed group), so only x0's is folded here
            launch_fold(g, act, S.B, nullptr, nullptr, w.x0.as<double2>(), w.x0acc.p, s);
            launch_dslash(0, false, 0, c->U64.p, w.x0.p, rs64, 0, w.tmp64.p, rs64, nullptr, 0, 0, g,
                          c->kappa, 0.0, act, S.B, nullptr, s);
            launch_dslash(0, true, 1, c->U64.p, w.tmp64.p, rs64, 0, w.ap64.p, rs64, w.x0.p, rs64, 0, g,
                          c->kappa, s0, act, S.B, S.partial, s);
            launch_reliable(vp, g, S, src, w.ap64.as<double2>(), w.r.p, s);
            launch_scalars_rr(S, np_unit, s);
            res.n_reliable++;
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(c->h_count, S.count, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (tm && st) {
            st->dslash_ms += tm->dslash.sum();
            st->update_ms += tm->update.sum();
        }
        if (*c->h_count == 0) {
            if (mixed)   // the slots finished at different iterations: fold every one of them
                launch_fold(g, Slots{nullptr, nullptr, nslots}, nslots, w.y.as<double2>(), w.yacc.p,
                            w.x0.as<double2>(), w.x0acc.p, s);
            break;
        }
        if (iter >= c->max_iter)
            throw Fail{SMPQ_ENOCONV, "multi-shift CG did not converge within max_iter = " + std::to_string(c->max_iter)};
    }
    if (mixed) {
        // FP64 true residual ||b - (H^2 + s0) x0|| / ||b|| of the base system of every slot,
        // x0 being FP64 after the final fold
        std::vector<int> all(nslots);
        for (int k = 0; k < nslots; ++k) all[k] = k;
        *c->h_count = nslots;
        HIPCHK(hipMemcpyAsync(S.list, all.data(), sizeof(int) * nslots, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(S.count, c->h_count, sizeof(int), hipMemcpyHostToDevice, s));
        launch_dslash(0, false, 0, c->U64.p, w.x0.p, rs64, 0, w.tmp64.p, rs64, nullptr, 0, 0, g, c->kappa, 0.0, act,
                      S.B, nullptr, s);
        launch_dslash(0, true, 1, c->U64.p, w.tmp64.p, rs64, 0, w.ap64.p, rs64, w.x0.p, rs64, 0, g, c->kappa, s0,
                      act, S.B, S.partial, s);
        launch_reliable(vp, g, S, src, w.ap64.as<double2>(), w.r.p, s);
        launch_scalars_rr(S, np_unit, s);
        HIPCHK(hipGetLastError());
        std::vector<double> rr(nslots), bn(nslots);
        HIPCHK(hipMemcpyAsync(rr.data(), S.rr, sizeof(double) * nslots, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(bn.data(), S.bnorm, sizeof(double) * nslots, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int k = 0; k < nslots; ++k)
            res.max_true_resid = std::max(res.max_true_resid, std::sqrt(rr[k]) / bn[k]);
    }
    c->cur_xs = nullptr;
    std::vector<int> status(nslots), iters(nslots);
    std::vector<long long> ent(nslots), pup(nslots), actv(nslots), bpup(nslots);
    HIPCHK(hipMemcpy(status.data(), S.status, sizeof(int) * nslots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(iters.data(), S.iters, sizeof(int) * nslots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ent.data(), S.cnt_entries, sizeof(long long) * nslots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(pup.data(), S.cnt_pupd, sizeof(long long) * nslots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(actv.data(), S.cnt_active, sizeof(long long) * nslots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(bpup.data(), S.cnt_base_pupd, sizeof(long long) * nslots, hipMemcpyDeviceToHost));
    long long base_pupd = 0;
    for (int k = 0; k < nslots; ++k) {
        if (status[k] != kStatusOK) throw Fail{SMPQ_ENUMERIC, "CG breakdown: <p, A p> <= 0 or not finite"};
        res.iters_sum += iters[k];
        res.iters_max = std::max<long long>(res.iters_max, iters[k]);
        res.entries += ent[k];
        res.pupd += pup[k];
        res.active += actv[k];
        base_pupd += bpup[k];
    }
    if (st) {
        const double s_t = prec == 0 ? 16.0 : 8.0;           // bytes per complex spinor entry
        const double link_site = prec == 0 ? 576.0 : 192.0;   // link bytes per site (FP32: two rows)
        // bytes per complex entry of a listed direction: the base direction (one entry per
        // slot-iteration) is stored like r, 16-bit shifted directions take 4
        const double s_dir = dir == kDirF32 ? s_t : 4.0;
        const double V = c->V;
        // algorithmic bytes: each stencil reads the links once and each input spinor once; the
        // first writes tmp, the second reads p for the "+ s0 p" term and reads and writes r.
        // Six vector passes per active slot-iteration; every slot starts at iteration 0, so
        // iterations_max launches carried work.
        const double launched = (double)res.iters_max;
        st->dslash_bytes += launched * 2.0 * link_site * V + (double)res.active * V * 12.0 * s_t * 6.0;
        st->dslash_launches += 2LL * res.iters_max;
        // update kernel: r read, the running sum read+write and, in the FP32 path, the running
        // base solution read+write (both in the iteration precision), every listed p_i read,
        // every updated p_i written.
        // All slots of a batch start together, so slot k ran iterations 0 .. iters[k]-1: the
        // first min(iters, kDirectY) of them summed y in FP64, the first min(iters, reliable)
        // summed x0 in FP64 (FP32 path).
        double acc_bytes = 0.0;
        for (int k = 0; k < nslots; ++k) {
            const double n = iters[k];
            if (prec == 0) {
                acc_bytes += n * 2.0 * 192.0;
            } else {
                const double ny = std::min<double>(n, kDirectY);
                const double nx = c->reliable > 0 ? std::min<double>(n, c->reliable) : n;
                acc_bytes += ny * 2.0 * 192.0 + (n - ny) * 2.0 * 96.0 + nx * 2.0 * 192.0 + (n - nx) * 2.0 * 96.0;
            }
        }
        const double dir_units = (double)(res.active + base_pupd) * s_t +
                                 (double)(res.entries - res.active + res.pupd - base_pupd) * s_dir;
        st->update_bytes += V * ((double)res.active * 12.0 * s_t + acc_bytes + 12.0 * dir_units);
        st->update_launches += res.iters_max;
        st->n_reliable_updates += res.n_reliable;
        st->max_true_resid = std::max(st->max_true_resid, res.max_true_resid);
        st->shift_updates += res.entries;
    }
    if (check) check_shifts(c, prec, nslots, src, st);
    return res;
}

// Every shift's FP64 true residual ||b - (H^2 + q_i) x_i|| / ||b|| for the first nslots slots
// of the solve just finished (x_i accumulated in FP64 beside y); shifts above refine_tol get one
// refinement solve (H^2 + q_i) e = b - (H^2 + q_i) x_i in the solve's precision, from the FP64
// residual, and x_i += e, y += c_i e.  Each shifted system of Eqs. 6-8 is thereby held to its
// own FP64 residual, not only the base system of the reliable updates.
void check_shifts(smpq_ctx *c, int prec, int nslots, const Source &src, smpq_stats *st) {
    Workspace &w = c->ws;
    const Geom g = c->geom();
    hipStream_t s = c->stream;
    const smpq_ctx::Coef coef = *c->coef;
    const smpq_ctx::Coef *coef_ptr = c->coef;
    const int NS = coef.n;
    const size_t rs64 = 12 * c->vs;
    const size_t vbytes = rs64 * sizeof(double2);
    const size_t pstride = partial_stride(g);
    const int np = unit_parts(0, g);
    if (!c->inv_cd.p) {
        const double cd[2] = {1.0, 0.0};
        c->inv_cd.ensure(sizeof(cd));
        HIPCHK(hipMemcpy(c->inv_cd.p, cd, sizeof(cd), hipMemcpyHostToDevice));
    }
    std::vector<double> ch(NS), dh(NS), bn(nslots);
    HIPCHK(hipMemcpyAsync(ch.data(), coef.c, sizeof(double) * NS, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dh.data(), coef.delta, sizeof(double) * NS, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(bn.data(), w.S.bnorm, sizeof(double) * nslots, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(w.ysave.p, w.y.p, vbytes * nslots, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    const Slots all{nullptr, nullptr, nslots};
    std::vector<double> rr(nslots);
    auto resid = [&](int i, std::vector<double> &out) {
        double2 *xi = w.xs.as<double2>() + (size_t)i * rs64;
        launch_dslash(0, false, 0, c->U64.p, xi, NS * rs64, 0, w.tmp64.p, rs64, nullptr, 0, 0, g, c->kappa, 0.0, all,
                      nslots, nullptr, s);
        launch_dslash(0, true, 1, c->U64.p, w.tmp64.p, rs64, 0, w.ap64.p, rs64, xi, NS * rs64, 0, g, c->kappa,
                      coef.s0 + dh[i], all, nslots, w.S.partial, s);
        launch_resid64(g, nslots, src, w.ap64.as<double2>(), w.rres.as<double2>(), w.S.partial, pstride, s);
        launch_slot_sums(nslots, w.S.partial, pstride, np, w.sums.as<double>(), s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(rr.data(), w.sums.p, sizeof(double) * nslots, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        out.assign(nslots, 0.0);
        for (int k = 0; k < nslots; ++k) out[k] = bn[k] > 0.0 ? std::sqrt(rr[k]) / bn[k] : 0.0;
    };
    const double tol_main = c->tol;
    std::vector<double> before, after;
    std::vector<int> flag(nslots);
    for (int i = 0; i < NS; ++i) {
        resid(i, before);
        double mx = 0.0, rho = 0.0;
        int nref = 0;
        for (int k = 0; k < nslots; ++k) {
            mx = std::max(mx, before[k]);
            flag[k] = c->refine_tol > 0.0 && before[k] > c->refine_tol;
            if (flag[k]) {
                ++nref;
                rho = std::max(rho, before[k]);
            }
        }
        if (st) st->max_shift_resid = std::max(st->max_shift_resid, mx);
        if (nref == 0) {
            if (st) st->max_shift_resid_final = std::max(st->max_shift_resid_final, mx);
            continue;
        }
        HIPCHK(hipMemcpyAsync(w.flags.p, flag.data(), sizeof(int) * nslots, hipMemcpyHostToDevice, s));
        launch_zero_unflagged(g, nslots, w.flags.as<int>(), w.rres.as<double2>(), s);
        // (H^2 + q_i) e = r_i: one shift of coefficient 1 and no constant term; the residual
        // must fall below refine_tol |b|, i.e. by refine_tol / rho relative to r_i
        c->coef_ref = smpq_ctx::Coef{1, 0.0, coef.s0 + dh[i], c->inv_cd.as<double>(), c->inv_cd.as<double>() + 1};
        c->coef = &c->coef_ref;
        c->tol = std::min(0.5, std::max(tol_main, 0.5 * c->refine_tol / rho));
        c->refining = true;
        c->gen++;
        const Source rsrc{nullptr, nullptr, nullptr, w.rres.as<double2>()};
        smpq_stats rst{};
        BatchResult rb;
        try {
            rb = run_batch(c, prec, nslots, rsrc, &rst);
        } catch (...) {
            c->coef = coef_ptr;
            c->tol = tol_main;
            c->refining = false;
            c->gen++;
            throw;
        }
        c->coef = coef_ptr;
        c->tol = tol_main;
        c->refining = false;
        c->gen++;
        launch_refine_acc(g, nslots, w.y.as<double2>(), ch[i], w.ysave.as<double2>(),
                          w.xs.as<double2>() + (size_t)i * rs64, NS * rs64, s);
        resid(i, after);
        double mf = 0.0;
        for (int k = 0; k < nslots; ++k) mf = std::max(mf, after[k]);
        if (st) {
            st->max_shift_resid_final = std::max(st->max_shift_resid_final, mf);
            st->n_refined += nref;
            st->refine_iters += rb.iters_sum;
        }
    }
    HIPCHK(hipMemcpyAsync(w.y.p, w.ysave.p, vbytes * nslots, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
}

void ensure_scheme_device(smpq_ctx *c) {
    if (c->d_colour.p) return;
    c->d_colour.ensure(sizeof(int) * c->V);
    c->d_cptr.ensure(sizeof(int) * (c->n_classes + 1));
    c->d_csites.ensure(sizeof(int) * c->V);
    HIPCHK(hipMemcpy(c->d_colour.p, c->colour.data(), sizeof(int) * c->V, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_cptr.p, c->cptr.data(), sizeof(int) * (c->n_classes + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_csites.p, c->csites.data(), sizeof(int) * c->V, hipMemcpyHostToDevice));
}

void ensure_point_device(smpq_ctx *c) {
    if (c->d_pcolour.p) return;
    std::vector<int> id(c->V + 1);
    for (int i = 0; i <= c->V; ++i) id[i] = i;
    c->d_pcolour.ensure(sizeof(int) * c->V);
    c->d_pptr.ensure(sizeof(int) * (c->V + 1));
    HIPCHK(hipMemcpy(c->d_pcolour.p, id.data(), sizeof(int) * c->V, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_pptr.p, id.data(), sizeof(int) * (c->V + 1), hipMemcpyHostToDevice));
}

void lanczos(smpq_ctx *c, int steps, uint64_t seed, double *tmin, double *tmax) {
    const Geom g = c->geom();
    const size_t v64 = 12 * 16 * c->vs;
    c->lz.ensure(4 * v64);
    double2 *v = c->lz.as<double2>(), *vp = v + 12 * c->vs, *w = vp + 12 * c->vs, *t = w + 12 * c->vs;
    const int np_ds = dslash_partials(0, g, true), np_unit = unit_parts(0, g);
    DevMem part;
    part.ensure(sizeof(double) * partial_stride(g));
    std::vector<double> h((size_t)24 * c->V), stage;
    for (size_t i = 0; i < h.size(); ++i) h[i] = 2.0 * splitmix64_uniform(seed, i) - 1.0;
    double nrm = 0.0;
    for (double x : h) nrm += x * x;
    nrm = std::sqrt(nrm);
    for (double &x : h) x /= nrm;
    spinor_to_device(c, h.data(), 1, stage);
    HIPCHK(hipMemsetAsync(c->lz.p, 0, 4 * v64, c->stream));
    HIPCHK(hipMemcpyAsync(v, stage.data(), v64, hipMemcpyHostToDevice, c->stream));
    std::vector<double> alpha, beta, hp(partial_stride(g));
    Slots one{nullptr, nullptr, 1};
    double bprev = 0.0;
    for (int j = 0; j < steps; ++j) {
        launch_dslash(0, false, 0, c->U64.p, v, 0, 0, t, 0, nullptr, 0, 0, g, c->kappa, 0.0, one, 1, nullptr,
                      c->stream);
        launch_dslash(0, true, 1, c->U64.p, t, 0, 0, w, 0, v, 0, 0, g, c->kappa, 0.0, one, 1, part.as<double>(),
                      c->stream);
        HIPCHK(hipMemcpyAsync(hp.data(), part.p, sizeof(double) * np_ds, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double a = 0.0;
        for (int i = 0; i < np_ds; ++i) a += hp[i];
        alpha.push_back(a);
        if (j == steps - 1) break;
        launch_lanczos_update(g, w, v, vp, a, bprev, part.as<double>(), c->stream);
        HIPCHK(hipMemcpyAsync(hp.data(), part.p, sizeof(double) * np_unit, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double b2 = 0.0;
        for (int i = 0; i < np_unit; ++i) b2 += hp[i];
        const double b = std::sqrt(b2);
        if (!(b > 0.0) || !std::isfinite(b)) break;
        beta.push_back(b);
        launch_scale(g, vp, w, 1.0 / b, c->stream);
        std::swap(v, vp);
        bprev = b;
    }
    HIPCHK(hipGetLastError());
    beta.resize(alpha.size() - 1);
    tridiag_extremes(alpha, beta, tmin, tmax);
}

// Lanczos with full (two-pass classical Gram-Schmidt) reorthogonalisation in FP64 for the
// hermitian operator `apply` (w = A q), every vector kept in Q; returns the tridiagonal
// (alpha, beta) of the steps taken (fewer when an invariant subspace is found).
template <class Apply>
void lanczos_full(smpq_ctx *c, int steps, uint64_t seed, double2 *Qp, DevMem &w, DevMem &part, DevMem &h,
                  Apply apply, std::vector<double> &alpha, std::vector<double> &beta) {
    const Geom g = c->geom();
    const size_t vl = 12 * c->vs;
    hipStream_t s = c->stream;
    std::vector<double> hv((size_t)24 * c->V), stage;
    double nrm = 0.0;
    for (size_t i = 0; i < hv.size(); ++i) {
        hv[i] = 2.0 * splitmix64_uniform(seed, i) - 1.0;
        nrm += hv[i] * hv[i];
    }
    for (double &x : hv) x /= std::sqrt(nrm);
    spinor_to_device(c, hv.data(), 1, stage);
    HIPCHK(hipMemcpyAsync(Qp, stage.data(), vl * sizeof(double2), hipMemcpyHostToDevice, s));
    double2 *wp = w.as<double2>();
    double2 hw[1];
    alpha.clear();
    beta.clear();
    for (int j = 0; j < steps; ++j) {
        double2 *qj = Qp + (size_t)j * vl;
        apply(qj, wp);
        launch_multi_dot(g, qj, 0, 1, wp, part.as<double>(), h.as<double2>(), s);
        HIPCHK(hipMemcpyAsync(hw, h.p, sizeof(double2), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double a = hw[0].x;
        alpha.push_back(a);
        if (j == steps - 1) break;
        launch_lanczos_update(g, wp, qj, j > 0 ? qj - vl : qj, a, j > 0 ? beta.back() : 0.0, part.as<double>(), s);
        for (int pass = 0; pass < 2; ++pass) {
            launch_multi_dot(g, Qp, vl, j + 1, wp, part.as<double>(), h.as<double2>(), s);
            launch_multi_axpy(g, Qp, vl, j + 1, h.as<double2>(), wp, false, s);
        }
        launch_multi_dot(g, wp, 0, 1, wp, part.as<double>(), h.as<double2>(), s);
        HIPCHK(hipMemcpyAsync(hw, h.p, sizeof(double2), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double b = std::sqrt(hw[0].x);
        if (!(b > 1e-14 * (std::fabs(a) + (beta.empty() ? 0.0 : beta.back()))) || !std::isfinite(b)) break;
        beta.push_back(b);
        launch_scale(g, Qp + (size_t)(j + 1) * vl, wp, 1.0 / b, s);
    }
    HIPCHK(hipGetLastError());
    beta.resize(alpha.size() - 1);
}

// largest relative residual ||H^2 u - theta u|| / theta_max a deflated mode may have: the
// angle to the true eigenvector is about this times theta_max / (gap to the next eigenvalue)
constexpr double kDeflTol = 1e-12;

void drop_deflation(smpq_ctx *c) {
    c->defl_k = 0;
    c->defl_theta.clear();
    c->defl_u.release();
    c->defl_w.release();
}

// The k lowest eigenpairs of H^2 by shift-and-invert Lanczos: Lanczos on (H^2)^-1, applied
// by an FP64 CG solve to relative residual 1e-14 (the multi-shift solver with the single
// shift 0), turns the lowest eigenvalues theta of H^2 into the largest, best separated ones,
// 1/theta; the Ritz vectors u_i of the k largest are refined by their Rayleigh quotients
// theta_i = <u_i, H^2 u_i>, and w_i = H u_i / sqrt(theta_i) = gamma5 D_W u_i / sqrt(theta_i).
// theta_max comes from the plain Lanczos bound of the context (300 steps).
void deflate(smpq_ctx *c, int k, int steps, double *theta_out, double *tmax_out, double *resid_out) {
    const Geom g = c->geom();
    const size_t vl = 12 * c->vs;   // double2 per vector
    const size_t v64 = vl * sizeof(double2);
    hipStream_t s = c->stream;
    const Slots one{nullptr, nullptr, 1};
    steps = std::min(steps, 12 * c->V);
    DevMem Q, t, w, part, h;
    Q.ensure(v64 * steps);
    t.ensure(v64);
    w.ensure(v64);
    const int np = unit_parts(0, g);
    part.ensure(sizeof(double) * std::max<size_t>((size_t)2 * steps * np, partial_stride(g)));
    h.ensure(sizeof(double2) * (steps + 2));
    double2 *Qp = Q.as<double2>(), *tp = t.as<double2>(), *wp = w.as<double2>();
    auto h2 = [&](const double2 *in, double2 *out, double sigma) {   // out = (H^2 + sigma) in
        launch_dslash(0, false, 0, c->U64.p, in, 0, 0, tp, 0, nullptr, 0, 0, g, c->kappa, 0.0, one, 1, nullptr, s);
        launch_dslash(0, true, 1, c->U64.p, tp, 0, 0, out, 0, in, 0, 0, g, c->kappa, sigma, one, 1,
                      part.as<double>(), s);
    };
    // the inner solves run in FP64 at tolerance 1e-14 with the unshifted coefficient set
    struct Keep {
        smpq_ctx *c;
        smpq_precision prec;
        double tol;
        bool check;
        ~Keep() {
            c->prec = prec;
            c->tol = tol;
            c->shift_check = check;
            use_coef(c, false);
        }
    } keep{c, c->prec, c->tol, c->shift_check};
    c->prec = SMPQ_FP64;
    c->tol = 1e-14;
    c->shift_check = false;   // the inner solves are single-shift FP64 solves to 1e-14
    use_coef(c, true);
    ensure_workspace(c, 0, 1, c->ws.prec == 0 && c->ws.NS == 1 ? c->ws.B : 1);
    auto inverse = [&](const double2 *q, double2 *o) {
        Source src{nullptr, nullptr, nullptr, q};
        run_batch(c, 0, 1, src, nullptr);
        HIPCHK(hipMemcpyAsync(o, c->ws.y.p, v64, hipMemcpyDeviceToDevice, s));
    };
    std::vector<double> alpha, beta, ev, Z;
    lanczos_full(c, steps, 1, Qp, w, part, h, inverse, alpha, beta);
    try {
        tridiag_eigen(alpha, beta, ev, Z);
    } catch (const std::exception &e) {
        throw Fail{SMPQ_ENUMERIC, e.what()};
    }
    const int m = (int)ev.size();
    if (m <= k) throw Fail{SMPQ_ENUMERIC, "Lanczos ended before n_modes + 1 steps"};
    double tmin_b, tmax_b;
    lanczos(c, 300, 0, &tmin_b, &tmax_b);
    c->defl_k = 0;
    c->defl_u.release();
    c->defl_w.release();
    c->defl_u.ensure(v64 * k);
    c->defl_w.ensure(v64 * k);
    std::vector<double2> sv(m);
    std::vector<double> th(k);
    double2 hw[1];
    double worst = 0.0;
    for (int i = 0; i < k; ++i) {
        const int col = m - 1 - i;   // largest eigenvalues of (H^2)^-1 first
        for (int j = 0; j < m; ++j) sv[j] = make_double2(Z[(size_t)col * m + j], 0.0);
        HIPCHK(hipMemcpyAsync(h.p, sv.data(), sizeof(double2) * m, hipMemcpyHostToDevice, s));
        double2 *ui = c->defl_u.as<double2>() + (size_t)i * vl, *wi = c->defl_w.as<double2>() + (size_t)i * vl;
        launch_multi_axpy(g, Qp, vl, m, h.as<double2>(), ui, true, s);
        h2(ui, wp, 0.0);
        launch_multi_dot(g, ui, 0, 1, wp, part.as<double>(), h.as<double2>() + m, s);
        HIPCHK(hipMemcpyAsync(hw, h.as<double2>() + m, sizeof(double2), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        th[i] = hw[0].x;
        if (!(th[i] > 0.0)) throw Fail{SMPQ_ENUMERIC, "non-positive Rayleigh quotient of H^2"};
        h2(ui, wp, -th[i]);   // residual H^2 u - theta u
        launch_multi_dot(g, wp, 0, 1, wp, part.as<double>(), h.as<double2>() + m, s);
        HIPCHK(hipMemcpyAsync(hw, h.as<double2>() + m, sizeof(double2), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        worst = std::max(worst, std::sqrt(hw[0].x) / tmax_b);
        launch_dslash(0, false, 0, c->U64.p, ui, 0, 0, wi, 0, nullptr, 0, 0, g, c->kappa, 0.0, one, 1, nullptr, s);
        launch_g5_scale(g, wi, 1.0 / std::sqrt(th[i]), s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    if (!(worst <= kDeflTol)) {   // unconverged modes would bend eps: refuse them
        drop_deflation(c);
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "deflated modes not converged: residual %.2e of theta_max after %d Lanczos steps "
                      "(needs <= %.0e; take more steps)", worst, m, kDeflTol);
        throw Fail{SMPQ_ENOCONV, msg};
    }
    c->defl_theta = th;
    c->defl_next = 1.0 / ev[m - 1 - k];
    c->defl_tmax = tmax_b;
    c->defl_k = k;
    c->gen++;
    if (theta_out) {
        for (int i = 0; i < k; ++i) theta_out[i] = th[i];
        theta_out[k] = c->defl_next;
    }
    if (tmax_out) *tmax_out = tmax_b;
    if (resid_out) *resid_out = worst;
}

void set_zolo(smpq_ctx *c, int n, double lo, double hi) {
    if (n < 1 || n > SMPQ_MAX_POLES) throw Fail{SMPQ_EINVAL, "n_poles must be in 1..SMPQ_MAX_POLES"};
    if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi))
        throw Fail{SMPQ_EINVAL, "need 0 < lam_min < lam_max"};
    try {
        c->zolo = zolotarev(n, lo, hi);
    } catch (const std::exception &e) {
        throw Fail{SMPQ_ENUMERIC, e.what()};
    }
    c->have_zolo = true;
    c->gen++;
    if (c->device >= 0) upload_zolo(c);
}

void auto_zolo(smpq_ctx *c, smpq_stats *st) {
    if (c->have_zolo) return;
    if (c->defl_k > 0) {   // the deflation's Lanczos already bounds the rest of the spectrum
        set_zolo(c, 14, 0.9 * std::sqrt(c->defl_next), 1.02 * std::sqrt(c->defl_tmax));
        return;
    }
    const double t0 = now_s();
    double tmin, tmax;
    lanczos(c, 300, 0, &tmin, &tmax);
    set_zolo(c, 14, 0.9 * std::sqrt(tmin), 1.02 * std::sqrt(tmax));
    if (st) st->t_bounds_s += now_s() - t0;
}

// q(x) for the listed classes of a colouring (scheme or point), written into the
// device arrays qx/qxi (which the caller zeroes).
void qx_classes(smpq_ctx *c, const std::vector<int> &classes, bool point, smpq_stats *st, bool inverse = false) {
    const int prec = (int)c->prec;
    use_coef(c, inverse);
    const int NS = c->coef->n;
    const int total = (int)classes.size() * 12;
    if (total == 0) return;
    const int B = choose_batch(c, prec, NS, total, true);
    ensure_workspace(c, prec, NS, B);
    Workspace &w = c->ws;
    const int *colour = point ? c->d_pcolour.as<int>() : c->d_colour.as<int>();
    const int *cptr = point ? c->d_pptr.as<int>() : c->d_cptr.as<int>();
    const int *csites = point ? c->d_pcolour.as<int>() : c->d_csites.as<int>();
    const int per = B / 12;
    std::vector<int> sc(B), sp(B);
    for (size_t k0 = 0; k0 < classes.size(); k0 += per) {
        const int nc = (int)std::min<size_t>(per, classes.size() - k0);
        int maxsize = 1;
        for (int i = 0; i < nc; ++i) {
            const int cl = classes[k0 + i];
            for (int j = 0; j < 12; ++j) {
                sc[12 * i + j] = cl;
                sp[12 * i + j] = j;
            }
            maxsize = std::max(maxsize, point ? 1 : c->cptr[cl + 1] - c->cptr[cl]);
        }
        HIPCHK(hipMemcpyAsync(w.slot_class.p, sc.data(), sizeof(int) * 12 * nc, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(w.slot_comp.p, sp.data(), sizeof(int) * 12 * nc, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(w.batch_classes.p, classes.data() + k0, sizeof(int) * nc, hipMemcpyHostToDevice,
                              c->stream));
        Source src{colour, w.slot_class.as<int>(), w.slot_comp.as<int>(), nullptr};
        const int dk = inverse ? 0 : c->defl_k;
        if (dk > 0) {
            c->defl_coef.ensure(sizeof(double2) * (size_t)B * dk);
            launch_defl_coef_probe(c->geom(), c->defl_u.as<double2>(), dk, w.slot_class.as<int>(),
                                   w.slot_comp.as<int>(), cptr, csites, 12 * nc, c->defl_coef.as<double2>(),
                                   c->stream);
            src.du = c->defl_u.as<double2>();
            src.dcoef = c->defl_coef.as<double2>();
            src.dk = dk;
        }
        const double t0 = now_s();
        BatchResult r = run_batch(c, prec, 12 * nc, src, st);
        const double t1 = now_s();
        launch_contract(c->geom(), c->U64.as<double2>(), w.y.as<double2>(), c->kappa, w.batch_classes.as<int>(), nc,
                        maxsize, cptr, csites, c->qx.as<double>(), c->qxi.as<double>(), inverse,
                        c->defl_w.as<double2>(), c->defl_coef.as<double2>(), dk, c->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(c->stream));
        if (c->trace)
            std::fprintf(stderr, "smpq: batch of %d sources on V = %d: %lld iterations (max %lld), %.3f s solve\n",
                         12 * nc, c->V, r.iters_sum, r.iters_max, t1 - t0);
        if (st) {
            st->t_solve_s += t1 - t0;
            st->t_contract_s += now_s() - t1;
            st->n_sources += 12 * nc;
            st->n_batches += 1;
            st->total_iters += r.iters_sum;
            st->max_iters = std::max<int64_t>(st->max_iters, r.iters_max);
        }
    }
}

void prepare_q(smpq_ctx *c, smpq_stats *st) {
    need_device(c);
    if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
    auto_zolo(c, st);
    c->qx.ensure(sizeof(double) * c->V);
    c->qxi.ensure(sizeof(double) * c->V);
    HIPCHK(hipMemsetAsync(c->qx.p, 0, sizeof(double) * c->V, c->stream));
    HIPCHK(hipMemsetAsync(c->qxi.p, 0, sizeof(double) * c->V, c->stream));
    if (st) {
        st->lam_min = c->zolo.lam_min;
        st->lam_max = c->zolo.lam_max;
        st->zolo_delta = c->zolo.delta;
    }
}

void finish_q(smpq_ctx *c, double *qx, double *qxi, smpq_stats *st) {
    const double t0 = now_s();
    std::vector<double> hi(c->V);
    HIPCHK(hipMemcpy(qx, c->qx.p, sizeof(double) * c->V, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hi.data(), c->qxi.p, sizeof(double) * c->V, hipMemcpyDeviceToHost));
    if (qxi) std::memcpy(qxi, hi.data(), sizeof(double) * c->V);
    if (st) {
        double sum = 0.0, mx = 0.0;
        for (double v : hi) {
            sum += v;
            mx = std::max(mx, std::fabs(v));
        }
        st->sum_imag_q = sum;
        st->max_abs_imag_q = mx;
        st->t_contract_s += now_s() - t0;
    }
}

// Checked class list of the context's scheme; classes == NULL with n < 0 means every class.
std::vector<int> class_list(const smpq_ctx *c, const int32_t *classes, int n) {
    if (!c->have_scheme) throw Fail{SMPQ_ESTATE, "no scheme set"};
    if (!classes && n < 0) {
        std::vector<int> all(c->n_classes);
        for (int i = 0; i < c->n_classes; ++i) all[i] = i;
        return all;
    }
    if (n < 0 || (!classes && n > 0)) throw Fail{SMPQ_EINVAL, "bad class list"};
    std::vector<int> cls(classes, classes + n);
    std::vector<char> seen(c->n_classes, 0);
    for (int v : cls) {
        if (v < 0 || v >= c->n_classes) throw Fail{SMPQ_EINVAL, "class index out of range"};
        if (seen[v]++) throw Fail{SMPQ_EINVAL, "duplicate class index"};
    }
    return cls;
}

// Buffers of the stencil timings: n_sets disjoint (input, output[, aux]) sets of n_rhs vectors
// and link copies, allocated and cleared once and kept while the layout (precision, sets,
// right-hand sides, pair) stays the same, so that an autotuning sweep does not allocate per
// candidate.
struct StencilBench {
    int p = -1, n_rhs = 0, n_sets = 0;
    bool pair = false;
    std::vector<DevMem> vecs, links;
    DevMem part, alpha, status;   // pair: the partials, alpha = 0 and status OK per right-hand side
};

// Mean duration of the stencil (D_W, epilogue 0) on n_rhs right-hand sides, rotating through
// n_sets disjoint input/output/link sets; *bytes = algorithmic bytes per launch.  With pair, one
// timed unit is the solver's pair: D_W with the <p, (H^2 + sigma) p> partials (epilogue 3), then
// D_W^dag + sigma with the in-place residual update (epilogue 2, alpha = 0 so r keeps its
// values but is read and written), and *bytes covers both launches.  n_rhs is lowered where the
// buffers would take more than half of the free device memory.
// mode 0: D_W alone (no epilogue); 1: the solver's pair, D_W p with the partials of
// <p, (H^2 + s) p> (epilogue 3) then D_W^dag with r -= alpha (H^2 + s) p (epilogue 2); 2 and 3:
// the first or the second of the pair alone.  Returns ms per launch (per pair in mode 1).
double time_dslash(smpq_ctx *c, StencilBench &tb, int p, int n_rhs, int n_sets, int launches, double *bytes,
                   int mode = 0) {
    const bool pair = mode != 0;   // buffers of the pair
    const Geom g = c->geom();
    const size_t units = p == 0 ? 12 : 6;
    const size_t vbytes = units * 16 * c->vs;
    const size_t lbytes = (size_t)c->V * (p == 0 ? 72 * 8 : 48 * 4);
    const int nvec = pair ? 3 : 2;   // pair: p, tmp, r
    if (!(tb.p == p && tb.n_sets == n_sets && tb.pair == pair && tb.n_rhs > 0 && tb.n_rhs <= n_rhs)) {
        tb.vecs.clear();
        tb.links.clear();
        tb.part.release();
        tb.alpha.release();
        tb.status.release();
        tb.p = -1;
        size_t freeb = 0, totalb = 0;
        HIPCHK(hipMemGetInfo(&freeb, &totalb));
        const size_t per_rhs = nvec * vbytes * n_sets + (pair ? sizeof(double) * partial_stride(g) : 0);
        if (freeb / 2 < lbytes * n_sets + per_rhs)
            throw Fail{SMPQ_ENOMEM, "not enough device memory to time the stencil"};
        const int fit = (int)std::min<size_t>(n_rhs, (freeb / 2 - lbytes * n_sets) / per_rhs);
        tb.vecs = std::vector<DevMem>((size_t)nvec * n_sets);
        tb.links = std::vector<DevMem>(n_sets);
        if (pair) {
            tb.part.ensure(sizeof(double) * partial_stride(g) * fit);
            tb.alpha.ensure(sizeof(double) * fit);
            tb.status.ensure(sizeof(int) * fit);
            HIPCHK(hipMemsetAsync(tb.alpha.p, 0, sizeof(double) * fit, c->stream));
            HIPCHK(hipMemsetAsync(tb.status.p, 0, sizeof(int) * fit, c->stream));   // kStatusOK
        }
        for (int k = 0; k < n_sets; ++k) {
            for (int v = 0; v < nvec; ++v) {
                tb.vecs[(size_t)k * nvec + v].ensure(vbytes * fit);
                HIPCHK(hipMemsetAsync(tb.vecs[(size_t)k * nvec + v].p, 0, vbytes * fit, c->stream));
            }
            tb.links[k].ensure(lbytes);
            HIPCHK(hipMemcpyAsync(tb.links[k].p, p == 0 ? c->U64.p : c->U32.p, lbytes, hipMemcpyDeviceToDevice,
                                  c->stream));
        }
        tb.p = p;
        tb.n_rhs = fit;
        tb.n_sets = n_sets;
        tb.pair = pair;
    }
    n_rhs = std::min(n_rhs, tb.n_rhs);
    Slots sl{nullptr, nullptr, n_rhs};
    const size_t st = units * c->vs;
    auto one = [&](int i) {
        const int k = i % n_sets;
        void *a = tb.vecs[(size_t)k * nvec].p, *b = tb.vecs[(size_t)k * nvec + 1].p;
        if (!pair) {
            launch_dslash(p, false, 0, tb.links[k].p, a, st, 0, b, st, nullptr, 0, 0, g, c->kappa, 0.0, sl, n_rhs,
                          nullptr, c->stream);
            return;
        }
        if (mode != 3)
            launch_dslash(p, false, 3, tb.links[k].p, a, st, 0, b, st, nullptr, 0, 0, g, c->kappa, 0.1, sl, n_rhs,
                          tb.part.as<double>(), c->stream);
        if (mode != 2)
            launch_dslash(p, true, 2, tb.links[k].p, b, st, 0, tb.vecs[(size_t)k * nvec + 2].p, st, a, st, 0, g,
                          c->kappa, 0.1, sl, n_rhs, tb.part.as<double>(), c->stream, tb.alpha.as<double>(),
                          tb.status.as<int>());
    };
    for (int i = 0; i < n_sets; ++i) one(i);   // warm-up
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, c->stream));
    for (int i = 0; i < launches; ++i) one(i);
    HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    const double u = p == 0 ? 16.0 : 8.0;
    *bytes = (double)c->V * ((double)lbytes / c->V + (double)n_rhs * 24.0 * u);
    // the pair: + the aux read (p) and the r read; the second stencil alone: D_W plus those
    if (mode == 1) *bytes = 2.0 * *bytes + (double)c->V * n_rhs * 24.0 * u;
    if (mode == 3) *bytes = *bytes + (double)c->V * n_rhs * 24.0 * u;
    return t / launches;
}

}  // namespace

// =============================================================================== C ABI
extern "C" {

const char *smpq_strerror(smpq_status s) {
    switch (s) {
        case SMPQ_OK: return "ok";
        case SMPQ_EINVAL: return "invalid argument";
        case SMPQ_EDIM: return "dimension mismatch";
        case SMPQ_ENOMEM: return "out of memory";
        case SMPQ_EDEVICE: return "device error";
        case SMPQ_ENOCONV: return "solver did not converge";
        case SMPQ_ESTATE: return "call out of order";
        case SMPQ_ENUMERIC: return "numerical error";
    }
    return "unknown status";
}

const char *smpq_last_error(const smpq_ctx *c) { return c ? c->err.c_str() : "null context"; }

smpq_status smpq_create(const int dims[4], int device, smpq_ctx **out) {
    if (!dims || !out) return SMPQ_EINVAL;
    *out = nullptr;
    long long V = 1;
    for (int i = 0; i < 4; ++i) {
        if (dims[i] < 1) return SMPQ_EDIM;
        V *= dims[i];
    }
    if (V >= (1LL << 31) / 16) return SMPQ_EDIM;
    smpq_ctx *c = new smpq_ctx();
    std::memcpy(c->dims, dims, sizeof(int) * 4);
    c->V = (int)V;
    c->vs = (size_t)((V + 255) / 256) * 256;
    c->device = device;
    if (dims[0] * dims[1] == 256) {
        c->f32_kind = c->f32_dag_kind = 1;
        c->f32_nr = c->f32_dag_nr = 8;
    } else if (tile_rows(dims[0], dims[1]) > 0) {
        c->f32_kind = c->f32_dag_kind = 2;
        c->f32_nr = c->f32_dag_nr = 8;
    }
    if (device >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
            (void)hipGetLastError();
            delete c;
            return SMPQ_EDEVICE;
        }
        if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc((void **)&c->h_count, sizeof(int) * 4) != hipSuccess || !scratch_address(device)) {
            (void)hipGetLastError();
            delete c;
            return SMPQ_EDEVICE;
        }
        c->stream = c->own;
    }
    *out = c;
    return SMPQ_OK;
}

void smpq_destroy(smpq_ctx *c) {
    if (!c) return;
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        if (c->stream) (void)hipStreamSynchronize(c->stream);
    }
    hipStream_t own = c->own;
    int *hc = c->h_count;
    int dev = c->device;
    for (auto &row : c->graphs)
        for (auto &gx : row)
            if (gx) (void)hipGraphExecDestroy(gx);
    delete c;
    if (dev >= 0) {
        if (hc) (void)hipHostFree(hc);
        if (own) (void)hipStreamDestroy(own);
    }
}

smpq_status smpq_load_gauge(smpq_ctx *c, const double *U, size_t n) {
    return guarded(c, [&] {
        if (!U) throw Fail{SMPQ_EINVAL, "null gauge pointer"};
        if (n != (size_t)72 * c->V) throw Fail{SMPQ_EDIM, "gauge field must hold 72*V doubles"};
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(U[i])) throw Fail{SMPQ_ENUMERIC, "non-finite gauge link entry"};
        for (size_t l = 0; l < (size_t)4 * c->V; ++l) {
            const double *u = U + 18 * l;
            double err = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double re = 0.0, im = 0.0;   // (U^dag U)_ab = sum_k conj(U_ka) U_kb
                    for (int k = 0; k < 3; ++k) {
                        const double ar = u[2 * (3 * k + a)], ai = u[2 * (3 * k + a) + 1];
                        const double br = u[2 * (3 * k + b)], bi = u[2 * (3 * k + b) + 1];
                        re += ar * br + ai * bi;
                        im += ar * bi - ai * br;
                    }
                    err = std::max(err, std::hypot(re - (a == b), im));
                }
            // det by cofactor expansion along the first row
            auto C = [&](int r, int k) { return std::pair<double, double>(u[2 * (3 * r + k)], u[2 * (3 * r + k) + 1]); };
            auto mul = [](std::pair<double, double> x, std::pair<double, double> y) {
                return std::pair<double, double>(x.first * y.first - x.second * y.second,
                                                 x.first * y.second + x.second * y.first);
            };
            auto sub = [](std::pair<double, double> x, std::pair<double, double> y) {
                return std::pair<double, double>(x.first - y.first, x.second - y.second);
            };
            auto m0 = sub(mul(C(1, 1), C(2, 2)), mul(C(1, 2), C(2, 1)));
            auto m1 = sub(mul(C(1, 0), C(2, 2)), mul(C(1, 2), C(2, 0)));
            auto m2 = sub(mul(C(1, 0), C(2, 1)), mul(C(1, 1), C(2, 0)));
            auto det = mul(C(0, 0), m0);
            auto t1 = mul(C(0, 1), m1), t2 = mul(C(0, 2), m2);
            det.first += -t1.first + t2.first;
            det.second += -t1.second + t2.second;
            if (err > 1e-10 || std::hypot(det.first - 1.0, det.second) > 1e-10)
                throw Fail{SMPQ_ENUMERIC, "gauge link is not in SU(3) (|U^dag U - 1| or |det U - 1| > 1e-10)"};
        }
        need_device(c);
        const size_t V = c->V;
        // FP64: all nine entries [mu][k][site]; FP32: rows 0 and 1, [mu][j][site] float4
        std::vector<double> u64(V * 72);
        std::vector<float> u32(V * 48);
        for (size_t s = 0; s < V; ++s)
            for (int mu = 0; mu < 4; ++mu)
                for (int k = 0; k < 9; ++k) {
                    const double *src = U + ((s * 4 + mu) * 9 + k) * 2;
                    const size_t d = ((size_t)(mu * 9 + k) * V + s) * 2;
                    u64[d] = src[0];
                    u64[d + 1] = src[1];
                    if (k < 6) {
                        const size_t f = ((size_t)(mu * 3 + k / 2) * V + s) * 4 + 2 * (k % 2);
                        u32[f] = (float)src[0];
                        u32[f + 1] = (float)src[1];
                    }
                }
        c->U64.ensure(sizeof(double) * V * 72);
        c->U32.ensure(sizeof(float) * V * 48);
        HIPCHK(hipMemcpy(c->U64.p, u64.data(), sizeof(double) * V * 72, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->U32.p, u32.data(), sizeof(float) * V * 48, hipMemcpyHostToDevice));
        uint64_t h = 0xcbf29ce484222325ull;   // FNV-1a, 64 bit
        const unsigned char *bytes = reinterpret_cast<const unsigned char *>(U);
        for (size_t i = 0; i < n * sizeof(double); ++i) h = (h ^ bytes[i]) * 0x100000001b3ull;
        c->gauge_hash = h;
        c->have_gauge = true;
        drop_deflation(c);   // eigenvectors of the previous operator
        c->gen++;
    });
}

smpq_status smpq_set_kappa(smpq_ctx *c, double kappa) {
    return guarded(c, [&] {
        if (!(kappa > 0.0 && kappa < 0.25)) throw Fail{SMPQ_EINVAL, "kappa must be in (0, 0.25)"};
        c->kappa = kappa;
        drop_deflation(c);
        c->gen++;
    });
}

smpq_status smpq_lanczos(smpq_ctx *c, int steps, uint64_t seed, double *tmin, double *tmax) {
    return guarded(c, [&] {
        if (steps < 2 || !tmin || !tmax) throw Fail{SMPQ_EINVAL, "need steps >= 2 and output pointers"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        lanczos(c, steps, seed, tmin, tmax);
    });
}

smpq_status smpq_estimate_bounds(smpq_ctx *c, int steps, double *lo, double *hi) {
    return guarded(c, [&] {
        if (steps < 2 || !lo || !hi) throw Fail{SMPQ_EINVAL, "need steps >= 2 and output pointers"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        double tmin, tmax;
        lanczos(c, steps, 0, &tmin, &tmax);
        *lo = 0.9 * std::sqrt(tmin);
        *hi = 1.02 * std::sqrt(tmax);
    });
}

smpq_status smpq_set_zolotarev(smpq_ctx *c, int n, double lo, double hi) {
    return guarded(c, [&] {
        if (c->device >= 0) HIPCHK(hipSetDevice(c->device));
        set_zolo(c, n, lo, hi);
    });
}

smpq_status smpq_get_zolotarev(const smpq_ctx *cc, int *n, double *c0, double *cv, double *q, double *delta) {
    smpq_ctx *c = const_cast<smpq_ctx *>(cc);
    return guarded(c, [&] {
        if (!c->have_zolo) throw Fail{SMPQ_ESTATE, "no Zolotarev coefficients set"};
        if (n) *n = c->zolo.n;
        if (c0) *c0 = c->zolo.c0;
        if (cv) std::memcpy(cv, c->zolo.c.data(), sizeof(double) * c->zolo.n);
        if (q) std::memcpy(q, c->zolo.q.data(), sizeof(double) * c->zolo.n);
        if (delta) *delta = c->zolo.delta;
    });
}

smpq_status smpq_set_solver(smpq_ctx *c, smpq_precision prec, double tol, int max_iter, int reliable) {
    return guarded(c, [&] {
        if (prec < SMPQ_FP64 || prec > SMPQ_MIXED_BF16VEC) throw Fail{SMPQ_EINVAL, "unknown precision"};
        if (!(tol > 0.0 && tol < 1.0)) throw Fail{SMPQ_EINVAL, "tol must be in (0, 1)"};
        if (max_iter < 1) throw Fail{SMPQ_EINVAL, "max_iter must be >= 1"};
        if (reliable < 0 || reliable % kGroup != 0)
            throw Fail{SMPQ_EINVAL, "reliable_interval must be 0 or a positive multiple of " + std::to_string(kGroup) +
                                        " (the solver runs in groups of that many iterations)"};
        c->prec = prec;
        c->tol = tol;
        c->max_iter = max_iter;
        c->reliable = reliable;
        c->gen++;
    });
}

smpq_status smpq_get_settings(const smpq_ctx *cc, smpq_settings *out) {
    smpq_ctx *c = const_cast<smpq_ctx *>(cc);
    return guarded(c, [&] {
        if (!out) throw Fail{SMPQ_EINVAL, "null output"};
        out->kappa = c->kappa;
        out->precision = (int)c->prec;
        out->tol = c->tol;
        out->max_iter = c->max_iter;
        out->reliable_interval = c->reliable;
        out->gauge_hash = c->have_gauge ? c->gauge_hash : 0;
    });
}

smpq_status smpq_set_shift_check(smpq_ctx *c, int enable, double refine_tol) {
    return guarded(c, [&] {
        if (enable != 0 && enable != 1) throw Fail{SMPQ_EINVAL, "enable must be 0 or 1"};
        if (!std::isfinite(refine_tol) || refine_tol >= 1.0)
            throw Fail{SMPQ_EINVAL, "refine_tol must be finite and below 1 (<= 0: check only)"};
        c->shift_check = enable == 1;
        c->refine_tol = refine_tol;
        c->gen++;
    });
}

smpq_status smpq_set_batch(smpq_ctx *c, int max_rhs) {
    return guarded(c, [&] {
        if (max_rhs < 0) throw Fail{SMPQ_EINVAL, "max_rhs must be >= 0"};
        c->max_rhs = max_rhs >= 12 ? (max_rhs / 12) * 12 : max_rhs;
    });
}

static void install_scheme(smpq_ctx *c, std::vector<int32_t> &&col, int ncls) {
    c->colour = std::move(col);
    c->n_classes = ncls;
    c->cptr.assign(ncls + 1, 0);
    for (int v : c->colour) c->cptr[v + 1]++;
    for (int i = 0; i < ncls; ++i) c->cptr[i + 1] += c->cptr[i];
    c->csites.assign(c->V, 0);
    std::vector<int> fill(c->cptr.begin(), c->cptr.end() - 1);
    for (int s = 0; s < c->V; ++s) c->csites[fill[c->colour[s]]++] = s;
    c->have_scheme = true;
    c->d_colour.release();
    c->d_cptr.release();
    c->d_csites.release();
}

smpq_status smpq_set_scheme(smpq_ctx *c, const int r[4], int mode, int *ncls, int *nsrc) {
    return guarded(c, [&] {
        if (!r) throw Fail{SMPQ_EINVAL, "null gap array"};
        std::vector<int32_t> col;
        std::string err;
        const int n = make_colouring(c->dims, r, mode, col, err);
        if (n < 0) throw Fail{mode < 0 || mode > 2 ? SMPQ_EINVAL : SMPQ_EDIM, err};
        install_scheme(c, std::move(col), n);
        if (ncls) *ncls = n;
        if (nsrc) *nsrc = 12 * n;
    });
}

smpq_status smpq_set_point_scheme(smpq_ctx *c, int *ncls, int *nsrc) {
    return guarded(c, [&] {
        std::vector<int32_t> col(c->V);
        for (int s = 0; s < c->V; ++s) col[s] = s;
        install_scheme(c, std::move(col), c->V);
        if (ncls) *ncls = c->V;
        if (nsrc) *nsrc = 12 * c->V;
    });
}

smpq_status smpq_get_coloring(const smpq_ctx *cc, int32_t *colour) {
    smpq_ctx *c = const_cast<smpq_ctx *>(cc);
    return guarded(c, [&] {
        if (!colour) throw Fail{SMPQ_EINVAL, "null output"};
        if (!c->have_scheme) throw Fail{SMPQ_ESTATE, "no scheme set"};
        std::memcpy(colour, c->colour.data(), sizeof(int32_t) * c->V);
    });
}

smpq_status smpq_get_scheme_rmin(const smpq_ctx *cc, double *r_min, int *nearest) {
    smpq_ctx *c = const_cast<smpq_ctx *>(cc);
    return guarded(c, [&] {
        if (!c->have_scheme) throw Fail{SMPQ_ESTATE, "no scheme set"};
        // every class of the three modes is a coset of one sublattice, so the distances
        // from site 0 to the other sites of its class are those of any class
        long long best = -1;
        int cnt = 0;
        for (int s = 1; s < c->V; ++s) {
            if (c->colour[s] != c->colour[0]) continue;
            long long d2 = 0;
            int t = s;
            for (int mu = 0; mu < 4; ++mu) {
                const int x = t % c->dims[mu];
                t /= c->dims[mu];
                const int d = std::min(x, c->dims[mu] - x);
                d2 += (long long)d * d;
            }
            if (best < 0 || d2 < best) {
                best = d2;
                cnt = 1;
            } else if (d2 == best) {
                ++cnt;
            }
        }
        if (r_min) *r_min = best < 0 ? 0.0 : std::sqrt((double)best);
        if (nearest) *nearest = best < 0 ? 0 : cnt;
    });
}

smpq_status smpq_apply_dw(smpq_ctx *c, const double *in, double *out, int n, int dagger, smpq_precision prec) {
    return guarded(c, [&] {
        if (!in || !out || n < 1) throw Fail{SMPQ_EINVAL, "need input, output and n_rhs >= 1"};
        if (prec != SMPQ_FP64 && prec != SMPQ_MIXED_FP32) throw Fail{SMPQ_EINVAL, "unknown precision"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        const Geom g = c->geom();
        const size_t v64 = 12 * 16 * c->vs, v32 = 6 * 16 * c->vs;
        std::vector<double> stage;
        spinor_to_device(c, in, n, stage);
        DevMem a, b, a32, b32;
        a.ensure(v64 * n);
        b.ensure(v64 * n);
        HIPCHK(hipMemcpyAsync(a.p, stage.data(), v64 * n, hipMemcpyHostToDevice, c->stream));
        Slots sl{nullptr, nullptr, n};
        if (prec == SMPQ_FP64) {
            launch_dslash(0, dagger != 0, 0, c->U64.p, a.p, 12 * c->vs, 0, b.p, 12 * c->vs, nullptr, 0, 0, g,
                          c->kappa, 0.0, sl, n, nullptr, c->stream);
        } else {
            a32.ensure(v32 * n);
            b32.ensure(v32 * n);
            launch_convert(1, g, a.p, a32.p, n, c->stream);
            launch_dslash(1, dagger != 0, 0, c->U32.p, a32.p, 6 * c->vs, 0, b32.p, 6 * c->vs, nullptr, 0, 0, g,
                          c->kappa, 0.0, sl, n, nullptr, c->stream);
            launch_convert(0, g, b32.p, b.p, n, c->stream);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(stage.data(), b.p, v64 * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        spinor_from_device(c, stage, n, out);
    });
}

// The same as smpq_apply_dw without allocating: host input and output go through the device's
// fixed scratch array (the host layout is converted on the device), and the staging vectors
// live there too.  Calls that overlap on one GPU share that array and race.
static size_t noalloc_dw_bytes_per_rhs(const smpq_ctx *c, smpq_precision prec) {
    const size_t aos = (size_t)c->V * 12 * sizeof(double2), v64 = 12 * 16 * c->vs, v32 = 6 * 16 * c->vs;
    return aos + 2 * v64 + (prec == SMPQ_FP64 ? 0 : 2 * v32);
}

smpq_status smpq_apply_dw_noalloc(smpq_ctx *c, const double *in, double *out, int n, int dagger,
                                  smpq_precision prec) {
    return guarded(c, [&] {
        if (!in || !out || n < 1) throw Fail{SMPQ_EINVAL, "need input, output and n_rhs >= 1"};
        if (prec != SMPQ_FP64 && prec != SMPQ_MIXED_FP32) throw Fail{SMPQ_EINVAL, "unknown precision"};
        const size_t per = noalloc_dw_bytes_per_rhs(c, prec);
        if ((size_t)n > kScratchBytes / per)
            throw Fail{SMPQ_EDIM, std::to_string(n) + " right-hand sides of " + std::to_string(per) +
                                      " bytes each exceed the allocation-free call's scratch of " +
                                      std::to_string(kScratchBytes >> 20) + " MiB (at most " +
                                      std::to_string(kScratchBytes / per) + " here)"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        unsigned char *base = static_cast<unsigned char *>(scratch_ptr[c->device]);
        if (!base) throw Fail{SMPQ_EDEVICE, "no scratch address for this device"};
        const Geom g = c->geom();
        const size_t aos = (size_t)c->V * 12 * sizeof(double2), v64 = 12 * 16 * c->vs, v32 = 6 * 16 * c->vs;
        double2 *h = reinterpret_cast<double2 *>(base);                  // host layout, in and out
        double2 *a = reinterpret_cast<double2 *>(base + n * aos);        // [slot][12][vs] FP64
        double2 *b = reinterpret_cast<double2 *>(base + n * (aos + v64));
        void *a32 = base + n * (aos + 2 * v64), *b32 = base + n * (aos + 2 * v64 + v32);
        HIPCHK(hipMemcpyAsync(h, in, aos * n, hipMemcpyHostToDevice, c->stream));
        launch_layout(true, g, h, a, n, c->stream);
        Slots sl{nullptr, nullptr, n};
        if (prec == SMPQ_FP64) {
            launch_dslash(0, dagger != 0, 0, c->U64.p, a, 12 * c->vs, 0, b, 12 * c->vs, nullptr, 0, 0, g, c->kappa,
                          0.0, sl, n, nullptr, c->stream);
        } else {
            launch_convert(1, g, a, a32, n, c->stream);
            launch_dslash(1, dagger != 0, 0, c->U32.p, a32, 6 * c->vs, 0, b32, 6 * c->vs, nullptr, 0, 0, g, c->kappa,
                          0.0, sl, n, nullptr, c->stream);
            launch_convert(0, g, b32, b, n, c->stream);
        }
        launch_layout(false, g, b, h, n, c->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out, h, aos * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    });
}

smpq_status smpq_apply_dw_dev(smpq_ctx *c, const double *in_dev, double *out_dev, int n, int dagger,
                              smpq_precision prec) {
    return guarded(c, [&] {
        if (!in_dev || !out_dev || n < 1) throw Fail{SMPQ_EINVAL, "need input, output and n_rhs >= 1"};
        if (prec != SMPQ_FP64 && prec != SMPQ_MIXED_FP32) throw Fail{SMPQ_EINVAL, "unknown precision"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        const Geom g = c->geom();
        const size_t v64 = 12 * 16 * c->vs, v32 = 6 * 16 * c->vs;
        DevMem a, b, a32, b32;
        a.ensure(v64 * n);
        b.ensure(v64 * n);
        launch_layout(true, g, reinterpret_cast<const double2 *>(in_dev), a.as<double2>(), n, c->stream);
        Slots sl{nullptr, nullptr, n};
        if (prec == SMPQ_FP64) {
            launch_dslash(0, dagger != 0, 0, c->U64.p, a.p, 12 * c->vs, 0, b.p, 12 * c->vs, nullptr, 0, 0, g,
                          c->kappa, 0.0, sl, n, nullptr, c->stream);
        } else {
            a32.ensure(v32 * n);
            b32.ensure(v32 * n);
            launch_convert(1, g, a.p, a32.p, n, c->stream);
            launch_dslash(1, dagger != 0, 0, c->U32.p, a32.p, 6 * c->vs, 0, b32.p, 6 * c->vs, nullptr, 0, 0, g,
                          c->kappa, 0.0, sl, n, nullptr, c->stream);
            launch_convert(0, g, b32.p, b.p, n, c->stream);
        }
        launch_layout(false, g, b.as<double2>(), reinterpret_cast<double2 *>(out_dev), n, c->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(c->stream));   // the staging vectors are freed on return
    });
}

smpq_status smpq_apply_dov(smpq_ctx *c, const double *in, double *out, int n) {
    return guarded(c, [&] {
        if (!in || !out || n < 1) throw Fail{SMPQ_EINVAL, "need input, output and n_rhs >= 1"};
        need_device(c);
        require_gauge_zolo(c);
        const int prec = (int)c->prec;
        use_coef(c, false);
        const int NS = c->zolo.n;
        const Geom g = c->geom();
        const size_t v64 = 12 * 16 * c->vs;
        std::vector<double> stage;
        spinor_to_device(c, in, n, stage);
        DevMem bin, bout, defl_part;
        bin.ensure(v64 * n);
        bout.ensure(v64 * n);
        HIPCHK(hipMemcpyAsync(bin.p, stage.data(), v64 * n, hipMemcpyHostToDevice, c->stream));
        const int B = choose_batch(c, prec, NS, n, false);
        ensure_workspace(c, prec, NS, B);
        for (int k0 = 0; k0 < n; k0 += B) {
            const int nb = std::min(B, n - k0);
            const double2 *bptr = bin.as<double2>() + (size_t)k0 * 12 * c->vs;
            Source src{nullptr, nullptr, nullptr, bptr};
            const int dk = c->defl_k;
            if (dk > 0) {   // coefficients <u_i, b> of every right-hand side of the batch
                c->defl_coef.ensure(sizeof(double2) * (size_t)B * dk);
                defl_part.ensure(sizeof(double) * 2 * (size_t)dk * unit_parts(0, g));
                for (int j = 0; j < nb; ++j)
                    launch_multi_dot(g, c->defl_u.as<double2>(), 12 * c->vs, dk, bptr + (size_t)j * 12 * c->vs,
                                     defl_part.as<double>(), c->defl_coef.as<double2>() + (size_t)j * dk, c->stream);
                src.du = c->defl_u.as<double2>();
                src.dcoef = c->defl_coef.as<double2>();
                src.dk = dk;
            }
            run_batch(c, prec, nb, src, nullptr);
            // D_ov b = b + gamma5 eps b = b + D_W y   (eps b = gamma5 D_W y)
            Slots sl{nullptr, nullptr, nb};
            launch_dslash(0, false, 1, c->U64.p, c->ws.y.p, 12 * c->vs, 0,
                          bout.as<double2>() + (size_t)k0 * 12 * c->vs, 12 * c->vs, bptr, 12 * c->vs, 0, g, c->kappa,
                          1.0, sl, nb, c->ws.partial.as<double>(), c->stream);
            if (dk > 0)
                launch_add_defl(g, bout.as<double2>() + (size_t)k0 * 12 * c->vs, c->defl_w.as<double2>(), dk,
                                c->defl_coef.as<double2>(), nb, c->stream);
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipMemcpyAsync(stage.data(), bout.p, v64 * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        spinor_from_device(c, stage, n, out);
    });
}

smpq_status smpq_deflate(smpq_ctx *c, int n_modes, int steps, double *theta, double *theta_max, double *max_resid) {
    return guarded(c, [&] {
        if (n_modes < 0 || n_modes > SMPQ_MAX_DEFLATED) throw Fail{SMPQ_EINVAL, "n_modes out of range"};
        if (n_modes == 0) {
            drop_deflation(c);
            c->gen++;
            return;
        }
        if (steps <= n_modes) throw Fail{SMPQ_EINVAL, "need steps > n_modes"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        deflate(c, n_modes, steps, theta, theta_max, max_resid);
    });
}

smpq_status smpq_compute_qx(smpq_ctx *c, double *qx, double *qxi, double *Q, smpq_stats *st) {
    return guarded(c, [&] {
        if (!qx) throw Fail{SMPQ_EINVAL, "null output"};
        if (!c->have_scheme) throw Fail{SMPQ_ESTATE, "no scheme set"};
        if (st) std::memset(st, 0, sizeof(*st));
        prepare_q(c, st);
        ensure_scheme_device(c);
        std::vector<int> cls(c->n_classes);
        for (int i = 0; i < c->n_classes; ++i) cls[i] = i;
        qx_classes(c, cls, false, st);
        finish_q(c, qx, qxi, st);
        if (Q) {
            double s = 0.0;
            for (int i = 0; i < c->V; ++i) s += qx[i];
            *Q = s;
        }
    });
}

smpq_status smpq_compute_qx_dev(smpq_ctx *c, double *qx_dev, double *qxi_dev, double *Q, smpq_stats *st) {
    return guarded(c, [&] {
        if (!qx_dev) throw Fail{SMPQ_EINVAL, "null output"};
        if (!c->have_scheme) throw Fail{SMPQ_ESTATE, "no scheme set"};
        if (st) std::memset(st, 0, sizeof(*st));
        prepare_q(c, st);
        ensure_scheme_device(c);
        std::vector<int> cls(c->n_classes);
        for (int i = 0; i < c->n_classes; ++i) cls[i] = i;
        qx_classes(c, cls, false, st);
        // the map stays on the device: copies into the caller's buffers on the context's stream;
        // Q and the statistics from a host copy, summed as smpq_compute_qx sums them
        const size_t bytes = sizeof(double) * c->V;
        HIPCHK(hipMemcpyAsync(qx_dev, c->qx.p, bytes, hipMemcpyDeviceToDevice, c->stream));
        if (qxi_dev) HIPCHK(hipMemcpyAsync(qxi_dev, c->qxi.p, bytes, hipMemcpyDeviceToDevice, c->stream));
        std::vector<double> h(c->V);
        finish_q(c, h.data(), nullptr, st);
        if (Q) {
            double s = 0.0;
            for (int i = 0; i < c->V; ++i) s += h[i];
            *Q = s;
        }
    });
}

smpq_status smpq_compute_qx_classes(smpq_ctx *c, const int32_t *classes, int n, double *qx, double *qxi,
                                    smpq_stats *st) {
    return guarded(c, [&] {
        if (!qx || (!classes && n > 0) || n < 0) throw Fail{SMPQ_EINVAL, "bad class list or output"};
        const std::vector<int> cls = class_list(c, classes, n);
        if (st) std::memset(st, 0, sizeof(*st));
        prepare_q(c, st);
        ensure_scheme_device(c);
        qx_classes(c, cls, false, st);
        finish_q(c, qx, qxi, st);
    });
}

smpq_status smpq_set_memory_limit(smpq_ctx *c, size_t bytes) {
    return guarded(c, [&] { c->mem_limit = bytes; });
}

smpq_status smpq_compute_qx_multi(smpq_ctx *const *ctxs, int n_ctx, const int32_t *const *classes,
                                  const int *n_classes, double *const *qx, double *const *qxi, smpq_stats *st,
                                  int *failed) {
    if (failed) *failed = -1;
    if (n_ctx < 1 || !ctxs || !qx || (classes && !n_classes)) return SMPQ_EINVAL;
    for (int k = 0; k < n_ctx; ++k)
        if (!ctxs[k] || !qx[k]) {
            if (failed) *failed = k;
            return SMPQ_EINVAL;
        }
    std::vector<std::vector<int>> cls(n_ctx);
    std::vector<double> work(n_ctx, 0.0);
    std::vector<int> planned(n_ctx, 0);
    auto give_up = [&](int k, smpq_status s) {
        for (int j = 0; j < n_ctx; ++j) ctxs[j]->run_limit = 0;
        if (failed) *failed = k;
        return s;
    };
    // host-side checks of every context first, then the set-up one context after another:
    // bounds, device arrays of the scheme and of the output
    for (int k = 0; k < n_ctx; ++k) {
        smpq_ctx *c = ctxs[k];
        const smpq_status s = guarded(c, [&] {
            for (int j = 0; j < k; ++j) {
                if (ctxs[j] == c) throw Fail{SMPQ_EINVAL, "context listed twice"};
                if (c->stream && ctxs[j]->stream == c->stream) throw Fail{SMPQ_EINVAL, "contexts share a stream"};
            }
            cls[k] = class_list(c, classes ? classes[k] : nullptr, classes && classes[k] ? n_classes[k] : -1);
        });
        if (s != SMPQ_OK) return give_up(k, s);
    }
    for (int k = 0; k < n_ctx; ++k) {
        smpq_ctx *c = ctxs[k];
        const smpq_status s = guarded(c, [&] {
            need_device(c);
            if (c->device != ctxs[0]->device) throw Fail{SMPQ_EINVAL, "contexts on different devices"};
            if (st) std::memset(&st[k], 0, sizeof(smpq_stats));
            prepare_q(c, st ? &st[k] : nullptr);
            ensure_scheme_device(c);
            work[k] = (double)c->V * (double)cls[k].size();
        });
        if (s != SMPQ_OK) return give_up(k, s);
    }
    // device memory: contexts without a limit of their own share 80% of what is free (plus what
    // their workspaces already hold) in proportion to their work, V x classes
    {
        size_t freeb = 0, totalb = 0, held = 0, fixed = 0;
        if (hipSetDevice(ctxs[0]->device) != hipSuccess || hipMemGetInfo(&freeb, &totalb) != hipSuccess)
            return give_up(0, SMPQ_EDEVICE);
        for (int k = 0; k < n_ctx; ++k) {
            held += workspace_bytes(ctxs[k]);
            if (ctxs[k]->mem_limit > 0) fixed += ctxs[k]->mem_limit;
        }
        double pool = std::max(0.0, 0.80 * (double)(freeb + held) - (double)fixed);
        // every context first gets one batch of 12 right-hand sides; the rest goes out in
        // proportion to the work, never beyond what a context can use (all its sources at
        // once), with what a capped context leaves handed on to the others
        std::vector<double> share(n_ctx, 0.0), cap(n_ctx, 0.0), slotb(n_ctx, 0.0);
        std::vector<char> open(n_ctx, 0);
        for (int k = 0; k < n_ctx; ++k) {
            smpq_ctx *c = ctxs[k];
            if (c->mem_limit > 0 || cls[k].empty()) continue;
            const double slot = (double)bytes_per_slot(c, (int)c->prec, c->zolo.n);
            slotb[k] = slot;
            share[k] = 12.0 * slot;
            cap[k] = 12.0 * (double)cls[k].size() * slot;
            pool -= share[k];
            open[k] = 1;
        }
        if (pool < 0.0) return give_up(0, SMPQ_ENOMEM);
        for (int round = 0; round < n_ctx && pool > 0.0; ++round) {
            double wopen = 0.0;
            for (int k = 0; k < n_ctx; ++k)
                if (open[k]) wopen += work[k];
            if (wopen <= 0.0) break;
            double left = 0.0;
            for (int k = 0; k < n_ctx; ++k) {
                if (!open[k]) continue;
                const double add = pool * work[k] / wopen;
                if (share[k] + add >= cap[k]) {
                    left += share[k] + add - cap[k];
                    share[k] = cap[k];
                    open[k] = 0;
                } else {
                    share[k] += add;
                }
            }
            pool = left;
        }
        for (int k = 0; k < n_ctx; ++k) {
            smpq_ctx *c = ctxs[k];
            // half a slot of slack so that rounding cannot drop the last whole slot
            c->run_limit = c->mem_limit > 0 ? c->mem_limit : (size_t)(share[k] + 0.5 * slotb[k]);
        }
        for (int k = 0; k < n_ctx; ++k) {
            smpq_ctx *c = ctxs[k];
            const smpq_status s = guarded(c, [&] {
                const int prec = (int)c->prec;
                if (cls[k].empty()) return;
                planned[k] = choose_batch(c, prec, c->zolo.n, (int)cls[k].size() * 12, true);
                if (c->ws.prec != prec || c->ws.NS != c->zolo.n || c->ws.B != planned[k]) release_workspace(c);
            });
            if (s != SMPQ_OK) return give_up(k, s);
        }
        for (int k = 0; k < n_ctx; ++k) {
            smpq_ctx *c = ctxs[k];
            const smpq_status s = guarded(c, [&] {
                if (planned[k] > 0) ensure_workspace(c, (int)c->prec, c->zolo.n, planned[k]);
                if (planned[k] > 0 && c->defl_k > 0)
                    c->defl_coef.ensure(sizeof(double2) * (size_t)planned[k] * c->defl_k);
            });
            if (s != SMPQ_OK) return give_up(k, s);
        }
    }
    // the solves: one host thread per context, each on the context's own stream
    std::vector<smpq_status> res(n_ctx, SMPQ_OK);
    {
        std::vector<std::thread> th;
        th.reserve(n_ctx);
        for (int k = 0; k < n_ctx; ++k)
            th.emplace_back([&, k] {
                smpq_ctx *c = ctxs[k];
                smpq_stats *sk = st ? &st[k] : nullptr;
                res[k] = guarded(c, [&] {
                    need_device(c);
                    qx_classes(c, cls[k], false, sk);
                    finish_q(c, qx[k], qxi ? qxi[k] : nullptr, sk);
                });
            });
        for (auto &t : th) t.join();
    }
    for (int k = 0; k < n_ctx; ++k) ctxs[k]->run_limit = 0;
    for (int k = 0; k < n_ctx; ++k)
        if (res[k] != SMPQ_OK) {
            if (failed) *failed = k;
            return res[k];
        }
    return SMPQ_OK;
}

smpq_status smpq_compute_trinv(smpq_ctx *c, const int32_t *classes, int n, double *t_re, double *t_im,
                               smpq_stats *st) {
    return guarded(c, [&] {
        if (!t_re) throw Fail{SMPQ_EINVAL, "null output"};
        const std::vector<int> cls = class_list(c, classes, classes ? n : -1);
        if (st) std::memset(st, 0, sizeof(*st));
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        c->qx.ensure(sizeof(double) * c->V);
        c->qxi.ensure(sizeof(double) * c->V);
        HIPCHK(hipMemsetAsync(c->qx.p, 0, sizeof(double) * c->V, c->stream));
        HIPCHK(hipMemsetAsync(c->qxi.p, 0, sizeof(double) * c->V, c->stream));
        ensure_scheme_device(c);
        qx_classes(c, cls, false, st, true);
        finish_q(c, t_re, t_im, st);
    });
}

smpq_status smpq_dov_locality(smpq_ctx *c, int64_t site, double *mean_abs, smpq_stats *st) {
    return guarded(c, [&] {
        if (!mean_abs) throw Fail{SMPQ_EINVAL, "null output"};
        if (site < 0 || site >= c->V) throw Fail{SMPQ_EINVAL, "site index out of range"};
        if (st) std::memset(st, 0, sizeof(*st));
        need_device(c);
        require_gauge_zolo(c);
        const int prec = (int)c->prec;
        use_coef(c, false);
        ensure_point_device(c);
        ensure_workspace(c, prec, c->zolo.n, std::max(12, c->ws.prec == prec && c->ws.NS == c->zolo.n ? c->ws.B : 12));
        Workspace &w = c->ws;
        std::vector<int> sc(12, (int)site), sp(12);
        for (int j = 0; j < 12; ++j) sp[j] = j;
        HIPCHK(hipMemcpyAsync(w.slot_class.p, sc.data(), sizeof(int) * 12, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(w.slot_comp.p, sp.data(), sizeof(int) * 12, hipMemcpyHostToDevice, c->stream));
        Source src{c->d_pcolour.as<int>(), w.slot_class.as<int>(), w.slot_comp.as<int>(), nullptr};
        const double t0 = now_s();
        BatchResult r = run_batch(c, prec, 12, src, st);
        // columns of D_ov: e_j + D_W y_j (gamma5 eps e_j = D_W y_j)
        const Geom g = c->geom();
        DevMem d, m;
        d.ensure((size_t)12 * 12 * 16 * c->vs);
        m.ensure(sizeof(double) * c->V);
        launch_dslash(0, false, 0, c->U64.p, w.y.p, 12 * c->vs, 0, d.p, 12 * c->vs, nullptr, 0, 0, g, c->kappa, 0.0,
                      Slots{nullptr, nullptr, 12}, 12, nullptr, c->stream);
        launch_block_mean_abs(g, d.as<double2>(), (int)site, m.as<double>(), c->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(mean_abs, m.p, sizeof(double) * c->V, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (st) {
            st->t_solve_s = now_s() - t0;
            st->n_sources = 12;
            st->n_batches = 1;
            st->total_iters = r.iters_sum;
            st->max_iters = r.iters_max;
        }
    });
}

smpq_status smpq_compute_qx_points(smpq_ctx *c, const int64_t *sites, int n, double *qx, smpq_stats *st) {
    return guarded(c, [&] {
        if ((!sites && n > 0) || !qx || n < 0) throw Fail{SMPQ_EINVAL, "bad site list or output"};
        std::vector<int> cls(n);
        std::vector<char> seen(c->V, 0);
        for (int i = 0; i < n; ++i) {
            if (sites[i] < 0 || sites[i] >= c->V) throw Fail{SMPQ_EINVAL, "site index out of range"};
            if (seen[sites[i]]++) throw Fail{SMPQ_EINVAL, "duplicate site"};
            cls[i] = (int)sites[i];
        }
        if (st) std::memset(st, 0, sizeof(*st));
        prepare_q(c, st);
        ensure_point_device(c);
        qx_classes(c, cls, true, st);
        std::vector<double> all(c->V);
        finish_q(c, all.data(), nullptr, st);
        for (int i = 0; i < n; ++i) qx[i] = all[sites[i]];
    });
}

smpq_status smpq_prepare(smpq_ctx *c) {
    return guarded(c, [&] {
        need_device(c);
        require_gauge_zolo(c);
        if (!c->have_scheme) throw Fail{SMPQ_ESTATE, "no scheme set"};
        const int prec = (int)c->prec;
        const int B = choose_batch(c, prec, c->zolo.n, 12 * c->n_classes, true);
        ensure_workspace(c, prec, c->zolo.n, B);
        ensure_scheme_device(c);
    });
}

smpq_status smpq_set_stream(smpq_ctx *c, void *stream) {
    return guarded(c, [&] {
        need_device(c);
        HIPCHK(hipStreamSynchronize(c->stream));
        c->stream = stream ? static_cast<hipStream_t>(stream) : c->own;
        c->gen++;
    });
}

smpq_status smpq_set_timing(smpq_ctx *c, int enable) {
    return guarded(c, [&] { c->timing = enable != 0; });
}

smpq_status smpq_set_graphs(smpq_ctx *c, int enable) {
    return guarded(c, [&] { c->use_graphs = enable != 0; });
}

smpq_status smpq_bench_dslash(smpq_ctx *c, smpq_precision prec, int n_rhs, int n_sets, int launches, double *ms,
                              double *bytes) {
    return guarded(c, [&] {
        if (n_rhs < 1 || n_sets < 1 || launches < 1 || !ms || !bytes) throw Fail{SMPQ_EINVAL, "bad arguments"};
        if (prec != SMPQ_FP64 && prec != SMPQ_MIXED_FP32) throw Fail{SMPQ_EINVAL, "unknown precision"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        StencilBench tb;
        *ms = time_dslash(c, tb, prec == SMPQ_FP64 ? 0 : 1, n_rhs, n_sets, launches, bytes);
    });
}

smpq_status smpq_bench_copy(smpq_ctx *c, size_t bytes, int launches, double *ms) {
    return guarded(c, [&] {
        if (bytes == 0 || launches < 1 || !ms) throw Fail{SMPQ_EINVAL, "bad arguments"};
        need_device(c);
        DevMem a, b;
        a.ensure(bytes);
        b.ensure(bytes);
        HIPCHK(hipMemsetAsync(a.p, 0, bytes, c->stream));
        HIPCHK(hipMemcpyAsync(b.p, a.p, bytes, hipMemcpyDeviceToDevice, c->stream));   // warm-up
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, c->stream));
        for (int i = 0; i < launches; ++i)
            HIPCHK(hipMemcpyAsync(i & 1 ? a.p : b.p, i & 1 ? b.p : a.p, bytes, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipEventRecord(e1, c->stream));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms = t / launches;
    });
}

smpq_status smpq_bench_stream(smpq_ctx *c, size_t bytes, int launches, int nontemporal, double *ms) {
    return guarded(c, [&] {
        if (bytes < 16 || launches < 1 || !ms || (nontemporal != 0 && nontemporal != 1))
            throw Fail{SMPQ_EINVAL, "need bytes >= 16, launches >= 1, nontemporal 0 or 1 and an output"};
        need_device(c);
        const size_t n = bytes / 16;
        DevMem a, b;
        a.ensure(n * 16);
        b.ensure(n * 16);
        HIPCHK(hipMemsetAsync(a.p, 0, n * 16, c->stream));
        HIPCHK(hipMemsetAsync(b.p, 0, n * 16, c->stream));
        launch_stream_copy(nontemporal == 1, a.p, b.p, n, c->stream);   // warm-up
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, c->stream));
        for (int i = 0; i < launches; ++i)
            launch_stream_copy(nontemporal == 1, i % 2 ? b.p : a.p, i % 2 ? a.p : b.p, n, c->stream);
        HIPCHK(hipEventRecord(e1, c->stream));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(hipGetLastError());
        *ms = t / launches;
    });
}

smpq_status smpq_set_tuning(smpq_ctx *c, const smpq_tuning *t) {
    return guarded(c, [&] {
        if (!t) throw Fail{SMPQ_EINVAL, "null tuning"};
        const smpq_tuning keep = c->tuning();
        c->set_tuning(*t);
        const Geom g = c->geom();
        if (!valid_tuning(0, g) || !valid_tuning(1, g)) {
            c->set_tuning(keep);
            throw Fail{SMPQ_EINVAL, "unsupported stencil variant for this lattice"};
        }
        c->gen++;
    });
}

smpq_status smpq_get_tuning(smpq_ctx *c, smpq_tuning *t) {
    return guarded(c, [&] {
        if (!t) throw Fail{SMPQ_EINVAL, "null tuning"};
        *t = c->tuning();
    });
}

smpq_status smpq_autotune(smpq_ctx *c, int n_rhs, smpq_tuning *chosen) {
    return guarded(c, [&] {
        if (n_rhs < 0) throw Fail{SMPQ_EINVAL, "n_rhs must be >= 0"};
        need_device(c);
        if (!c->have_gauge) throw Fail{SMPQ_ESTATE, "no gauge field loaded"};
        if (n_rhs == 0) {   // the batch a whole q(x) map of the current scheme would use
            if (c->n_classes == 0) throw Fail{SMPQ_ESTATE, "n_rhs = 0 needs a probing scheme"};
            if (!c->have_zolo) throw Fail{SMPQ_ESTATE, "n_rhs = 0 needs the Zolotarev coefficients"};
            n_rhs = choose_batch(c, (int)c->prec, c->zolo.n, 12 * c->n_classes, true);
        }
        double by;
        struct Cand {
            int kind, nr, band, il;
        };
        std::vector<Cand> cand = {{0, 2, 1, 1}, {0, 4, 1, 1}, {0, 8, 1, 1}};
        const Geom g0 = c->geom();
        for (int kind = 1; kind <= 4; ++kind) {
            if (kind == 2 || kind == 4 ? g0.tile_y == 0 : !plane_tileable(g0)) continue;
            for (int nr : kind == 4 ? std::vector<int>{1, 2, 4, 8} : std::vector<int>{4, 8, 16})
                for (int band : {1, 2, 4})
                    // interleaving pays with few right-hand sides per block (measured: 1 or 2)
                    for (int il : kind == 4 ? std::vector<int>{1, 2, 4} : std::vector<int>{1})
                        if (c->dims[2] % band == 0 && (il == 1 || nr * il <= 4)) cand.push_back({kind, nr, band, il});
        }
        const smpq_tuning keep = c->tuning();
        StencilBench tb;   // one set of timing buffers per precision for the whole sweep
        try {
            // FP32: the two stencils of an iteration (D_W p with its partials, D_W^dag with the
            // residual update) are timed alone and chosen separately; the plane band is shared,
            // so the band with the smallest sum of the two best times wins
            struct Best {
                double t3 = INFINITY, t2 = INFINITY;
                Cand k3{}, k2{};
            };
            Best per_band[5];
            double by3 = 0.0, by2 = 0.0;
            for (const Cand &k : cand) {
                c->f32_kind = c->f32_dag_kind = k.kind;
                c->f32_nr = c->f32_dag_nr = k.nr;
                c->band = k.band;
                c->f32_il = c->f32_dag_il = k.il;
                const double t3 = std::min(time_dslash(c, tb, 1, n_rhs, 2, 10, &by3, 2),
                                           time_dslash(c, tb, 1, n_rhs, 2, 10, &by3, 2));
                const double t2 = std::min(time_dslash(c, tb, 1, n_rhs, 2, 10, &by2, 3),
                                           time_dslash(c, tb, 1, n_rhs, 2, 10, &by2, 3));
                if (c->trace)
                    std::fprintf(stderr, "smpq: autotune FP32 kind %d, %d per block/thread, band %d, interleave %d: "
                                 "D_W %.3f ms (%.0f GB/s), D_W^dag %.3f ms (%.0f GB/s) on %d right-hand sides\n",
                                 k.kind, k.nr, k.band, k.il, t3, by3 / t3 * 1e-6, t2, by2 / t2 * 1e-6,
                                 std::min(n_rhs, tb.n_rhs));
                Best &b = per_band[k.band];
                if (t3 < b.t3) {
                    b.t3 = t3;
                    b.k3 = k;
                }
                if (t2 < b.t2) {
                    b.t2 = t2;
                    b.k2 = k;
                }
            }
            int band = 1;
            for (int bb : {2, 4})
                if (per_band[bb].t3 + per_band[bb].t2 < per_band[band].t3 + per_band[band].t2) band = bb;
            const Best &b = per_band[band];
            if (!std::isfinite(b.t3 + b.t2)) throw Fail{SMPQ_EDEVICE, "no FP32 stencil variant could be timed"};
            c->band = band;
            c->f32_kind = b.k3.kind;
            c->f32_nr = b.k3.nr;
            c->f32_il = b.k3.il;
            c->f32_dag_kind = b.k2.kind;
            c->f32_dag_nr = b.k2.nr;
            c->f32_dag_il = b.k2.il;
            // FP64: lanes interleaving 1, 2 or 4 right-hand sides; xy-tiles with 2, 4 or 8 per
            // block (same plane order band as the FP32 choice) where a tile fits
            double best = INFINITY;
            struct Cand64 {
                int kind, lgr, nr, il;
            };
            std::vector<Cand64> c64 = {{0, 0, 4, 1}, {0, 1, 4, 1}, {0, 2, 4, 1}};
            if (g0.tile_y > 0 && c->dims[2] % c->band == 0)
                for (int nr : {1, 2, 4, 8})
                    for (int il : {1, 2, 4})
                        if (il == 1 || nr * il <= 8) c64.push_back({1, keep.f64_lgr, nr, il});
            Cand64 p64{keep.f64_kind, keep.f64_lgr, keep.f64_nr, keep.f64_interleave};
            for (const Cand64 &k : c64) {
                c->f64_kind = k.kind;
                c->f64_lgr = k.lgr;
                c->f64_nr = k.nr;
                c->f64_il = k.il;
                const double t = std::min(time_dslash(c, tb, 0, n_rhs, 2, 10, &by, 1),
                                          time_dslash(c, tb, 0, n_rhs, 2, 10, &by, 1));
                if (c->trace)
                    std::fprintf(stderr, "smpq: autotune FP64 kind %d, lanes 2^%d / %d per block, interleave %d: "
                                 "%.3f ms per pair (%.0f GB/s) on %d right-hand sides\n", k.kind, k.lgr, k.nr, k.il, t,
                                 by / t * 1e-6, std::min(n_rhs, tb.n_rhs));
                if (t < best) {
                    best = t;
                    p64 = k;
                }
            }
            c->f64_kind = p64.kind;
            c->f64_lgr = p64.lgr;
            c->f64_nr = p64.nr;
            c->f64_il = p64.il;
        } catch (...) {
            c->set_tuning(keep);
            throw;
        }
        c->gen++;   // captured graphs used the previous variants
        if (chosen) *chosen = c->tuning();
    });
}

}  // extern "C"
