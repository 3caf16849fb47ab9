// Host driver and C ABI of libch (declared in include/ch.h).
//
// A run keeps its state in two library-owned FP64 buffers (ping-pong); the
// caller's field is copied in at the start and the last accepted state is
// copied back at the end, so a failing step never touches the caller's data.
// All step control lives in the device control block (Ctl): a run of EE2 steps
// is issued without host synchronisation, except where the number of launches
// depends on device data (LIM's Chebyshev order p, restarted Krylov cycles of a
// constant step) and a periodic check for t >= T when no step limit is given.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

#include "ch_internal.h"

struct ch_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuffers b{};
    size_t v_bytes = 0;      // bytes allocated for the Krylov basis
    size_t state_n = 0;      // points allocated for the FP64 state buffers
    size_t y32_n = 0;
    size_t z_n = 0;
    int rec_cap = 0;
    int cycle_id = 0;        // id of the last issued Krylov cycle
    int* hflag = nullptr;    // pinned, device-mapped: last finished cycle id
    Ctl* hctl = nullptr;     // pinned mirror of the control block
    std::string err;
};

namespace {

#define HIP_TRY(ctx, call)                                          \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) {                                     \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_); \
            return CH_EDEVICE;                                      \
        }                                                           \
    } while (0)

int alloc_dev(ch_ctx* ctx, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        ctx->err = std::string("hipMalloc: ") + hipGetErrorString(e);
        (void)hipGetLastError();
        return CH_ENOMEM;
    }
    return CH_OK;
}

void free_dev(void* p) {
    if (p) (void)hipFree(p);
}

int check_problem(const ch_problem* p, Grid* g) {
    if (!p) return CH_EINVAL;
    if (p->dim != 2 && p->dim != 3) return CH_EINVAL;
    if (p->n < 5) return CH_EINVAL;
    if (!(p->eps > 0.0) || !(p->eps < INFINITY)) return CH_EINVAL;
    if (p->eyre != 0 && p->eyre != 1) return CH_EINVAL;
    if (p->prec != CH_FP64 && p->prec != CH_FP32_MIXED) return CH_EINVAL;
    long long N = 1;
    for (int d = 0; d < p->dim; ++d) N *= p->n;
    if (N >= (1LL << 31)) return CH_EINVAL;
    g->dim = p->dim;
    g->n = p->n;
    g->N = N;
    g->eps2 = p->eps * p->eps;
    g->inv_h2 = double(p->n) * double(p->n);
    g->eyre = p->eyre;
    return CH_OK;
}

// Size the workspace for N points, a basis of m_max + 1 columns in `prec`,
// `recs` step records and (optionally) the LIM stage buffer.
int ensure(ch_ctx* ctx, long long N, int m_max, int prec, int recs, bool need_z) {
    DevBuffers& b = ctx->b;
    int rc;
    if (!b.ctl) {
        if ((rc = alloc_dev(ctx, (void**)&b.ctl, sizeof(Ctl)))) return rc;
        if ((rc = alloc_dev(ctx, (void**)&b.part, 2 * sizeof(double) * CH_NRED * CH_MAXB))) return rc;
        HIP_TRY(ctx, hipHostMalloc((void**)&ctx->hctl, sizeof(Ctl), hipHostMallocDefault));
        HIP_TRY(ctx, hipHostMalloc((void**)&ctx->hflag, 64, hipHostMallocMapped | hipHostMallocCoherent));
        *ctx->hflag = -1;
        HIP_TRY(ctx, hipHostGetDevicePointer((void**)&b.dflag, ctx->hflag, 0));
        b.hflag = ctx->hflag;
    }
    if ((size_t)N > ctx->state_n) {
        free_dev(b.ybuf[0]);
        free_dev(b.ybuf[1]);
        free_dev(b.fcur);
        b.ybuf[0] = b.ybuf[1] = b.fcur = nullptr;
        ctx->state_n = 0;
        for (double** p : {&b.ybuf[0], &b.ybuf[1], &b.fcur})
            if ((rc = alloc_dev(ctx, (void**)p, sizeof(double) * N))) return rc;
        ctx->state_n = N;
    }
    if (m_max > 0) {
        const size_t ldv = ((size_t)N + 63) / 64 * 64;
        const size_t esz = prec == CH_FP64 ? sizeof(double) : sizeof(float);
        const size_t bytes = (size_t)(m_max + 1) * ldv * esz;
        if (bytes > ctx->v_bytes) {
            free_dev(b.V);
            b.V = nullptr;
            ctx->v_bytes = 0;
            if ((rc = alloc_dev(ctx, &b.V, bytes))) return rc;
            ctx->v_bytes = bytes;
        }
        b.ldv = ldv;
        if (prec == CH_FP32_MIXED && (size_t)N > ctx->y32_n) {
            free_dev(b.y32);
            b.y32 = nullptr;
            ctx->y32_n = 0;
            if ((rc = alloc_dev(ctx, (void**)&b.y32, sizeof(float) * N))) return rc;
            ctx->y32_n = N;
        }
    }
    if (need_z && (size_t)N > ctx->z_n) {
        free_dev(b.zbuf);
        b.zbuf = nullptr;
        ctx->z_n = 0;
        if ((rc = alloc_dev(ctx, (void**)&b.zbuf, sizeof(double) * N))) return rc;
        ctx->z_n = N;
    }
    if (recs > ctx->rec_cap) {
        free_dev(b.rec);
        b.rec = nullptr;
        ctx->rec_cap = 0;
        if ((rc = alloc_dev(ctx, (void**)&b.rec, sizeof(ch_step_record) * recs))) return rc;
        ctx->rec_cap = recs;
    }
    return CH_OK;
}

void init_ctl(Ctl* c, int mode, double t0, double tau0, double T, double tol, double tol_phi_fixed, double tau_min,
              int m_max, int rec_cap) {
    memset(c, 0, sizeof(Ctl));
    c->mode = mode;
    c->t = t0;
    c->tau = tau0;
    c->tau_fixed = tau0;
    c->T = T;
    c->tol = tol;
    c->tol_phi_fixed = tol_phi_fixed;
    c->tau_min = tau_min;
    c->m_max = m_max;
    c->rec_cap = rec_cap;
}

// Bytes of the control block's scalar head (everything before the Arnoldi arrays).
constexpr size_t CTL_HEAD = offsetof(Ctl, H);

int read_head(ch_ctx* ctx) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->hctl, ctx->b.ctl, CTL_HEAD, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

// Remaining Krylov cycles of a constant step (linear RT restarts, reading in
// the oracle's header): re-start from the current sub-step state `z` with the
// residual of the frozen problem, until a cycle converges on the rest of tau.
int restart_cycles(ch_ctx* ctx, const Grid& g, int prec, PartSeq& ps, const double* y, double* z, int m_max) {
    const DevBuffers& b = ctx->b;
    for (int cyc = 0; cyc < 100000; ++cyc) {
        int rc = read_head(ctx);
        if (rc) return rc;
        const Ctl& h = *ctx->hctl;
        if (h.halted || h.converged) return CH_OK;
        HIP_TRY(ctx, launch_cycle_begin(b, ctx->stream));
        HIP_TRY(ctx, launch_resid(g, prec, b, ps, y, z, false, false, ctx->stream));
        HIP_TRY(ctx, launch_after_resid(b, ps, false, ctx->stream));
        HIP_TRY(ctx, launch_arnoldi(g, prec, b, ps, y, m_max, ++ctx->cycle_id, ctx->stream));
        HIP_TRY(ctx, launch_update(g, prec, b, z, z, ctx->stream));
    }
    ctx->err = "restart cycle limit reached";
    return CH_ETAU_UNDERFLOW;
}

void fill_stats(const Ctl& h, ch_run_stats* st) {
    if (!st) return;
    st->t = h.t;
    st->tau_next = h.tau;
    st->steps = h.steps;
    st->matvecs = h.matvecs;
    st->restarts = h.restarts;
    st->traces = h.traces;
    st->status = h.status;
}

int finish_run(ch_ctx* ctx, long long N, double* y, ch_run_stats* stats, ch_step_record* records, int max_rec) {
    int rc = read_head(ctx);
    if (rc) return rc;
    const Ctl h = *ctx->hctl;
    HIP_TRY(ctx, hipMemcpyAsync(y, ctx->b.ybuf[h.cur], sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
    const int nrec = std::min(h.steps, max_rec);
    if (records && nrec > 0)
        HIP_TRY(ctx, hipMemcpyAsync(records, ctx->b.rec, sizeof(ch_step_record) * nrec, hipMemcpyDeviceToHost,
                                    ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    fill_stats(h, stats);
    return h.status;
}

int run_ee(ch_ctx* ctx, const ch_problem* prob, double* y, double tau0, double t0, double T, int max_steps,
           const ch_ee_opts* opts, ch_run_stats* stats, ch_step_record* records) {
    Grid g;
    int rc = check_problem(prob, &g);
    if (rc) return rc;
    if (!y || !opts) return CH_EINVAL;
    if (opts->m_max < 1 || opts->m_max > CH_MMAX) return CH_EINVAL;
    if (!(tau0 > 0.0) || !(opts->tau_min >= 0.0)) return CH_EINVAL;
    if (!(opts->tol > 0.0) && !(opts->tol_phi_fixed > 0.0)) return CH_EINVAL;
    if (max_steps <= 0 && !(T < INFINITY)) return CH_EINVAL;
    if (!(t0 < INFINITY)) return CH_EINVAL;
    const int prec = prob->prec;
    const int recs = (records && max_steps > 0) ? max_steps : 0;
    if ((rc = ensure(ctx, g.N, opts->m_max, prec, recs, false))) return rc;
    const DevBuffers& b = ctx->b;
    const bool constant = opts->constant_step != 0;
    init_ctl(ctx->hctl, constant ? MODE_EE_CONST : MODE_EE, t0, tau0, T, opts->tol, opts->tol_phi_fixed,
             opts->tau_min, opts->m_max, recs);
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.ybuf[0], y, sizeof(double) * g.N, hipMemcpyDeviceToDevice, ctx->stream));
    PartSeq ps;
    ps.base = b.part;
    HIP_TRY(ctx, launch_resid(g, prec, b, ps, b.ybuf[0], b.ybuf[0], true, true, ctx->stream));
    HIP_TRY(ctx, launch_after_resid(b, ps, true, ctx->stream));
    for (long long s = 0;; ++s) {
        if (max_steps > 0 && s >= max_steps) break;
        const double* yin = b.ybuf[s & 1];
        double* yout = b.ybuf[(s + 1) & 1];
        HIP_TRY(ctx, launch_arnoldi(g, prec, b, ps, yin, opts->m_max, ++ctx->cycle_id, ctx->stream));
        HIP_TRY(ctx, launch_update(g, prec, b, yin, yout, ctx->stream));
        if (constant && (rc = restart_cycles(ctx, g, prec, ps, yin, yout, opts->m_max))) return rc;
        HIP_TRY(ctx, launch_est_ee(g, prec, b, ps, yin, yout, ctx->stream));
        HIP_TRY(ctx, launch_step_end(b, ps, true, ctx->stream));
        if (max_steps <= 0 && (s % 16) == 15) {
            if ((rc = read_head(ctx))) return rc;
            if (ctx->hctl->halted) break;
        }
    }
    return finish_run(ctx, g.N, y, stats, records, recs);
}

int run_lim(ch_ctx* ctx, const ch_problem* prob, double* y, double tau0, double t0, double T, int max_steps,
            double tol, ch_run_stats* stats, ch_step_record* records) {
    Grid g;
    int rc = check_problem(prob, &g);
    if (rc) return rc;
    if (!y || !(tau0 > 0.0)) return CH_EINVAL;
    if (max_steps <= 0 && !(T < INFINITY)) return CH_EINVAL;
    const int recs = (records && max_steps > 0) ? max_steps : 0;
    if ((rc = ensure(ctx, g.N, 0, CH_FP64, recs, true))) return rc;
    const DevBuffers& b = ctx->b;
    init_ctl(ctx->hctl, tol > 0.0 ? MODE_LIM : MODE_LIM_CONST, t0, tau0, T, tol, 0.0, 0.0, 0, recs);
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.ybuf[0], y, sizeof(double) * g.N, hipMemcpyDeviceToDevice, ctx->stream));
    PartSeq ps;
    ps.base = b.part;
    for (long long s = 0;; ++s) {
        if (max_steps > 0 && s >= max_steps) break;
        const double* yin = b.ybuf[s & 1];
        double* yout = b.ybuf[(s + 1) & 1];
        HIP_TRY(ctx, launch_lim_begin(g, b, ps, yin, ctx->stream));
        HIP_TRY(ctx, launch_lim_plan(g, b, ps, ctx->stream));
        if ((rc = read_head(ctx))) return rc;
        if (ctx->hctl->halted) break;
        const int p = ctx->hctl->p;
        // 2p - 1 stages (m = 1..p, then m = 2..p) ping-pong between zbuf and
        // yout so that the last one lands in yout.
        const int nst = 2 * p - 1;
        const double* src = yin;
        for (int q = 0; q < nst; ++q) {
            const int m = q < p ? q + 1 : q - p + 2;
            double* dst = ((nst - 1 - q) % 2 == 0) ? yout : b.zbuf;
            HIP_TRY(ctx, launch_lim_stage(g, b, yin, src, dst, m, ctx->stream));
            src = dst;
        }
        HIP_TRY(ctx, launch_est_lim(g, b, ps, yin, yout, ctx->stream));
        HIP_TRY(ctx, launch_lim_end(b, ps, ctx->stream));
    }
    return finish_run(ctx, g.N, y, stats, records, recs);
}

void record_from_head(const Ctl& h, ch_step_record* out) {
    if (!out) return;
    memset(out, 0, sizeof(*out));
    out->t = h.t;
    out->tau = h.covered + h.tau_acc;
    out->tau_next = h.tau;
    out->tol_phi = h.tol_phi;
    out->beta = h.beta;
    out->resnorm = h.resnorm;
    out->j = h.j;
    out->cycles = h.cycles;
    out->traced = h.traced;
    out->matvecs = h.mv_step + 1 + h.j;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int ch_create(ch_ctx** out, int device, void* hip_stream) {
    if (!out) return CH_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return CH_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return CH_EDEVICE;
    ch_ctx* ctx = new (std::nothrow) ch_ctx();
    if (!ctx) return CH_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    *out = ctx;
    return CH_OK;
}

int ch_destroy(ch_ctx* ctx) {
    if (!ctx) return CH_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    DevBuffers& b = ctx->b;
    for (void* p : {(void*)b.V, (void*)b.ybuf[0], (void*)b.ybuf[1], (void*)b.fcur, (void*)b.y32, (void*)b.zbuf,
                    (void*)b.part, (void*)b.ctl, (void*)b.rec})
        free_dev(p);
    if (ctx->hctl) (void)hipHostFree(ctx->hctl);
    if (ctx->hflag) (void)hipHostFree(ctx->hflag);
    delete ctx;
    return CH_OK;
}

const char* ch_strerror(int status) {
    switch (status) {
        case CH_OK: return "ok";
        case CH_EINVAL: return "invalid argument";
        case CH_ENOMEM: return "device memory allocation failed";
        case CH_ENONFINITE: return "non-finite value in the field or in a step";
        case CH_ETAU_UNDERFLOW: return "residual-time trace found no admissible step";
        case CH_EBUSY: return "queue full";
        case CH_ENOENT: return "unknown ticket";
        case CH_EDEVICE: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* ch_last_error_message(ch_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int ch_run_ee(ch_ctx* ctx, const ch_problem* prob, double* y, double tau0, double t0, double T, int max_steps,
              const ch_ee_opts* opts, ch_run_stats* stats, ch_step_record* records) {
    if (!ctx) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    return run_ee(ctx, prob, y, tau0, t0, T, max_steps, opts, stats, records);
}

int ch_step_ee(ch_ctx* ctx, const ch_problem* prob, double* y, double tau, double t, double T,
               const ch_ee_opts* opts, ch_step_record* out) {
    ch_run_stats st;
    ch_step_record rec;
    memset(&rec, 0, sizeof(rec));
    const int rc = ch_run_ee(ctx, prob, y, tau, t, T, 1, opts, &st, &rec);
    if (out) *out = rec;
    return rc;
}

int ch_run_lim(ch_ctx* ctx, const ch_problem* prob, double* y, double tau0, double t0, double T, int max_steps,
               double tol, ch_run_stats* stats, ch_step_record* records) {
    if (!ctx) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    return run_lim(ctx, prob, y, tau0, t0, T, max_steps, tol, stats, records);
}

int ch_step_lim(ch_ctx* ctx, const ch_problem* prob, double* y, double tau, double t, double T, double tol,
                ch_step_record* out) {
    ch_run_stats st;
    ch_step_record rec;
    memset(&rec, 0, sizeof(rec));
    const int rc = ch_run_lim(ctx, prob, y, tau, t, T, 1, tol, &st, &rec);
    if (out) *out = rec;
    return rc;
}

int ch_phiv(ch_ctx* ctx, const ch_problem* prob, const double* y, double* y_out, double tau0, int mode,
            double tol_phi, int m_max, ch_step_record* out) {
    if (!ctx) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    Grid g;
    int rc = check_problem(prob, &g);
    if (rc) return rc;
    if (!y || !y_out || y == y_out) return CH_EINVAL;
    if (!(tau0 > 0.0) || !(tol_phi > 0.0) || m_max < 1 || m_max > CH_MMAX) return CH_EINVAL;
    if (mode != CH_PHI_SHRINK && mode != CH_PHI_RESTART) return CH_EINVAL;
    const int prec = prob->prec;
    if ((rc = ensure(ctx, g.N, m_max, prec, 0, false))) return rc;
    const DevBuffers& b = ctx->b;
    init_ctl(ctx->hctl, MODE_PHI, 0.0, tau0, INFINITY, 0.0, tol_phi, 0.0, m_max, 0);
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    PartSeq ps;
    ps.base = b.part;
    HIP_TRY(ctx, launch_resid(g, prec, b, ps, y, y, false, true, ctx->stream));
    HIP_TRY(ctx, launch_after_resid(b, ps, true, ctx->stream));
    HIP_TRY(ctx, launch_arnoldi(g, prec, b, ps, y, m_max, ++ctx->cycle_id, ctx->stream));
    HIP_TRY(ctx, launch_update(g, prec, b, y, y_out, ctx->stream));
    if (mode == CH_PHI_RESTART && (rc = restart_cycles(ctx, g, prec, ps, y, y_out, m_max))) return rc;
    if ((rc = read_head(ctx))) return rc;
    record_from_head(*ctx->hctl, out);
    return ctx->hctl->status;
}

int ch_time_kernel(ch_ctx* ctx, const ch_problem* prob, int kernel, int m_max, int reps, double* avg_us,
                   double* bytes) {
    if (!ctx || !avg_us || !bytes || reps < 1) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    Grid g;
    int rc = check_problem(prob, &g);
    if (rc) return rc;
    if (m_max < 2 || m_max > CH_MMAX) return CH_EINVAL;
    const int prec = prob->prec;
    const size_t esz = prec == CH_FP64 ? sizeof(double) : sizeof(float);
    const DevBuffers& b = ctx->b;
    if (!b.ctl || ctx->state_n < (size_t)g.N || ctx->v_bytes < (size_t)(m_max + 1) * b.ldv * esz ||
        b.ldv < (size_t)g.N || (prec == CH_FP32_MIXED && ctx->y32_n < (size_t)g.N))
        return CH_EINVAL;   // no run on this problem yet
    // Control block: live, coefficients of a no-op axpy, unit scales.
    HIP_TRY(ctx, hipMemcpyAsync(ctx->hctl, b.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    Ctl& h = *ctx->hctl;
    const int jlast = h.last_j;
    h.done = 0;
    h.halted = 0;
    h.vscale[0] = h.vscale[1] = h.vscale[2] = 1.0;
    h.tol_phi = 1.0;   // phi timing: the convergence branch, no trace
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    // partials slots: zeros in, so the timed axpy coefficient is 0 and the phi
    // kernel sees h_{j+1,j} = 0 (its convergence branch)
    HIP_TRY(ctx, hipMemsetAsync(b.part, 0, 2 * sizeof(double) * CH_NRED * CH_MAXB, ctx->stream));
    const double* y = b.ybuf[0];
    auto launch = [&]() -> hipError_t {
        PartSeq ps;
        ps.base = b.part;
        ps.np = 1;
        switch (kernel) {
            case CH_KERNEL_MGS: return launch_mgs_pass(g, prec, b, ps, 1, 1, ctx->stream);
            case CH_KERNEL_MATVEC: return launch_matvec(g, prec, b, ps, y, 0, ctx->stream);
            default: return launch_phi(b, ps, jlast > 0 ? jlast - 1 : 0, -2, ctx->stream);
        }
    };
    if (kernel != CH_KERNEL_MGS && kernel != CH_KERNEL_MATVEC && kernel != CH_KERNEL_PHI) return CH_EINVAL;
    if (kernel == CH_KERNEL_PHI && jlast < 1) return CH_EINVAL;
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    HIP_TRY(ctx, launch());   // warm
    HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
    for (int r = 0; r < reps; ++r) {
        if (kernel == CH_KERNEL_PHI)   // phi sets `done`; re-arm it between launches
            HIP_TRY(ctx, hipMemsetAsync(&b.ctl->done, 0, sizeof(int), ctx->stream));
        HIP_TRY(ctx, launch());
    }
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_us = 1000.0 * ms / reps;
    const double N = double(g.N);
    const double ysz = prec == CH_FP64 ? 8.0 : 4.0;
    if (kernel == CH_KERNEL_MGS) *bytes = 4.0 * esz * N;                 // read w, v_{i-1}, v_i; write w
    else if (kernel == CH_KERNEL_MATVEC) *bytes = (3.0 * esz + ysz) * N; // read v_k, y, v_1; write w
    else *bytes = 0.0;
    return CH_OK;
}

}  // extern "C"
