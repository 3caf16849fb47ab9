// Host driver and C ABI of libch (declared in include/ch.h).
//
// Every run works on a batch of instances laid out in pooled device arrays
// (a single-field call is a batch of one).  A run keeps each state in two
// library-owned FP64 buffers (ping-pong); the caller's fields are copied in at
// the start and the last accepted states are copied back at the end, so a
// failing step never touches the caller's data.  All step control lives in
// per-instance device control blocks (Ctl): a run of EE2 steps is issued
// without host synchronisation, except where the number of launches depends
// on device data (LIM's Chebyshev order p, restarted Krylov cycles of a
// constant step) and a periodic check for the end of the run.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ch_internal.h"
#include "ch_march.h"

struct ch_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuffers b{};
    size_t v_bytes = 0;      // bytes allocated for the Krylov basis
    size_t pts = 0;          // points allocated for the pooled FP64 state arrays
    size_t y32_pts = 0;
    size_t z_pts = 0;
    int slots = 0;           // control blocks allocated
    size_t rec_n = 0;        // step records allocated
    int phibig_slots = 0;    // slots of the phi scratch of orders above 48
    ch_step_record* rec = nullptr;
    std::vector<int> expect; // per slot: Krylov cycles issued (compared with the device's `cyc`)
    int* hflag = nullptr;    // pinned, device-mapped: `cyc` of the last finished cycle per slot, then
                             // the sequence number of the last DCGS2 update launch begun
    int useq = 0;            // DCGS2 update launches issued (their sequence numbers)
    int lseq = 0;            // LIM plan launches issued (the tags of their pinned orders)
    Ctl* hctl = nullptr;     // pinned mirror of the control blocks
    // instance tables: store 0 serves every run; the server keeps the
    // table of its LIM members in store 1 beside that of its EE members
    struct TableStore {
        Inst* d_inst = nullptr;
        int* d_sb2i = nullptr;
        int* d_cb2i = nullptr;
        int* d_wb2i = nullptr;
        size_t inst_cap = 0, map_cap = 0;
        std::vector<Inst> h_inst;
    } store[2];
    LaunchEnv env{};         // second stream for the DCGS2 phi tests, capture stream, graph switch
    GraphCache graphs;       // captured DCGS2 iterations
    struct ShapeEntry {      // launch shapes set or tuned for (dim, n, prec)
        int dim, n, prec;
        ch_shape s;
    };
    std::vector<ShapeEntry> shapes;
    std::string err;
};

namespace {

#define HIP_TRY(ctx, call)                                                  \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_); \
            return CH_EDEVICE;                                              \
        }                                                                   \
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

size_t pad64(size_t x) { return (x + 63) / 64 * 64; }

struct Shape {
    int dim, n;
    long long N;
    int bc = CH_BC_PERIODIC;
    double length = 1.0;
    int mob = 0;
    double m0 = 1.0, m1 = 0.0;
};

int check_grid(int dim, int n, double eps, int eyre, Shape* sh) {
    if (dim != 2 && dim != 3) return CH_EINVAL;
    if (n < 5) return CH_EINVAL;
    if (!(eps > 0.0) || !(eps < INFINITY)) return CH_EINVAL;
    if (eyre != 0 && eyre != 1) return CH_EINVAL;
    long long N = 1;
    for (int d = 0; d < dim; ++d) N *= n;
    if (N >= (1LL << 31)) return CH_EINVAL;
    sh->dim = dim;
    sh->n = n;
    sh->N = N;
    return CH_OK;
}

bool orth_ok(int orth) { return orth == CH_ORTH_DCGS2 || orth == CH_ORTH_MGS; }

int check_problem(const ch_problem* p, Shape* sh) {
    if (!p) return CH_EINVAL;
    if (p->prec != CH_FP64 && p->prec != CH_FP32_MIXED) return CH_EINVAL;
    if (p->bc != CH_BC_PERIODIC && p->bc != CH_BC_NEUMANN) return CH_EINVAL;
    if (p->bc == CH_BC_NEUMANN && p->dim != 2) return CH_EINVAL;   // the paper's 2-D setting only
    if (!(p->length < INFINITY) || p->length != p->length) return CH_EINVAL;
    if (p->mobility != 0 && p->mobility != 1) return CH_EINVAL;
    if (p->mobility) {   // 2-D periodic; M >= 0 somewhere
        if (p->dim != 2 || p->bc != CH_BC_PERIODIC) return CH_EINVAL;
        if (!(p->mob0 >= 0.0 && p->mob0 < INFINITY) || !(p->mob1 >= 0.0 && p->mob1 < INFINITY) ||
            !(p->mob0 + p->mob1 > 0.0))
            return CH_EINVAL;
    }
    const int rc = check_grid(p->dim, p->n, p->eps, p->eyre, sh);
    if (rc) return rc;
    sh->bc = p->bc;
    sh->length = p->length > 0.0 ? p->length : 1.0;
    sh->mob = p->mobility;
    sh->m0 = p->mobility ? p->mob0 : 1.0;
    sh->m1 = p->mobility ? p->mob1 : 0.0;
    return CH_OK;
}

// Workspace for `pts` pooled points, a basis of m_max + 1 columns in `prec`,
// `nslots` control blocks, `recs` step records and (optionally) the LIM stage buffer.
int ensure(ch_ctx* ctx, size_t pts, int m_max, int prec, int nslots, size_t recs, bool need_z) {
    DevBuffers& b = ctx->b;
    int rc;
    if (!b.part) {
        if ((rc = alloc_dev(ctx, (void**)&b.part, 2 * sizeof(double) * CH_NRED * CH_MAXB))) return rc;
    }
    if (!b.dots) {
        if ((rc = alloc_dev(ctx, (void**)&b.dots, sizeof(double) * CH_DROWS * CH_MAXB))) return rc;
    }
    if (nslots > ctx->slots) {
        free_dev(b.ctl);
        b.ctl = nullptr;
        if (ctx->hctl) (void)hipHostFree(ctx->hctl);
        if (ctx->hflag) (void)hipHostFree(ctx->hflag);
        ctx->hctl = nullptr;
        ctx->hflag = nullptr;
        b.hflag = nullptr;
        b.dflag = nullptr;
        b.hprog = nullptr;
        b.dprog = nullptr;
        b.hseq = nullptr;
        b.hlim = nullptr;
        b.dlim = nullptr;
        ctx->slots = 0;
        if ((rc = alloc_dev(ctx, (void**)&b.ctl, sizeof(Ctl) * nslots))) return rc;
        if (!b.dcount) {
            if ((rc = alloc_dev(ctx, (void**)&b.dcount, sizeof(int)))) return rc;
        }
        free_dev(b.lorder);
        free_dev(b.lcoef);
        b.lorder = nullptr;
        b.lcoef = nullptr;
        if ((rc = alloc_dev(ctx, (void**)&b.lorder, sizeof(int) * CH_PMAX * nslots))) return rc;
        if ((rc = alloc_dev(ctx, (void**)&b.lcoef, sizeof(double) * 4 * CH_PMAX * nslots))) return rc;
        HIP_TRY(ctx, hipHostMalloc((void**)&ctx->hctl, sizeof(Ctl) * nslots, hipHostMallocDefault));
        // the finished-cycle word of every slot, the update-launch progress
        // word, then the LIM order and its tag of every slot
        HIP_TRY(ctx, hipHostMalloc((void**)&ctx->hflag, sizeof(int) * (3 * nslots + 1),
                                   hipHostMallocMapped | hipHostMallocCoherent));
        for (int i = 0; i < 3 * nslots + 1; ++i) ctx->hflag[i] = -1;
        ctx->expect.assign(nslots, 0);
        HIP_TRY(ctx, hipHostGetDevicePointer((void**)&b.dflag, ctx->hflag, 0));
        b.hflag = ctx->hflag;
        b.dprog = b.dflag + nslots;
        b.hprog = ctx->hflag + nslots;
        b.dlim = b.dflag + nslots + 1;
        b.hlim = ctx->hflag + nslots + 1;
        // the device's count of update launches begun restarts with the host's count of those issued
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipMemset(b.dcount, 0, sizeof(int)));
        ctx->useq = 0;
        b.hseq = &ctx->useq;
        ctx->slots = nslots;
    }
    if (pts > ctx->pts) {
        free_dev(b.ybuf[0]);
        free_dev(b.ybuf[1]);
        free_dev(b.fcur);
        b.ybuf[0] = b.ybuf[1] = b.fcur = nullptr;
        ctx->pts = 0;
        for (double** p : {&b.ybuf[0], &b.ybuf[1], &b.fcur})
            if ((rc = alloc_dev(ctx, (void**)p, sizeof(double) * pts))) return rc;
        ctx->pts = pts;
    }
    if (m_max > 0) {
        const size_t ldv = pad64(pts);
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
        if (prec == CH_FP32_MIXED && pts > ctx->y32_pts) {
            free_dev(b.y32);
            b.y32 = nullptr;
            ctx->y32_pts = 0;
            if ((rc = alloc_dev(ctx, (void**)&b.y32, sizeof(float) * pts))) return rc;
            ctx->y32_pts = pts;
        }
    }
    if (m_max > CH_MSMALL && nslots > ctx->phibig_slots) {
        free_dev(b.phibig);
        b.phibig = nullptr;
        ctx->phibig_slots = 0;
        if ((rc = alloc_dev(ctx, &b.phibig, phi_big_bytes() * nslots))) return rc;
        ctx->phibig_slots = nslots;
    }
    if (need_z && pts > ctx->z_pts) {
        free_dev(b.zbuf);
        b.zbuf = nullptr;
        ctx->z_pts = 0;
        if ((rc = alloc_dev(ctx, (void**)&b.zbuf, sizeof(double) * pts))) return rc;
        ctx->z_pts = pts;
    }
    if (recs > ctx->rec_n) {
        free_dev(ctx->rec);
        ctx->rec = nullptr;
        ctx->rec_n = 0;
        if ((rc = alloc_dev(ctx, (void**)&ctx->rec, sizeof(ch_step_record) * recs))) return rc;
        ctx->rec_n = recs;
    }
    return CH_OK;
}

struct Member {
    Shape sh;
    double eps;
    int eyre;
    size_t off;     // pooled offset (points)
    int slot = -1;  // control block (default: the member's index)
};

// Workgroups of one instance: stencil tiles (at most CH_SBLK_MAX, larger
// grids loop) and streaming chunks of 2048 points (at most CH_CBLK_MAX).
void inst_blocks(int dim, int n, long long N, int* sblk, int* cblk) {
    long long tiles;
    if (dim == 2) tiles = (long long)((n + 63) / 64) * ((n + 7) / 8);
    else tiles = (long long)((n + 31) / 32) * ((n + 3) / 4) * ((n + 3) / 4);
    *sblk = (int)std::min<long long>(tiles, CH_SBLK_MAX);
    *cblk = (int)std::max<long long>(1, std::min<long long>((N + 2047) / 2048, CH_CBLK_MAX));
}

// 2-D strip workgroups of one instance: one strip per wave while that takes
// at most CH_WBLK_MAX workgroups; larger grids run STRIP_LOOP_BLOCKS (two per
// CU, all resident at once), each wave looping over its strips.  Against
// CH_WBLK_MAX workgroups with one or two strips per wave, the DCGS2 matvec
// (mean of iterations 1, 15, 29) took 25% less time at 2048^2 FP32, 15% at
// 2048^2 FP64, 23% at 1536^2 FP64 and 6-11% at 3000^2 and 4096^2.
constexpr int STRIP_LOOP_BLOCKS = 512;

int strip_blocks(int n, int vx) {
    const long long waves = strip_count(n, vx);
    const long long wg = (waves + CH_STRIP_WAVES - 1) / CH_STRIP_WAVES;
    return wg > CH_WBLK_MAX ? STRIP_LOOP_BLOCKS : (int)wg;
}

// Columns per lane of the 2-D strip kernels for one grid.
#ifndef CH_STRIP_VX32
#define CH_STRIP_VX32 4
#endif
int strip_vx(int n, int prec) {
    int vx = prec == CH_FP64 ? 2 : CH_STRIP_VX32;
    while (n % vx) vx >>= 1;
    return vx;
}

// Workgroups of the 3-D marching matvec of one instance: one per 64-wide x-y
// block (march_rows high) and run of planes, capped (larger grids loop over
// the work items).
static int march_blocks(int n, int prec) {
    const int my = march_rows(prec);
    const int len = prec == CH_FP64 ? CH_MARCH_L : march_len_fp32(n);
    const long long items = (long long)((n + 63) / 64) * ((n + my - 1) / my) * ((n + len - 1) / len);
    return (int)std::min<long long>(items, CH_WBLK_MAX);
}

// Workgroups of the 2-D strip kernels (dim 2) or the 3-D marching matvec
// (dim 3) of one instance.
int wide_blocks(int dim, int n, int prec) {
    return dim == 2 ? strip_blocks(n, strip_vx(n, prec)) : march_blocks(n, prec);
}

// Instance record of member m (index i) whose workgroup ranges start at
// sblk0, cblk0, wblk0.  prec: the precision of the run's basis (selects the
// strip width).
Inst make_inst(const Member& m, int i, int dim, int prec, int sblk0, int cblk0, int wblk0) {
    Inst I{};
    const int n = m.sh.n;
    int sblk, cblk;
    inst_blocks(dim, n, m.sh.N, &sblk, &cblk);
    I.off = (long long)m.off;
    I.N = m.sh.N;
    I.n = n;
    I.slot = m.slot >= 0 ? m.slot : i;
    I.sblk0 = sblk0;
    I.sblk = sblk;
    I.cblk0 = cblk0;
    I.cblk = cblk;
    I.wblk0 = wblk0;
    I.wblk = wide_blocks(dim, n, prec);
    I.vx = strip_vx(n, prec);
    I.eps2 = m.eps * m.eps;
    const double inv_h = double(n) / m.sh.length;   // h = L / n
    I.inv_h2 = inv_h * inv_h;
    I.eyre = m.eyre;
    I.bc = m.sh.bc;
    I.mob = m.sh.mob;
    return I;
}

// The built-in launch shape of one grid.
ch_shape default_shape(int dim, int n, int prec) {
    long long N = (long long)n * n;
    if (dim == 3) N *= n;
    int sblk, cblk;
    inst_blocks(dim, n, N, &sblk, &cblk);
    ch_shape s;
    s.vx = strip_vx(n, prec);
    s.wblk = wide_blocks(dim, n, prec);
    s.cblk = cblk;
    return s;
}

bool shape_ok(int dim, int n, int prec, const ch_shape& s) {
    if (s.wblk < 1 || s.wblk > CH_WBLK_MAX || s.cblk < 1 || s.cblk > CH_CBLK_MAX) return false;
    if (dim == 2) {
        const int maxvx = prec == CH_FP64 ? 2 : 4;
        if (s.vx < 1 || s.vx > maxvx || (s.vx & (s.vx - 1)) || n % s.vx) return false;
    }
    return true;
}

const ch_shape* find_shape(const ch_ctx* ctx, int dim, int n, int prec) {
    for (const auto& e : ctx->shapes)
        if (e.dim == dim && e.n == n && e.prec == prec) return &e.s;
    return nullptr;
}

// Workgroup ranges of each instance and the block-to-instance maps, kept in
// table store `which` of the context.
int build_table(ch_ctx* ctx, const std::vector<Member>& ms, int dim, int prec, Table* t, int which = 0) {
    const int ni = (int)ms.size();
    ch_ctx::TableStore& ts = ctx->store[which];
    ts.h_inst.assign(ni, Inst{});
    std::vector<int> sb, cb, wb;
    for (int i = 0; i < ni; ++i) {
        Inst& I = ts.h_inst[i];
        I = make_inst(ms[i], i, dim, prec, (int)sb.size(), (int)cb.size(), (int)wb.size());
        if (const ch_shape* sp = find_shape(ctx, dim, ms[i].sh.n, prec)) {
            I.vx = sp->vx;
            I.wblk = sp->wblk;
            I.cblk = sp->cblk;
        }
        sb.insert(sb.end(), I.sblk, i);
        cb.insert(cb.end(), I.cblk, i);
        wb.insert(wb.end(), I.wblk, i);
    }
    if (sb.size() > (size_t)CH_MAXB || cb.size() > (size_t)CH_MAXB || wb.size() > (size_t)CH_MAXB) {
        ctx->err = "batch too large for one launch (workgroup table)";
        return CH_EINVAL;
    }
    int rc;
    if ((size_t)ni > ts.inst_cap) {
        free_dev(ts.d_inst);
        ts.d_inst = nullptr;
        ts.inst_cap = 0;
        if ((rc = alloc_dev(ctx, (void**)&ts.d_inst, sizeof(Inst) * ni))) return rc;
        ts.inst_cap = ni;
    }
    const size_t mneed = std::max(std::max(sb.size(), cb.size()), std::max(wb.size(), (size_t)1));
    if (mneed > ts.map_cap) {
        free_dev(ts.d_sb2i);
        free_dev(ts.d_cb2i);
        free_dev(ts.d_wb2i);
        ts.d_sb2i = ts.d_cb2i = ts.d_wb2i = nullptr;
        ts.map_cap = 0;
        if ((rc = alloc_dev(ctx, (void**)&ts.d_sb2i, sizeof(int) * mneed))) return rc;
        if ((rc = alloc_dev(ctx, (void**)&ts.d_cb2i, sizeof(int) * mneed))) return rc;
        if ((rc = alloc_dev(ctx, (void**)&ts.d_wb2i, sizeof(int) * mneed))) return rc;
        ts.map_cap = mneed;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ts.d_inst, ts.h_inst.data(), sizeof(Inst) * ni, hipMemcpyHostToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ts.d_sb2i, sb.data(), sizeof(int) * sb.size(), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ts.d_cb2i, cb.data(), sizeof(int) * cb.size(), hipMemcpyHostToDevice, ctx->stream));
    if (!wb.empty())
        HIP_TRY(ctx, hipMemcpyAsync(ts.d_wb2i, wb.data(), sizeof(int) * wb.size(), hipMemcpyHostToDevice,
                                    ctx->stream));
    // the host vectors must outlive the asynchronous copies
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    t->inst = ts.d_inst;
    t->sb2i = ts.d_sb2i;
    t->cb2i = ts.d_cb2i;
    t->wb2i = ts.d_wb2i;
    t->ninst = ni;
    t->sgrid = (int)sb.size();
    t->cgrid = (int)cb.size();
    t->wgrid = (int)wb.size();
    t->dim = dim;
    t->hinst = ts.h_inst.data();
    return CH_OK;
}

// cyc0: the slot's count of Krylov cycles issued so far.  The count only
// grows (across runs), so a flag left by an earlier run never matches.
void init_ctl(Ctl* c, int mode, double t0, double tau0, double T, double tol, double tol_phi_fixed, double tau_min,
              int m_max, int max_steps, ch_step_record* rec, int rec_cap, int cyc0) {
    memset(c, 0, sizeof(Ctl));
    c->cyc = cyc0;
    c->mode = mode;
    c->t = t0;
    c->tau = tau0;
    c->tau_fixed = tau0;
    c->T = T;
    c->tol = tol;
    c->tol_phi_fixed = tol_phi_fixed;
    c->tau_min = tau_min;
    c->m_max = m_max;
    c->max_steps = max_steps;
    c->rec = rec;
    c->rec_cap = rec ? rec_cap : 0;
}

// The mobility coefficients of a single-grid run (M = 1 unless the problem sets them).
static void set_mobility(Ctl* c, const Shape& sh) {
    c->mob0 = sh.m0;
    c->mob1 = sh.m1;
}

// Bytes of the control block's scalar head (everything before the Arnoldi arrays).
constexpr size_t CTL_HEAD = offsetof(Ctl, H);

// The heads of the control blocks of slots [lo, hi] into hctl: one strided
// copy (the blocks are contiguous, sizeof(Ctl) apart), then a sync.
int copy_heads_to(ch_ctx* ctx, Ctl* h, const Ctl* d, int lo, int hi) {
    if (hi == lo)
        HIP_TRY(ctx, hipMemcpyAsync(h + lo, d + lo, CTL_HEAD, hipMemcpyDeviceToHost, ctx->stream));
    else if (hi > lo)
        HIP_TRY(ctx, hipMemcpy2DAsync(h + lo, sizeof(Ctl), d + lo, sizeof(Ctl), CTL_HEAD, (size_t)(hi - lo + 1),
                                      hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

int copy_heads(ch_ctx* ctx, int lo, int hi) { return copy_heads_to(ctx, ctx->hctl, ctx->b.ctl, lo, hi); }

int read_heads(ch_ctx* ctx, int n) { return copy_heads(ctx, 0, n - 1); }

bool all_halted(const ch_ctx* ctx, int n) {
    for (int i = 0; i < n; ++i)
        if (!ctx->hctl[i].halted) return false;
    return true;
}

// Remaining Krylov cycles of a constant step of one instance (linear RT
// restarts, reading in the oracle's header): re-start from the current
// sub-step state `z` with the residual of the frozen problem, until a cycle
// converges on the rest of tau.
int restart_cycles(ch_ctx* ctx, const Table& t, int prec, PartSeq& ps, const double* y, double* z, int m_max,
                   int orth) {
    const DevBuffers& b = ctx->b;
    for (int cyc = 0; cyc < 100000; ++cyc) {
        int rc = read_heads(ctx, 1);
        if (rc) return rc;
        const Ctl& h = ctx->hctl[0];
        if (h.halted || h.converged) return CH_OK;
        HIP_TRY(ctx, launch_cycle_begin(t, b, ctx->stream));
        ctx->expect[t.hinst[0].slot] += 1;
        HIP_TRY(ctx, launch_resid(t, prec, b, ps, y, z, false, false, ctx->stream));
        HIP_TRY(ctx, launch_after_resid(t, b, ps, false, ctx->stream));
        HIP_TRY(ctx, launch_arnoldi(t, prec, b, ps, y, m_max, orth, ctx->expect.data(), &ctx->env, ctx->stream));
        HIP_TRY(ctx, launch_update(t, prec, b, z, z, orth == CH_ORTH_DCGS2, ctx->stream));
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

// Issue EE2 steps for every instance of the table until all are halted (each
// stops at its own T or step limit) or `max_launch` steps have been issued.
bool graph_chunk_ok(const ch_ee_opts* o) { return o->graph_chunk >= 0 && o->graph_chunk <= CH_MMAX + 1; }

int issue_ee_steps(ch_ctx* ctx, const Table& t, int prec, int m_max, int orth, bool constant, long long max_launch) {
    const DevBuffers& b = ctx->b;
    PartSeq ps;
    ps.base = b.part;
    int rc;
    HIP_TRY(ctx, launch_resid(t, prec, b, ps, b.ybuf[0], b.ybuf[0], true, true, ctx->stream));
    HIP_TRY(ctx, launch_after_resid(t, b, ps, true, ctx->stream));
    for (int i = 0; i < t.ninst; ++i) ctx->expect[t.hinst[i].slot] += 1;
    for (long long s = 0; s < max_launch; ++s) {
        const int p = (int)(s & 1);
        HIP_TRY(ctx, launch_arnoldi(t, prec, b, ps, b.ybuf[p], m_max, orth, ctx->expect.data(), &ctx->env,
                                    ctx->stream));
        HIP_TRY(ctx, launch_update(t, prec, b, b.ybuf[p], b.ybuf[p ^ 1], orth == CH_ORTH_DCGS2, ctx->stream));
        if (constant && (rc = restart_cycles(ctx, t, prec, ps, b.ybuf[p], b.ybuf[p ^ 1], m_max, orth))) return rc;
        HIP_TRY(ctx, launch_est_ee(t, prec, b, ps, b.ybuf[p], b.ybuf[p ^ 1], ctx->stream));
        HIP_TRY(ctx, launch_step_end(t, b, ps, true, ctx->stream));
        for (int i = 0; i < t.ninst; ++i) ctx->expect[t.hinst[i].slot] += 1;
        if ((s % 16) == 15) {
            if ((rc = read_heads(ctx, t.ninst))) return rc;
            if (all_halted(ctx, t.ninst)) break;
        }
    }
    return CH_OK;
}

int copy_in(ch_ctx* ctx, const Member& m, const double* y) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->b.ybuf[0] + m.off, y, sizeof(double) * m.sh.N, hipMemcpyDeviceToDevice,
                                ctx->stream));
    return CH_OK;
}

int copy_out(ch_ctx* ctx, const Member& m, int slot, double* y) {
    const Ctl& h = ctx->hctl[slot];
    HIP_TRY(ctx, hipMemcpyAsync(y, ctx->b.ybuf[h.cur] + m.off, sizeof(double) * m.sh.N, hipMemcpyDeviceToDevice,
                                ctx->stream));
    return CH_OK;
}

int run_ee(ch_ctx* ctx, const ch_problem* prob, double* y, double tau0, double t0, double T, int max_steps,
           const ch_ee_opts* opts, ch_run_stats* stats, ch_step_record* records) {
    Shape sh;
    int rc = check_problem(prob, &sh);
    if (rc) return rc;
    if (!y || !opts) return CH_EINVAL;
    if (opts->m_max < 1 || opts->m_max > CH_MMAX || !orth_ok(opts->orth) || !graph_chunk_ok(opts)) return CH_EINVAL;
    if (!(tau0 > 0.0) || !(opts->tau_min >= 0.0)) return CH_EINVAL;
    if (!(opts->tol > 0.0) && !(opts->tol_phi_fixed > 0.0)) return CH_EINVAL;
    if (max_steps <= 0 && !(T < INFINITY)) return CH_EINVAL;
    if (!(t0 < INFINITY)) return CH_EINVAL;
    const int prec = prob->prec;
    const int recs = (records && max_steps > 0) ? max_steps : 0;
    if ((rc = ensure(ctx, pad64(sh.N), opts->m_max, prec, 1, recs, false))) return rc;
    Member m{sh, prob->eps, prob->eyre, 0};
    Table t;
    if ((rc = build_table(ctx, {m}, sh.dim, prec, &t))) return rc;
    const bool constant = opts->constant_step != 0;
    init_ctl(ctx->hctl, constant ? MODE_EE_CONST : MODE_EE, t0, tau0, T, opts->tol, opts->tol_phi_fixed,
             opts->tau_min, opts->m_max, max_steps, recs ? ctx->rec : nullptr, recs, ctx->expect[0]);
    set_mobility(ctx->hctl, sh);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    if ((rc = copy_in(ctx, m, y))) return rc;
    const long long limit = max_steps > 0 ? max_steps : (1LL << 40);
    ctx->env.graph_chunk = opts->graph_chunk;
    rc = issue_ee_steps(ctx, t, prec, opts->m_max, opts->orth, constant, limit);
    ctx->env.graph_chunk = 0;
    if (rc) return rc;
    if ((rc = read_heads(ctx, 1))) return rc;
    if ((rc = copy_out(ctx, m, 0, y))) return rc;
    const Ctl& h = ctx->hctl[0];
    const int nrec = std::min(h.steps, recs);
    if (records && nrec > 0)
        HIP_TRY(ctx, hipMemcpyAsync(records, ctx->rec, sizeof(ch_step_record) * nrec, hipMemcpyDeviceToHost,
                                    ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    fill_stats(h, stats);
    return h.status;
}

int run_ee_batch(ch_ctx* ctx, int count, const ch_batch_item* items, int dim, int eyre, int prec,
                 const ch_ee_opts* opts, ch_run_stats* stats) {
    if (count < 1 || !items || !opts) return CH_EINVAL;
    if (prec != CH_FP64 && prec != CH_FP32_MIXED) return CH_EINVAL;
    if (opts->m_max < 1 || opts->m_max > CH_MMAX || opts->constant_step || !orth_ok(opts->orth) ||
        !graph_chunk_ok(opts))
        return CH_EINVAL;
    if (!(opts->tol > 0.0) && !(opts->tol_phi_fixed > 0.0)) return CH_EINVAL;
    std::vector<Member> ms(count);
    size_t pts = 0;
    for (int i = 0; i < count; ++i) {
        const ch_batch_item& it = items[i];
        int rc = check_grid(dim, it.n, it.eps, eyre, &ms[i].sh);
        if (rc) return rc;
        if (!it.y || !(it.tau0 > 0.0) || (it.max_steps <= 0 && !(it.T < INFINITY))) return CH_EINVAL;
        ms[i].eps = it.eps;
        ms[i].eyre = eyre;
        ms[i].off = pts;
        pts += pad64(ms[i].sh.N);
    }
    int rc;
    if ((rc = ensure(ctx, pts, opts->m_max, prec, count, 0, false))) return rc;
    Table t;
    if ((rc = build_table(ctx, ms, dim, prec, &t))) return rc;
    long long limit = 0;
    for (int i = 0; i < count; ++i) {
        const ch_batch_item& it = items[i];
        init_ctl(ctx->hctl + i, MODE_EE, 0.0, it.tau0, it.T, opts->tol, opts->tol_phi_fixed, opts->tau_min,
                 opts->m_max, it.max_steps, nullptr, 0, ctx->expect[i]);
        limit = it.max_steps > 0 ? std::max<long long>(limit, it.max_steps) : (1LL << 40);
        if ((rc = copy_in(ctx, ms[i], it.y))) return rc;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->b.ctl, ctx->hctl, sizeof(Ctl) * count, hipMemcpyHostToDevice, ctx->stream));
    ctx->env.graph_chunk = opts->graph_chunk;
    rc = issue_ee_steps(ctx, t, prec, opts->m_max, opts->orth, false, limit);
    ctx->env.graph_chunk = 0;
    if (rc) return rc;
    if ((rc = read_heads(ctx, count))) return rc;
    int status = CH_OK;
    for (int i = 0; i < count; ++i) {
        if ((rc = copy_out(ctx, ms[i], i, items[i].y))) return rc;
        if (stats) fill_stats(ctx->hctl[i], stats + i);
        if (ctx->hctl[i].status != CH_OK && status == CH_OK) status = ctx->hctl[i].status;
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return status;
}

// Reads the scalar head of control block 0 into h (host memory of any kind).
int read_head(ch_ctx* ctx, const DevBuffers& b, Ctl* h) {
    HIP_TRY(ctx, hipMemcpyAsync(h, b.ctl, CTL_HEAD, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

// LIM step s of every instance of a table (Figs. 1 and 2): bounds of the
// spectrum, the plan (whose Chebyshev orders the host reads to size the
// stage launches: the largest order decides, instances of smaller order
// skip the launches past their last), the stages, the estimate and the
// controller.  Every live instance has taken s steps, so its state
// ping-pongs between b.ybuf[s & 1] and b.ybuf[(s + 1) & 1].  The orders come
// from the pinned words the plan writes when the buffers have them (one host
// wait on the plan, no copies), else from copies of the control heads into
// hctl (indexed by slot), which the caller must not rely on being current in
// the first case.  *halted: no instance had anything left to do (t >= T, the
// step limit, or an error in the plan).
int issue_lim_step(ch_ctx* ctx, const Table& t, const DevBuffers& b, PartSeq& ps, Ctl* hctl, long long s,
                   bool* halted) {
    const double* yin = b.ybuf[s & 1];
    double* yout = b.ybuf[(s + 1) & 1];
    const int seq = ++ctx->lseq;
    HIP_TRY(ctx, launch_lim_begin(t, b, ps, yin, ctx->stream));
    HIP_TRY(ctx, launch_lim_plan(t, b, ps, seq, ctx->stream));
    const bool pairs = lim_stage_pairs(t);
    auto stage = [&](int l) -> hipError_t {
        return pairs && l > 0 ? launch_lim_stage2(t, b, yin, yout, l, ctx->stream)
                              : launch_lim_stage(t, b, yin, yout, l, pairs, ctx->stream);
    };
    int nl = 0;
    // every instance's order from the pinned words the plan writes (a
    // bounded wait); else from copies of the control blocks
    bool got = false;
    if (b.hlim) {
        const auto t0 = std::chrono::steady_clock::now();
        for (long long spin = 0;; ++spin) {
            bool all = true;
            for (int i = 0; i < t.ninst && all; ++i) all = b.hlim[2 * t.hinst[i].slot + 1] == seq;
            if (all) {
                got = true;
                break;
            }
            if ((spin & 255) == 255 &&
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > CH_PLAN_WAIT_S)
                break;
        }
        if (got)
            for (int i = 0; i < t.ninst; ++i) {
                const int p = b.hlim[2 * t.hinst[i].slot];
                if (p > 0) nl = std::max(nl, lim_launches(p, pairs));
            }
    }
    if (!got) {
        int lo = INT_MAX, hi = -1;
        for (int i = 0; i < t.ninst; ++i) {
            lo = std::min(lo, t.hinst[i].slot);
            hi = std::max(hi, t.hinst[i].slot);
        }
        int rc = copy_heads_to(ctx, hctl, b.ctl, lo, hi);
        if (rc) return rc;
        for (int i = 0; i < t.ninst; ++i) {
            const Ctl& h = hctl[t.hinst[i].slot];
            if (!h.halted) nl = std::max(nl, lim_launches(h.p, pairs));
        }
    }
    *halted = nl == 0;
    if (*halted) return CH_OK;
    // 2p - 1 stages (the nodes in the plan's order, then again without
    // beta_1); on 2-D strips stage 0 runs alone and the rest in pairs
    for (int l = 0; l < nl; ++l) HIP_TRY(ctx, stage(l));
    HIP_TRY(ctx, launch_est_lim(t, b, ps, yin, yout, ctx->stream));
    HIP_TRY(ctx, launch_lim_end(t, b, ps, ctx->stream));
    return CH_OK;
}

int run_lim(ch_ctx* ctx, const ch_problem* prob, double* y, double tau0, double t0, double T, int max_steps,
            double tol, ch_run_stats* stats, ch_step_record* records) {
    Shape sh;
    int rc = check_problem(prob, &sh);
    if (rc) return rc;
    if (!y || !(tau0 > 0.0)) return CH_EINVAL;
    if (max_steps <= 0 && !(T < INFINITY)) return CH_EINVAL;
    const int recs = (records && max_steps > 0) ? max_steps : 0;
    if ((rc = ensure(ctx, pad64(sh.N), 0, CH_FP64, 1, recs, true))) return rc;
    Member m{sh, prob->eps, prob->eyre, 0};
    Table t;
    if ((rc = build_table(ctx, {m}, sh.dim, CH_FP64, &t))) return rc;
    const DevBuffers& b = ctx->b;
    init_ctl(ctx->hctl, tol > 0.0 ? MODE_LIM : MODE_LIM_CONST, t0, tau0, T, tol, 0.0, 0.0, 0, max_steps,
             recs ? ctx->rec : nullptr, recs, ctx->expect[0]);
    set_mobility(ctx->hctl, sh);
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    if ((rc = copy_in(ctx, m, y))) return rc;
    PartSeq ps;
    ps.base = b.part;
    for (long long s = 0;; ++s) {
        if (max_steps > 0 && s >= max_steps) break;
        bool halted = false;
        if ((rc = issue_lim_step(ctx, t, b, ps, ctx->hctl, s, &halted))) return rc;
        if (halted) break;
    }
    if ((rc = read_heads(ctx, 1))) return rc;
    if ((rc = copy_out(ctx, m, 0, y))) return rc;
    const Ctl& h = ctx->hctl[0];
    const int nrec = std::min(h.steps, recs);
    if (records && nrec > 0)
        HIP_TRY(ctx, hipMemcpyAsync(records, ctx->rec, sizeof(ch_step_record) * nrec, hipMemcpyDeviceToHost,
                                    ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    fill_stats(h, stats);
    return h.status;
}

int run_lim_batch(ch_ctx* ctx, int count, const ch_batch_item* items, int dim, int eyre, double tol,
                  ch_run_stats* stats) {
    if (count < 1 || !items) return CH_EINVAL;
    std::vector<Member> ms(count);
    size_t pts = 0;
    for (int i = 0; i < count; ++i) {
        const ch_batch_item& it = items[i];
        int rc = check_grid(dim, it.n, it.eps, eyre, &ms[i].sh);
        if (rc) return rc;
        if (!it.y || !(it.tau0 > 0.0) || (it.max_steps <= 0 && !(it.T < INFINITY))) return CH_EINVAL;
        ms[i].eps = it.eps;
        ms[i].eyre = eyre;
        ms[i].off = pts;
        pts += pad64(ms[i].sh.N);
    }
    int rc;
    if ((rc = ensure(ctx, pts, 0, CH_FP64, count, 0, true))) return rc;
    Table t;
    if ((rc = build_table(ctx, ms, dim, CH_FP64, &t))) return rc;
    const DevBuffers& b = ctx->b;
    for (int i = 0; i < count; ++i) {
        const ch_batch_item& it = items[i];
        init_ctl(ctx->hctl + i, tol > 0.0 ? MODE_LIM : MODE_LIM_CONST, 0.0, it.tau0, it.T, tol, 0.0, 0.0, 0,
                 it.max_steps, nullptr, 0, ctx->expect[i]);
        if ((rc = copy_in(ctx, ms[i], it.y))) return rc;
    }
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl) * count, hipMemcpyHostToDevice, ctx->stream));
    PartSeq ps;
    ps.base = b.part;
    for (long long s = 0;; ++s) {
        bool halted = false;
        if ((rc = issue_lim_step(ctx, t, b, ps, ctx->hctl, s, &halted))) return rc;
        if (halted) break;
    }
    if ((rc = read_heads(ctx, count))) return rc;
    int status = CH_OK;
    for (int i = 0; i < count; ++i) {
        if ((rc = copy_out(ctx, ms[i], i, items[i].y))) return rc;
        if (stats) fill_stats(ctx->hctl[i], stats + i);
        if (ctx->hctl[i].status != CH_OK && status == CH_OK) status = ctx->hctl[i].status;
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return status;
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

// ---------------------------------------------------------------------------
// Serving: continuous batching (ch_server_create / ch_submit / ch_poll)
// ---------------------------------------------------------------------------
double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    unsigned long long id = 0;
    int n = 0, steps = 0;
    double eps = 0, tau0 = 0;
    int method = CH_METHOD_EE;
    double T = INFINITY, tol = 0.0;
    long long N = 0;
    size_t len = 0;            // pooled points (padded)
    int sblk = 0, cblk = 0;    // workgroups in a batched launch
    int wblk = 0;              // 2-D strip workgroups
    double* buf = nullptr;     // device: y0 until admission, the result after
    size_t cap = 0;            // bytes of buf (a pooled buffer may be larger than needed)
    int state = CH_REQ_QUEUED;
    int status = CH_OK;
    ch_run_stats stats{};
    double t_submit = 0, t_start = 0, t_done = 0;
    int slot = -1;
    size_t off = 0;
};

}  // namespace

struct ch_server {
    ch_ctx* ctx = nullptr;     // private context on a private stream
    hipStream_t stream = nullptr;   // the scheduler's stream (non-blocking)
    hipStream_t io = nullptr;       // copies of ch_submit / ch_poll (non-blocking)
    std::mutex buf_mu;
    std::multimap<size_t, double*> spare;   // request buffers released by ch_poll, by size
    int device = 0, prec = CH_FP64, max_slots = 0;
    ch_ee_opts opts{};
    size_t pool_pts = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req*> queue;
    std::unordered_map<unsigned long long, Req*> reqs;
    std::vector<Req*> slot_req;         // slot -> request in flight
    std::map<size_t, size_t> free_;     // free pooled ranges: offset -> points
    int sblk_used = 0, cblk_used = 0, wblk_used = 0, running = 0;
    unsigned long long next_id = 1;
    bool stop = false;
    int fatal = CH_OK;
    std::thread th;
};

namespace {

// Request buffers are recycled: a released one of at least `bytes` (and at
// most twice that) is reused, so steady serving makes no hipMalloc or hipFree
// calls (hipFree synchronises the device).
double* take_buffer(ch_server* S, size_t bytes, size_t* cap) {
    {
        std::lock_guard<std::mutex> lk(S->buf_mu);
        auto it = S->spare.lower_bound(bytes);
        if (it != S->spare.end() && it->first <= 2 * bytes) {
            double* p = it->second;
            *cap = it->first;
            S->spare.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    *cap = bytes;
    return static_cast<double*>(p);
}

void give_buffer(ch_server* S, double* p, size_t cap) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(S->buf_mu);
    S->spare.emplace(cap, p);
}

bool pool_alloc(ch_server* S, size_t len, size_t* off) {
    for (auto it = S->free_.begin(); it != S->free_.end(); ++it) {
        if (it->second >= len) {
            *off = it->first;
            const size_t rest = it->second - len;
            const size_t roff = it->first + len;
            S->free_.erase(it);
            if (rest) S->free_[roff] = rest;
            return true;
        }
    }
    return false;
}

void pool_free(ch_server* S, size_t off, size_t len) {
    auto it = S->free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != S->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        S->free_.erase(nx);
    }
    if (it != S->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            S->free_.erase(it);
        }
    }
}

// The heads of the given requests' slots (one strided copy over the range
// they span: the slots in between are copied too and not read).
int read_slot_heads(ch_ctx* ctx, const std::vector<Req*>& rs) {
    int lo = INT_MAX, hi = -1;
    for (Req* r : rs) {
        lo = std::min(lo, r->slot);
        hi = std::max(hi, r->slot);
    }
    return copy_heads(ctx, lo, hi);
}

Member member_of(const Req* r) {
    Member m;
    m.sh.dim = 2;
    m.sh.n = r->n;
    m.sh.N = r->N;
    m.eps = r->eps;
    m.eyre = 0;
    m.off = r->off;
    m.slot = r->slot;
    return m;
}

// One iteration of the scheduler: admit, start, one batch step, retire.
// t: the tables of the EE2 members (t[0]) and the LIM members (t[1]).
int serve_once(ch_server* S, long long* par, Table* t, bool* dirty) {
    ch_ctx* ctx = S->ctx;
    const DevBuffers& b = ctx->b;
    std::vector<Req*> admitted, live;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->stop || !S->queue.empty() || S->running > 0; });
        if (S->stop && S->running == 0) return 1;
        while (!S->stop && !S->queue.empty()) {
            Req* r = S->queue.front();
            int slot = -1;
            for (int i = 0; i < S->max_slots; ++i)
                if (!S->slot_req[i]) {
                    slot = i;
                    break;
                }
            if (slot < 0) break;
            if (S->sblk_used + r->sblk > CH_MAXB || S->cblk_used + r->cblk > CH_MAXB ||
                S->wblk_used + r->wblk > CH_MAXB)
                break;
            size_t off;
            if (!pool_alloc(S, r->len, &off)) break;
            S->queue.pop_front();
            r->slot = slot;
            r->off = off;
            r->state = CH_REQ_RUNNING;
            r->t_start = now_s();
            S->slot_req[slot] = r;
            S->sblk_used += r->sblk;
            S->cblk_used += r->cblk;
            S->wblk_used += r->wblk;
            S->running += 1;
            admitted.push_back(r);
        }
        for (Req* r : S->slot_req)
            if (r) live.push_back(r);
    }
    int rc;
    const int p = (int)(*par & 1);
    if (!admitted.empty()) {
        // start: state into the buffer of the current parity; EE2: f(y0) and
        // the first step's begin
        std::vector<Member> ms;
        for (Req* r : admitted) {
            const double tol = r->tol > 0.0 ? r->tol : S->opts.tol;
            if (r->method == CH_METHOD_LIM)
                init_ctl(ctx->hctl + r->slot, tol > 0.0 ? MODE_LIM : MODE_LIM_CONST, 0.0, r->tau0, r->T, tol, 0.0,
                         0.0, 0, r->steps, nullptr, 0, ctx->expect[r->slot]);
            else
                init_ctl(ctx->hctl + r->slot, MODE_EE, 0.0, r->tau0, r->T, tol, r->tol > 0.0 ? 0.0 : S->opts.tol_phi_fixed,
                         S->opts.tau_min, S->opts.m_max, r->steps, nullptr, 0, ctx->expect[r->slot]);
            ctx->hctl[r->slot].cur = p;
            HIP_TRY(ctx, hipMemcpyAsync(b.ctl + r->slot, ctx->hctl + r->slot, sizeof(Ctl), hipMemcpyHostToDevice,
                                        ctx->stream));
            HIP_TRY(ctx, hipMemcpyAsync(b.ybuf[p] + r->off, r->buf, sizeof(double) * r->N, hipMemcpyDeviceToDevice,
                                        ctx->stream));
            if (r->method == CH_METHOD_EE) ms.push_back(member_of(r));
        }
        if (!ms.empty()) {
            Table ta;
            if ((rc = build_table(ctx, ms, 2, S->prec, &ta))) return rc;
            PartSeq ps;
            ps.base = b.part;
            HIP_TRY(ctx, launch_resid(ta, S->prec, b, ps, b.ybuf[p], b.ybuf[p], true, true, ctx->stream));
            HIP_TRY(ctx, launch_after_resid(ta, b, ps, true, ctx->stream));
            for (Req* r : admitted)
                if (r->method == CH_METHOD_EE) ctx->expect[r->slot] += 1;
        }
        *dirty = true;
    }
    if (live.empty()) return CH_OK;
    std::vector<Req*> ee, lim;
    for (Req* r : live) (r->method == CH_METHOD_LIM ? lim : ee).push_back(r);
    if (*dirty) {
        // EE2 members in table store 0 (t[0]), LIM members in store 1 (t[1])
        std::vector<Member> me, ml;
        for (Req* r : ee) me.push_back(member_of(r));
        for (Req* r : lim) ml.push_back(member_of(r));
        if (!me.empty() && (rc = build_table(ctx, me, 2, S->prec, &t[0], 0))) return rc;
        if (!ml.empty() && (rc = build_table(ctx, ml, 2, CH_FP64, &t[1], 1))) return rc;
        *dirty = false;
    }
    if (!ee.empty()) {
        PartSeq ps;
        ps.base = b.part;
        HIP_TRY(ctx, launch_arnoldi(t[0], S->prec, b, ps, b.ybuf[p], S->opts.m_max, S->opts.orth, ctx->expect.data(),
                                    &ctx->env, ctx->stream));
        HIP_TRY(ctx, launch_update(t[0], S->prec, b, b.ybuf[p], b.ybuf[p ^ 1], S->opts.orth == CH_ORTH_DCGS2,
                                   ctx->stream));
        HIP_TRY(ctx, launch_est_ee(t[0], S->prec, b, ps, b.ybuf[p], b.ybuf[p ^ 1], ctx->stream));
        HIP_TRY(ctx, launch_step_end(t[0], b, ps, true, ctx->stream));
        for (Req* r : ee) ctx->expect[r->slot] += 1;
    }
    if (!lim.empty()) {
        PartSeq ps;
        ps.base = b.part;
        bool halted = false;
        if ((rc = issue_lim_step(ctx, t[1], b, ps, ctx->hctl, *par, &halted))) return rc;
    }
    *par += 1;
    if ((rc = read_slot_heads(ctx, live))) return rc;
    std::vector<Req*> done;
    for (Req* r : live)
        if (ctx->hctl[r->slot].halted) {
            const Ctl& h = ctx->hctl[r->slot];
            HIP_TRY(ctx, hipMemcpyAsync(r->buf, b.ybuf[h.cur] + r->off, sizeof(double) * r->N,
                                        hipMemcpyDeviceToDevice, ctx->stream));
            done.push_back(r);
        }
    if (!done.empty()) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        const double tnow = now_s();
        std::lock_guard<std::mutex> lk(S->mu);
        for (Req* r : done) {
            const Ctl& h = ctx->hctl[r->slot];
            fill_stats(h, &r->stats);
            r->status = h.status;
            r->state = h.status == CH_OK ? CH_REQ_DONE : CH_REQ_FAILED;
            r->t_done = tnow;
            S->slot_req[r->slot] = nullptr;
            pool_free(S, r->off, r->len);
            S->sblk_used -= r->sblk;
            S->cblk_used -= r->cblk;
            S->wblk_used -= r->wblk;
            S->running -= 1;
        }
        *dirty = true;
    }
    return CH_OK;
}

void serve_loop(ch_server* S) {
    (void)hipSetDevice(S->device);
    long long par = 0;
    Table t[2]{};
    bool dirty = true;
    for (;;) {
        const int rc = serve_once(S, &par, t, &dirty);
        if (rc == 1) break;
        if (rc != CH_OK) {   // device error: fail everything and stop
            std::lock_guard<std::mutex> lk(S->mu);
            S->fatal = rc;
            for (Req* r : S->slot_req)
                if (r) {
                    r->state = CH_REQ_FAILED;
                    r->status = rc;
                }
            for (Req* r : S->queue) {
                r->state = CH_REQ_FAILED;
                r->status = rc;
            }
            S->queue.clear();
            S->stop = true;
            break;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of ch_step_lim_noalloc: one file-scope device array (each GPU the
// library runs on holds its own copy until the process ends) carved into the
// two state buffers and the stage buffer of a grid of at most
// CH_NOALLOC_MAX_POINTS points, the reduction partials, the LIM node order
// and stage coefficients, one control block, one step record and the
// instance table.  Host code never names the array: it uses the per-device
// address hipGetSymbolAddress returns.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t na_align(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t NA_PTS = (size_t)CH_NOALLOC_MAX_POINTS;
constexpr size_t NA_MAP = CH_SBLK_MAX > CH_WBLK_MAX ? CH_SBLK_MAX : CH_WBLK_MAX;   // >= CH_CBLK_MAX too
constexpr size_t NA_Y0 = 0;
constexpr size_t NA_Y1 = NA_Y0 + na_align(sizeof(double) * NA_PTS);
constexpr size_t NA_Z = NA_Y1 + na_align(sizeof(double) * NA_PTS);
constexpr size_t NA_PART = NA_Z + na_align(sizeof(double) * NA_PTS);
constexpr size_t NA_ORDER = NA_PART + na_align(sizeof(double) * 2 * CH_NRED * CH_MAXB);
constexpr size_t NA_COEF = NA_ORDER + na_align(sizeof(int) * CH_PMAX);
constexpr size_t NA_CTL = NA_COEF + na_align(sizeof(double) * 4 * CH_PMAX);
constexpr size_t NA_REC = NA_CTL + na_align(sizeof(Ctl));
constexpr size_t NA_INST = NA_REC + na_align(sizeof(ch_step_record));
constexpr size_t NA_MAPS = NA_INST + na_align(sizeof(Inst));
constexpr size_t NA_BYTES = NA_MAPS + na_align(sizeof(int) * NA_MAP);
static_assert(CH_CBLK_MAX <= NA_MAP, "map of the streaming workgroups");

}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mu;
void* na_ptr[NA_MAX_DEVICES];   // address of `scratch` on each device (null: not looked up)

// Once per device, with that device current: the device address of the
// scratch array.  Called by ch_create; a failure is reported by the entry
// point that needs it, not by ch_create.
void noalloc_setup(int device) {
    if (device < 0 || device >= NA_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(na_mu);
    if (na_ptr[device]) return;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    na_ptr[device] = p;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= NA_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(na_mu);
    return na_ptr[device];
}

// Host copy of the control block and zeros for the workgroup maps (a
// single-grid launch never reads them; they are kept valid regardless).
thread_local Ctl na_hctl;
const int na_zero_map[NA_MAP] = {};

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
    noalloc_setup(device);
    LaunchEnv& sd = ctx->env;
    sd.graphs = &ctx->graphs;
    if (hipStreamCreateWithFlags(&sd.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sd.ev_main, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sd.ev_side, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&sd.cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        if (sd.ev_main) (void)hipEventDestroy(sd.ev_main);
        if (sd.ev_side) (void)hipEventDestroy(sd.ev_side);
        if (sd.side) (void)hipStreamDestroy(sd.side);
        delete ctx;
        return CH_EDEVICE;
    }
    *out = ctx;
    return CH_OK;
}

int ch_destroy(ch_ctx* ctx) {
    if (!ctx) return CH_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamSynchronize(ctx->env.side);
    DevBuffers& b = ctx->b;
    destroy_graphs(ctx->graphs);
    for (void* p : {(void*)b.V, (void*)b.ybuf[0], (void*)b.ybuf[1], (void*)b.fcur, (void*)b.y32, (void*)b.zbuf,
                    (void*)b.part, (void*)b.dots, (void*)b.lorder, (void*)b.ctl, (void*)ctx->rec, b.phibig,
                    (void*)b.lcoef, (void*)b.dcount})
        free_dev(p);
    for (auto& ts : ctx->store)
        for (void* p : {(void*)ts.d_inst, (void*)ts.d_sb2i, (void*)ts.d_cb2i, (void*)ts.d_wb2i}) free_dev(p);
    if (ctx->hctl) (void)hipHostFree(ctx->hctl);
    if (ctx->hflag) (void)hipHostFree(ctx->hflag);
    (void)hipEventDestroy(ctx->env.ev_main);
    (void)hipEventDestroy(ctx->env.ev_side);
    (void)hipStreamDestroy(ctx->env.side);
    (void)hipStreamDestroy(ctx->env.cap);
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

int ch_run_ee_batch(ch_ctx* ctx, int count, ch_batch_item* items, int dim, int eyre, int prec,
                    const ch_ee_opts* opts, ch_run_stats* stats) {
    if (!ctx) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    return run_ee_batch(ctx, count, items, dim, eyre, prec, opts, stats);
}

int ch_run_lim_batch(ch_ctx* ctx, int count, ch_batch_item* items, int dim, int eyre, double tol,
                     ch_run_stats* stats) {
    if (!ctx) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    return run_lim_batch(ctx, count, items, dim, eyre, tol, stats);
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

int ch_step_lim_noalloc(ch_ctx* ctx, const ch_problem* prob, double* y, double tau, double t, double T, double tol,
                        ch_step_record* out) {
    if (!ctx) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    Shape sh;
    int rc = check_problem(prob, &sh);
    if (rc) return rc;
    if (!y || !(tau > 0.0)) return CH_EINVAL;
    if ((size_t)sh.N > NA_PTS) {
        ctx->err = "grid larger than the no-allocation scratch (CH_NOALLOC_MAX_POINTS points)";
        return CH_EINVAL;
    }
    unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(ctx->device));
    if (!base) {
        ctx->err = "no device address for the no-allocation scratch on this device";
        return CH_EDEVICE;
    }
    DevBuffers b{};
    b.ybuf[0] = reinterpret_cast<double*>(base + NA_Y0);
    b.ybuf[1] = reinterpret_cast<double*>(base + NA_Y1);
    b.zbuf = reinterpret_cast<double*>(base + NA_Z);
    b.part = reinterpret_cast<double*>(base + NA_PART);
    b.lorder = reinterpret_cast<int*>(base + NA_ORDER);
    b.lcoef = reinterpret_cast<double*>(base + NA_COEF);
    b.ctl = reinterpret_cast<Ctl*>(base + NA_CTL);
    ch_step_record* drec = reinterpret_cast<ch_step_record*>(base + NA_REC);
    Inst* dinst = reinterpret_cast<Inst*>(base + NA_INST);
    int* dmap = reinterpret_cast<int*>(base + NA_MAPS);
    const Member m{sh, prob->eps, prob->eyre, 0};
    const Inst I = make_inst(m, 0, sh.dim, CH_FP64, 0, 0, 0);
    Table tb{};
    tb.inst = dinst;
    tb.sb2i = tb.cb2i = tb.wb2i = dmap;
    tb.ninst = 1;
    tb.sgrid = I.sblk;
    tb.cgrid = I.cblk;
    tb.wgrid = I.wblk;
    tb.dim = sh.dim;
    tb.hinst = &I;
    Ctl* h = &na_hctl;
    init_ctl(h, tol > 0.0 ? MODE_LIM : MODE_LIM_CONST, t, tau, T, tol, 0.0, 0.0, 0, 1, drec, 1, 0);
    set_mobility(h, sh);
    // every control value, the instance record and the maps are written before
    // the first launch; partials are written by their producers before use
    HIP_TRY(ctx, hipMemcpyAsync(dinst, &I, sizeof(Inst), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(dmap, na_zero_map, sizeof(na_zero_map), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, h, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.ybuf[0], y, sizeof(double) * sh.N, hipMemcpyDeviceToDevice, ctx->stream));
    PartSeq ps;
    ps.base = b.part;
    bool halted = false;
    if ((rc = issue_lim_step(ctx, tb, b, ps, h, 0, &halted))) return rc;
    if ((rc = read_head(ctx, b, h))) return rc;
    ch_step_record rec;
    memset(&rec, 0, sizeof(rec));
    if (h->status == CH_OK && h->steps == 1) {
        HIP_TRY(ctx, hipMemcpyAsync(y, b.ybuf[h->cur], sizeof(double) * sh.N, hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(&rec, drec, sizeof(rec), hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (out) *out = rec;
    return h->status;
}

int ch_phiv(ch_ctx* ctx, const ch_problem* prob, const double* y, double* y_out, double tau0, int mode,
            double tol_phi, int m_max, ch_step_record* out) {
    if (!ctx) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    Shape sh;
    int rc = check_problem(prob, &sh);
    if (rc) return rc;
    if (!y || !y_out || y == y_out) return CH_EINVAL;
    if (!(tau0 > 0.0) || !(tol_phi > 0.0) || m_max < 1 || m_max > CH_MMAX) return CH_EINVAL;
    if (mode != CH_PHI_SHRINK && mode != CH_PHI_RESTART) return CH_EINVAL;
    const int prec = prob->prec;
    if ((rc = ensure(ctx, pad64(sh.N), m_max, prec, 1, 0, false))) return rc;
    Member m{sh, prob->eps, prob->eyre, 0};
    Table t;
    if ((rc = build_table(ctx, {m}, sh.dim, prec, &t))) return rc;
    const DevBuffers& b = ctx->b;
    init_ctl(ctx->hctl, MODE_PHI, 0.0, tau0, INFINITY, 0.0, tol_phi, 0.0, m_max, 0, nullptr, 0, ctx->expect[0]);
    set_mobility(ctx->hctl, sh);
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    if ((rc = copy_in(ctx, m, y))) return rc;
    PartSeq ps;
    ps.base = b.part;
    HIP_TRY(ctx, launch_resid(t, prec, b, ps, b.ybuf[0], b.ybuf[0], false, true, ctx->stream));
    HIP_TRY(ctx, launch_after_resid(t, b, ps, true, ctx->stream));
    ctx->expect[0] += 1;
    HIP_TRY(ctx, launch_arnoldi(t, prec, b, ps, b.ybuf[0], m_max, CH_ORTH_DCGS2, ctx->expect.data(), &ctx->env,
                                ctx->stream));
    HIP_TRY(ctx, launch_update(t, prec, b, b.ybuf[0], b.ybuf[1], true, ctx->stream));
    if (mode == CH_PHI_RESTART && (rc = restart_cycles(ctx, t, prec, ps, b.ybuf[0], b.ybuf[1], m_max, CH_ORTH_DCGS2)))
        return rc;
    if ((rc = read_heads(ctx, 1))) return rc;
    const Ctl& h = ctx->hctl[0];
    if (h.status == CH_OK)
        HIP_TRY(ctx, hipMemcpyAsync(y_out, b.ybuf[1], sizeof(double) * sh.N, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    record_from_head(h, out);
    return h.status;
}

static int time_kernel_core(ch_ctx* ctx, const Shape& sh, const ch_problem* prob, int kernel, int m_max,
                            const int* iters, int count, double* total_us, double* total_bytes);

int ch_time_kernel(ch_ctx* ctx, const ch_problem* prob, int kernel, int m_max, const int* iters, int count,
                   double* total_us, double* total_bytes) {
    const bool lim = kernel == CH_KERNEL_LIM_STAGE || kernel == CH_KERNEL_LIM_STAGE2;
    if (!ctx || !total_us || !total_bytes || count < 1 || (!iters && !lim)) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    Shape sh;
    int rc = check_problem(prob, &sh);
    if (rc) return rc;
    if (m_max < 1 || m_max > CH_MMAX || kernel < CH_KERNEL_MGS || kernel > CH_KERNEL_LIM_STAGE2) return CH_EINVAL;
    const int prec = lim ? CH_FP64 : prob->prec;
    const size_t esz = prec == CH_FP64 ? sizeof(double) : sizeof(float);
    const DevBuffers& b = ctx->b;
    // the workspace of an earlier run on this problem
    if (!b.ctl || ctx->pts < (size_t)sh.N) return CH_EINVAL;
    if (lim ? ctx->z_pts < (size_t)sh.N
            : (ctx->v_bytes < (size_t)(m_max + 1) * b.ldv * esz ||
               (prec == CH_FP32_MIXED && ctx->y32_pts < (size_t)sh.N)))
        return CH_EINVAL;
    return time_kernel_core(ctx, sh, prob, kernel, m_max, iters, count, total_us, total_bytes);
}

// ch_time_kernel after its checks: the workspace holds this problem.
static int time_kernel_core(ch_ctx* ctx, const Shape& sh, const ch_problem* prob, int kernel, int m_max,
                            const int* iters, int count, double* total_us, double* total_bytes) {
    const bool lim = kernel == CH_KERNEL_LIM_STAGE || kernel == CH_KERNEL_LIM_STAGE2;
    const int prec = lim ? CH_FP64 : prob->prec;
    const size_t esz = prec == CH_FP64 ? sizeof(double) : sizeof(float);
    const DevBuffers& b = ctx->b;
    int rc;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->hctl, b.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    Ctl& h = ctx->hctl[0];
    for (int i = 0; !lim && i < count; ++i) {
        const int k = iters[i];
        bool ok;
        switch (kernel) {
            case CH_KERNEL_MGS: ok = k >= 1 && k < m_max; break;
            case CH_KERNEL_MATVEC: ok = k >= 0 && k < m_max; break;
            case CH_KERNEL_PHI: ok = k >= 1 && k < m_max && k <= h.last_j; break;
            case CH_KERNEL_DC_MATVEC: ok = k >= 0 && k <= m_max; break;
            default: ok = k >= 0 && k < m_max;
        }
        if (!ok) return CH_EINVAL;
    }
    Member m{sh, prob->eps, prob->eyre, 0};
    Table t;
    if ((rc = build_table(ctx, {m}, sh.dim, prec, &t))) return rc;
    // A live control block.  Unit scales and zero totals: the timed passes
    // move every operand; values are not meaningful afterwards.  tol_phi = 0:
    // every phi test takes the not-converged branch (one exponential).
    h.done = 0;
    h.halted = 0;
    h.tol_phi = 0.0;
    for (int i = 0; i <= CH_MMAX; ++i) h.vscale[i] = 1.0;
    for (int i = 0; i < CH_DROWS; ++i) h.dt[i] = 0.0;
    for (int i = 0; i <= CH_MMAX; ++i) h.h1[0][i] = h.h1[1][i] = 0.0;
    if (kernel == CH_KERNEL_LIM_STAGE2 && !lim_stage_pairs(t)) return CH_EINVAL;
    if (lim) {
        // order 2, both stage positions with a_m = 0 (node beta_1)
        h.p = 2;
        h.lam = 1.0;
        if (!(h.tau0 > 0.0)) h.tau0 = 1e-9;
        const int ord[2] = {0, 1};
        const double cf[4] = {0.0, 1.0, 0.0, 1.0};
        HIP_TRY(ctx, hipMemcpyAsync(b.lorder, ord, sizeof(ord), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(b.lcoef, cf, sizeof(cf), hipMemcpyHostToDevice, ctx->stream));
    }
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(b.part, 0, 2 * sizeof(double) * CH_NRED * CH_MAXB, ctx->stream));
    const double* y = b.ybuf[0];
    const double N = double(sh.N);
    double bytes = 0.0;
    auto launch = [&](int k) -> hipError_t {
        PartSeq ps;
        ps.base = b.part;
        switch (kernel) {
            case CH_KERNEL_MGS:
                bytes += 4.0 * esz * N;   // read w, v_{i-1}, v_i; write w
                return launch_mgs_pass(t, prec, b, ps, k, 1, ctx->stream);
            case CH_KERNEL_MATVEC:
                bytes += 4.0 * esz * N;   // read v_k, the state, v_0; write w
                return launch_matvec(t, prec, b, ps, y, k, MV_DOTS_ONE, true, ctx->stream);
            case CH_KERNEL_PHI:
                return launch_phi(t, b, ps, k, k, true, ctx->stream);
            case CH_KERNEL_DC_MATVEC:   // read u_k, the state, q_0..q_{k-1}; write w (k < m_max)
                bytes += (k + 2 + (k < m_max ? 1 : 0)) * esz * N;
                return launch_matvec(t, prec, b, ps, y, k, MV_DOTS_DC, k < m_max, ctx->stream, true);
            case CH_KERNEL_DC_UPDATE:   // read q_0..q_{k-1}, u_k, w; write q_k, u_{k+1}
                bytes += (k + 4) * esz * N;
                return launch_dc_update(t, prec, b, k, ctx->stream, true);
            case CH_KERNEL_DC_ITER: {   // both passes and the dot totals between them
                bytes += (2 * k + 7) * esz * N;
                hipError_t e = launch_matvec(t, prec, b, ps, y, k, MV_DOTS_DC, true, ctx->stream, true);
                if (e == hipSuccess) e = launch_dots_reduce(t, b, k, ctx->stream);
                if (e == hipSuccess) e = launch_dc_update(t, prec, b, k, ctx->stream, true);
                return e;
            }
            case CH_KERNEL_LIM_STAGE2:  // read y^n, the stage before the pair; write the second
                bytes += 24.0 * N;
                return launch_lim_stage2(t, b, y, b.ybuf[1], 1, ctx->stream, true);
            default:                    // read y^n, the previous stage; write the next
                bytes += 24.0 * N;
                return launch_lim_stage(t, b, y, b.ybuf[1], 0, lim_stage_pairs(t), ctx->stream, true);
        }
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    auto timed_sequence = [&]() -> hipError_t {
        hipError_t e;
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) return e;
        if ((e = launch(lim ? 0 : iters[0])) != hipSuccess) return e;   // warm
        bytes = 0.0;
        if ((e = hipEventRecord(e0, ctx->stream)) != hipSuccess) return e;
        for (int i = 0; i < count; ++i)
            if ((e = launch(lim ? 0 : iters[i])) != hipSuccess) return e;
        if ((e = hipEventRecord(e1, ctx->stream)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
        return hipEventElapsedTime(&ms, e0, e1);
    };
    const hipError_t err = timed_sequence();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    HIP_TRY(ctx, err);
    *total_us = 1000.0 * ms;
    *total_bytes = bytes;
    return CH_OK;
}

static bool grid_ok(int dim, int n, int prec) {
    return (dim == 2 || dim == 3) && n >= 5 && (prec == CH_FP64 || prec == CH_FP32_MIXED);
}

static void put_shape(ch_ctx* ctx, int dim, int n, int prec, const ch_shape& s) {
    for (auto& e : ctx->shapes)
        if (e.dim == dim && e.n == n && e.prec == prec) {
            e.s = s;
            return;
        }
    ctx->shapes.push_back({dim, n, prec, s});
}

static void drop_shape(ch_ctx* ctx, int dim, int n, int prec) {
    auto& v = ctx->shapes;
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i].dim == dim && v[i].n == n && v[i].prec == prec) {
            v.erase(v.begin() + (long)i);
            return;
        }
}

int ch_get_shape(ch_ctx* ctx, int dim, int n, int prec, ch_shape* out) {
    if (!ctx || !out || !grid_ok(dim, n, prec)) return CH_EINVAL;
    const ch_shape* s = find_shape(ctx, dim, n, prec);
    *out = s ? *s : default_shape(dim, n, prec);
    return CH_OK;
}

int ch_set_shape(ch_ctx* ctx, int dim, int n, int prec, const ch_shape* shape) {
    if (!ctx || !grid_ok(dim, n, prec)) return CH_EINVAL;
    if (!shape) {
        drop_shape(ctx, dim, n, prec);
        return CH_OK;
    }
    if (!shape_ok(dim, n, prec, *shape)) return CH_EINVAL;
    put_shape(ctx, dim, n, prec, *shape);
    return CH_OK;
}

// Workgroup counts the shape tuners try below the built-in count d: d, 3d/4,
// d/2, d/4, and whole rounds of two, three and four workgroups per CU (all
// resident at once, each looping over an equal share); distinct, >= 1.
static std::vector<int> tuner_counts(const ch_ctx* ctx, int d) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) cus = 0;
    std::vector<int> v;
    for (int c : {d, (3 * d) / 4, d / 2, d / 4, 2 * cus, 3 * cus, 4 * cus})
        if (c >= 1 && c <= d && std::find(v.begin(), v.end(), c) == v.end()) v.push_back(c);
    return v;
}

int ch_tune_shape(ch_ctx* ctx, const ch_problem* prob, int m_max, ch_shape* best, double* best_us,
                  double* default_us) {
    if (!ctx || !best || !best_us || !default_us) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    Shape sh;
    int rc = check_problem(prob, &sh);
    if (rc) return rc;
    if (m_max < 2 || m_max > CH_MMAX) return CH_EINVAL;
    const int prec = prob->prec, dim = sh.dim, n = sh.n;
    if ((rc = ensure(ctx, pad64(sh.N), m_max, prec, 1, 0, false))) return rc;
    // the workspace of a run: zero fields and a live control block
    const DevBuffers& b = ctx->b;
    const size_t esz = prec == CH_FP64 ? sizeof(double) : sizeof(float);
    HIP_TRY(ctx, hipMemsetAsync(b.V, 0, (size_t)(m_max + 1) * b.ldv * esz, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(b.ybuf[0], 0, sizeof(double) * sh.N, ctx->stream));
    if (prec == CH_FP32_MIXED) HIP_TRY(ctx, hipMemsetAsync(b.y32, 0, sizeof(float) * sh.N, ctx->stream));
    init_ctl(ctx->hctl, MODE_EE, 0.0, 1e-6, INFINITY, 1e-4, 0.0, 0.0, m_max, 0, nullptr, 0, ctx->expect[0]);
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
    const ch_shape* prev = find_shape(ctx, dim, n, prec);
    const bool had = prev != nullptr;
    const ch_shape saved = had ? *prev : default_shape(dim, n, prec);
    const ch_shape dflt = default_shape(dim, n, prec);
    // per-iteration time of `kernel` with shape s: iterations 1, m_max/2,
    // m_max - 1 five times over, best of three sequences
    auto timed = [&](const ch_shape& s, int kernel, double* us) -> int {
        put_shape(ctx, dim, n, prec, s);
        const int its[3] = {1, m_max / 2, m_max - 1};
        int seq[15];
        for (int i = 0; i < 15; ++i) seq[i] = its[i % 3];
        double bt = INFINITY;
        for (int trial = 0; trial < 3; ++trial) {
            double t_us = 0.0, bytes = 0.0;
            const int r = time_kernel_core(ctx, sh, prob, kernel, m_max, seq, 15, &t_us, &bytes);
            if (r) return r;
            bt = std::min(bt, t_us / 15.0);
        }
        *us = bt;
        return CH_OK;
    };
    auto counts = [ctx](int d) { return tuner_counts(ctx, d); };
    auto restore = [&]() {
        if (had) put_shape(ctx, dim, n, prec, saved);
        else drop_shape(ctx, dim, n, prec);
    };
    std::vector<int> vxs;
    if (dim == 2) {
        for (int vx : {1, 2, 4})
            if (shape_ok(dim, n, prec, ch_shape{vx, 1, 1})) vxs.push_back(vx);
    } else {
        vxs.push_back(dflt.vx);
    }
    ch_shape bs = dflt;
    double bmv = INFINITY, dmv = INFINITY;
    for (int vx : vxs) {
        const int w0 = dim == 2 ? strip_blocks(n, vx) : dflt.wblk;
        for (int w : counts(w0)) {
            const ch_shape c{vx, w, dflt.cblk};
            double us;
            if ((rc = timed(c, CH_KERNEL_DC_MATVEC, &us))) {
                restore();
                return rc;
            }
            if (vx == dflt.vx && w == dflt.wblk) dmv = us;
            if (us < bmv) {
                bmv = us;
                bs = c;
            }
        }
    }
    double bup = INFINITY, dup = INFINITY;
    int bc = dflt.cblk;
    for (int c : counts(dflt.cblk)) {
        double us;
        if ((rc = timed(ch_shape{bs.vx, bs.wblk, c}, CH_KERNEL_DC_UPDATE, &us))) {
            restore();
            return rc;
        }
        if (c == dflt.cblk) dup = us;
        if (us < bup) {
            bup = us;
            bc = c;
        }
    }
    bs.cblk = bc;
    put_shape(ctx, dim, n, prec, bs);
    *best = bs;
    *best_us = bmv + bup;
    *default_us = dmv + dup;
    return CH_OK;
}

int ch_tune_batch_shapes(ch_ctx* ctx, int count, const ch_batch_item* items, int dim, int eyre, int prec, int m_max,
                         double* best_us, double* default_us) {
    if (!ctx || count < 1 || !items || !best_us || !default_us) return CH_EINVAL;
    if (prec != CH_FP64 && prec != CH_FP32_MIXED) return CH_EINVAL;
    if (m_max < 2 || m_max > CH_MMAX) return CH_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return CH_EDEVICE;
    std::vector<Member> ms(count);
    size_t pts = 0;
    for (int i = 0; i < count; ++i) {
        const int rc = check_grid(dim, items[i].n, items[i].eps, eyre, &ms[i].sh);
        if (rc) return rc;
        ms[i].eps = items[i].eps;
        ms[i].eyre = eyre;
        ms[i].off = pts;
        pts += pad64(ms[i].sh.N);
    }
    int rc;
    if ((rc = ensure(ctx, pts, m_max, prec, count, 0, false))) return rc;
    const DevBuffers& b = ctx->b;
    const size_t esz = prec == CH_FP64 ? sizeof(double) : sizeof(float);
    HIP_TRY(ctx, hipMemsetAsync(b.V, 0, (size_t)(m_max + 1) * b.ldv * esz, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(b.ybuf[0], 0, sizeof(double) * pts, ctx->stream));
    if (prec == CH_FP32_MIXED) HIP_TRY(ctx, hipMemsetAsync(b.y32, 0, sizeof(float) * pts, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(b.part, 0, 2 * sizeof(double) * CH_NRED * CH_MAXB, ctx->stream));
    for (int i = 0; i < count; ++i)
        init_ctl(ctx->hctl + i, MODE_EE, 0.0, 1e-6, INFINITY, 1e-4, 0.0, 0.0, m_max, 0, nullptr, 0, ctx->expect[i]);
    HIP_TRY(ctx, hipMemcpyAsync(b.ctl, ctx->hctl, sizeof(Ctl) * count, hipMemcpyHostToDevice, ctx->stream));
    // distinct sides, largest total size first
    std::vector<std::pair<long long, int>> sides;
    for (const Member& m : ms) {
        auto it = std::find_if(sides.begin(), sides.end(), [&](const auto& e) { return e.second == m.sh.n; });
        if (it == sides.end()) sides.push_back({m.sh.N, m.sh.n});
        else it->first += m.sh.N;
    }
    std::sort(sides.begin(), sides.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
    for (const auto& e : sides) drop_shape(ctx, dim, e.second, prec);   // start from the built-in shapes
    // one batched DCGS2 iteration: iterations 1, m/2, m - 1 five times over, best of three sequences
    auto timed = [&](double* us) -> int {
        Table t;
        int r = build_table(ctx, ms, dim, prec, &t);
        if (r) return r;
        PartSeq ps;
        ps.base = b.part;
        const int its[3] = {1, m_max / 2, m_max - 1};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float ms_ = 0.f;
        double bt = INFINITY;
        auto seq = [&]() -> hipError_t {
            hipError_t e;
            if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) return e;
            for (int trial = 0; trial < 4; ++trial) {   // the first is a warm sequence
                if ((e = hipEventRecord(e0, ctx->stream)) != hipSuccess) return e;
                for (int q = 0; q < 15; ++q) {
                    const int k = its[q % 3];
                    if ((e = launch_matvec(t, prec, b, ps, b.ybuf[0], k, MV_DOTS_DC, true, ctx->stream)) != hipSuccess)
                        return e;
                    if ((e = launch_dots_reduce(t, b, k, ctx->stream)) != hipSuccess) return e;
                    if ((e = launch_dc_update(t, prec, b, k, ctx->stream, false, false)) != hipSuccess) return e;
                }
                if ((e = hipEventRecord(e1, ctx->stream)) != hipSuccess) return e;
                if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
                if ((e = hipEventElapsedTime(&ms_, e0, e1)) != hipSuccess) return e;
                if (trial > 0) bt = std::min(bt, 1000.0 * ms_ / 15.0);
            }
            return hipSuccess;
        };
        const hipError_t err = seq();
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        HIP_TRY(ctx, err);
        *us = bt;
        return CH_OK;
    };
    auto counts = [ctx](int d) { return tuner_counts(ctx, d); };
    double cur;
    if ((rc = timed(&cur))) return rc;
    const double dflt_us = cur;
    for (const auto& e : sides) {
        const int n = e.second;
        ch_shape bs = default_shape(dim, n, prec);
        auto try_shape = [&](const ch_shape& c) -> int {
            put_shape(ctx, dim, n, prec, c);
            double us;
            const int r = timed(&us);
            if (r) return r;
            if (us < 0.995 * cur) {
                cur = us;
                bs = c;
            }
            put_shape(ctx, dim, n, prec, bs);
            return CH_OK;
        };
        const ch_shape d = bs;
        for (int vx : {1, 2, 4}) {
            if (dim == 3 && vx != d.vx) continue;
            if (!shape_ok(dim, n, prec, ch_shape{vx, 1, 1})) continue;
            const int w0 = dim == 2 ? strip_blocks(n, vx) : d.wblk;
            for (int w : counts(w0)) {
                if (vx == d.vx && w == d.wblk) continue;
                if ((rc = try_shape(ch_shape{vx, w, bs.cblk}))) return rc;
            }
        }
        for (int c : counts(d.cblk)) {
            if (c == bs.cblk) continue;
            if ((rc = try_shape(ch_shape{bs.vx, bs.wblk, c}))) return rc;
        }
        if (bs.vx == d.vx && bs.wblk == d.wblk && bs.cblk == d.cblk) drop_shape(ctx, dim, n, prec);
    }
    *best_us = cur;
    *default_us = dflt_us;
    return CH_OK;
}

int ch_server_create(int device, int prec, const ch_ee_opts* opts, size_t hbm_budget, int max_slots,
                     ch_server** out) {
    if (!out || !opts) return CH_EINVAL;
    *out = nullptr;
    if (prec != CH_FP64 && prec != CH_FP32_MIXED) return CH_EINVAL;
    if (opts->m_max < 1 || opts->m_max > CH_MMAX || opts->constant_step || !orth_ok(opts->orth) ||
        !graph_chunk_ok(opts))
        return CH_EINVAL;
    if (!(opts->tol > 0.0) && !(opts->tol_phi_fixed > 0.0)) return CH_EINVAL;
    if (max_slots < 1 || max_slots > 4096) return CH_EINVAL;
    const size_t esz = prec == CH_FP64 ? 8 : 4;
    const size_t per_pt = (size_t)(opts->m_max + 1) * esz + 28;
    const size_t pts = hbm_budget / per_pt / 64 * 64;
    if (pts < 64) return CH_EINVAL;
    ch_server* S = new (std::nothrow) ch_server();
    if (!S) return CH_ENOMEM;
    S->device = device;
    S->prec = prec;
    S->opts = *opts;
    S->max_slots = max_slots;
    S->pool_pts = pts;
    S->slot_req.assign(max_slots, nullptr);
    S->free_[0] = pts;
    int rc;
    // Non-blocking streams: neither the scheduler's work nor the request
    // copies wait for (or hold up) work on the null stream.
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
        delete S;
        return CH_EDEVICE;
    }
    if (hipStreamCreateWithFlags(&S->io, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(S->stream);
        delete S;
        return CH_EDEVICE;
    }
    if ((rc = ch_create(&S->ctx, device, S->stream)) != CH_OK ||
        (rc = ensure(S->ctx, pts, opts->m_max, prec, max_slots, 0, true)) != CH_OK) {
        if (S->ctx) ch_destroy(S->ctx);
        (void)hipStreamDestroy(S->io);
        (void)hipStreamDestroy(S->stream);
        delete S;
        return rc;
    }
    S->th = std::thread(serve_loop, S);
    *out = S;
    return CH_OK;
}

int ch_server_destroy(ch_server* S) {
    if (!S) return CH_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Req* r : S->queue) {
            r->state = CH_REQ_FAILED;
            r->status = CH_EBUSY;
        }
        S->queue.clear();
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    (void)hipSetDevice(S->device);
    for (auto& kv : S->reqs) {
        free_dev(kv.second->buf);
        delete kv.second;
    }
    for (auto& kv : S->spare) free_dev(kv.second);
    ch_destroy(S->ctx);
    (void)hipStreamDestroy(S->io);
    (void)hipStreamDestroy(S->stream);
    delete S;
    return CH_OK;
}

int ch_submit(ch_server* S, const ch_request* q, unsigned long long* ticket) {
    const double t_enter = now_s();   // latencies count from here
    if (!S || !q || !ticket || !q->y0) return CH_EINVAL;
    Shape sh;
    int rc = check_grid(2, q->n, q->eps, 0, &sh);
    if (rc) return rc;
    if (!(q->tau0 > 0.0) || (q->method != CH_METHOD_EE && q->method != CH_METHOD_LIM)) return CH_EINVAL;
    if ((q->steps < 1 && !(q->T < INFINITY)) || !(q->T > 0.0) || !(q->tol < INFINITY)) return CH_EINVAL;
    if (q->y0_on_host != 0 && q->y0_on_host != 1) return CH_EINVAL;
    Req* r = new (std::nothrow) Req();
    if (!r) return CH_ENOMEM;
    r->n = q->n;
    r->eps = q->eps;
    r->steps = q->steps;
    r->tau0 = q->tau0;
    r->method = q->method;
    r->T = q->T;
    r->tol = q->tol;
    r->N = sh.N;
    r->len = pad64(sh.N);
    inst_blocks(2, q->n, sh.N, &r->sblk, &r->cblk);
    r->wblk = wide_blocks(2, q->n, S->prec);
    if (r->len > S->pool_pts || r->sblk > CH_MAXB || r->cblk > CH_MAXB || r->wblk > CH_MAXB) {
        delete r;
        return CH_ENOMEM;
    }
    if (hipSetDevice(S->device) != hipSuccess || !(r->buf = take_buffer(S, sizeof(double) * r->N, &r->cap))) {
        (void)hipGetLastError();
        delete r;
        return CH_ENOMEM;
    }
    if (hipMemcpyAsync(r->buf, q->y0, sizeof(double) * r->N,
                       q->y0_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, S->io) != hipSuccess ||
        hipStreamSynchronize(S->io) != hipSuccess) {
        (void)hipGetLastError();
        give_buffer(S, r->buf, r->cap);
        delete r;
        return CH_EDEVICE;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            give_buffer(S, r->buf, r->cap);
            delete r;
            return S->fatal != CH_OK ? S->fatal : CH_EBUSY;
        }
        r->id = S->next_id++;
        r->t_submit = t_enter;
        S->reqs[r->id] = r;
        S->queue.push_back(r);
        *ticket = r->id;
    }
    S->cv.notify_all();
    return CH_OK;
}

int ch_poll(ch_server* S, unsigned long long ticket, int* state, double* y_out, ch_run_stats* stats,
            double* latency_s) {
    if (!S || !state) return CH_EINVAL;
    Req* r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) return CH_ENOENT;
        r = it->second;
        *state = r->state;
        if (stats) *stats = r->stats;
        if (latency_s) {
            const bool fin = r->state == CH_REQ_DONE || r->state == CH_REQ_FAILED;
            latency_s[0] = r->t_start > 0 ? r->t_start - r->t_submit : 0.0;
            latency_s[1] = fin ? r->t_done - r->t_start : 0.0;
            latency_s[2] = fin ? r->t_done - r->t_submit : 0.0;
        }
        if (!((r->state == CH_REQ_DONE || r->state == CH_REQ_FAILED) && y_out)) return r->status;
        S->reqs.erase(it);   // released: the result is handed over below
    }
    int rc = r->status;
    if (r->state == CH_REQ_DONE) {
        (void)hipSetDevice(S->device);
        if (hipMemcpyAsync(y_out, r->buf, sizeof(double) * r->N, hipMemcpyDeviceToDevice, S->io) != hipSuccess ||
            hipStreamSynchronize(S->io) != hipSuccess) {
            (void)hipGetLastError();
            rc = CH_EDEVICE;
        }
    }
    give_buffer(S, r->buf, r->cap);
    delete r;
    return rc;
}

}  // extern "C"
