// Internal declarations shared by the kernels and the host driver of libch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <vector>


#include "../../include/ch.h"

#define CH_LDH (CH_MMAX + 1)     // leading dimension of the Hessenberg matrix
#define CH_MAXB 32768            // most workgroups of a reducing launch (partials per reduction)
#define CH_SBLK_MAX 2048         // most stencil workgroups per instance (larger grids loop over tiles);
#ifndef CH_WBLK_MAX
#define CH_WBLK_MAX 2048         // most strip workgroups per instance (larger grids loop over strips)
#endif
                                 // <= 8 * CH_BLOCK partials per instance (sum_partials)
#ifndef CH_LOOKAHEAD
#define CH_LOOKAHEAD 2           // DCGS2 iterations the host issues ahead of the device's update launches
#endif
#define CH_LOOKAHEAD_WAIT_S 0.05 // longest host wait for that progress (then it issues anyway)
#define CH_PLAN_WAIT_S 1.0       // longest host wait for the LIM orders a plan publishes (then it copies them)
#ifndef CH_MARCH_L
#define CH_MARCH_L 16            // planes per run of the 3-D marching matvec
#endif
#ifndef CH_CBLK_MAX
#define CH_CBLK_MAX 512          // most streaming workgroups per instance
#endif
#define CH_NRED 4                // most sums reduced by one launch
#define CH_BLOCK 256             // threads per workgroup of the streaming and stencil kernels
#define CH_DROWS (2 * CH_MMAX + 2)   // dot-product rows of one DCGS2 iteration
#define CH_MSMALL 47                 // Krylov dimensions up to which the LDS-sized forms apply
#define CH_DROWS_SMALL (2 * CH_MSMALL + 2)

// Dot products a matvec launch produces (see k_matvec).
enum MatvecDots { MV_DOTS_ONE = 0, MV_DOTS_DC = 1 };

enum CtlMode { MODE_EE = 0, MODE_EE_CONST = 1, MODE_LIM = 2, MODE_LIM_CONST = 3, MODE_PHI = 4 };

// Device-resident control block: every scalar of the step controllers lives
// here, so a whole run is issued without host round trips (except where a
// launch count depends on device data: LIM's p and the number of restarted
// Krylov cycles).
struct Ctl {
    // run constants
    double T, tol, tol_phi_fixed, tau_min, tau_fixed;
    int mode, m_max, rec_cap, max_steps;   // max_steps <= 0: no step limit
    ch_step_record* rec;                   // rec_cap records (device), or null
    double mob0, mob1;                     // mobility M(c) = max(mob0 + mob1 (1 - c^2), 0) (Inst::mob)
    // run state
    double t, tau;
    int cur;         // ping-pong buffer holding the latest accepted state
    int halted;      // nothing more to do (t >= T or an error)
    int status;      // ch_status
    int steps;
    long long matvecs;
    int restarts, traces;
    int cyc;         // Krylov cycles begun (the host compares it with the cycles it issued)
    // current step
    double tau0;     // proposal of the current Krylov cycle (after the final-time clip)
    double tau_step; // whole step (constant mode: the fixed tau, clipped)
    double tau_acc;  // step covered by the last cycle
    double covered;  // constant mode: time covered by completed cycles
    double tol_phi, beta, gnorm, est, resnorm, lam;
    int clipped, done, j, converged, traced, p, cycles, mv_step;
    int last_j;      // Krylov dimension of the last finished step
    // Arnoldi
    double H[CH_LDH * CH_MMAX];   // h_{i+1,k+1} at H[i + k*CH_LDH]
    double vscale[CH_MMAX + 1];   // v_i = vscale[i] * V(:, i)
    // DCGS2: first-projection coefficients h' of the newest column, in two
    // buffers (iteration j reads [j & 1], writes [(j + 1) & 1]), and the
    // dot-product totals of the current iteration
    double h1[2][CH_MMAX + 1];
    double dt[CH_DROWS];
    double u[CH_MMAX];            // tau phi(-tau H) e_1
};

// One instance of a batch: a periodic grid whose fields live at `off` in
// every pooled array.  Kernels cover all instances of a batch in one launch;
// a block-to-instance map gives each workgroup its instance, and each
// instance owns a contiguous range of workgroups (and so of partials).
struct Inst {
    long long off;      // first point of the instance in the pooled arrays
    long long N;        // points
    int n;              // points per direction
    int slot;           // control block index
    int sblk0, sblk;    // stencil (tile) workgroups [sblk0, sblk0 + sblk)
    int cblk0, cblk;    // streaming workgroups [cblk0, cblk0 + cblk)
    double eps2, inv_h2;
    int eyre;
    int wblk0, wblk;    // 2-D row-strip / 3-D marching workgroups [wblk0, wblk0 + wblk)
    int vx;             // 2-D strips: columns per lane (divides n)
    int bc;             // ch_bc
    int mob;            // variable mobility, coefficients in the control block
};

// The mobility of a state value (Section 2, Remark 1).
template <typename T>
__host__ __device__ inline T mobility_of(T y, T m0, T m1) {
    const T m = m0 + m1 * (T(1) - y * y);
    return m > T(0) ? m : T(0);
}

// Grid index of a point g outside [0, n) (within n of it): periodic wrap,
// or the mirror of the cell-centred Neumann grid (ghost -1 -> 0, n -> n - 1).
__host__ __device__ inline int bc_index(int g, int n, int bc) {
    if (bc == CH_BC_NEUMANN) return g < 0 ? -g - 1 : (g >= n ? 2 * n - 1 - g : g);
    return g < 0 ? g + n : (g >= n ? g - n : g);
}

// 2-D row strips (ch_strip.hip): each wave of a strip workgroup owns a strip
// of CH_STRIP_ROWS rows by strip_cols(vx) columns; lane L holds vx
// consecutive columns, the first and last CH_STRIP_HALO(vx) lanes only halo.
// vx: 16-byte rows of the basis type (4 FP32 or 2 FP64 values), halved until
// it divides n.
#ifndef CH_STRIP_ROWS
#define CH_STRIP_ROWS 2
#endif
static_assert(CH_STRIP_ROWS <= 4, "strip rows: the periodic row wrap assumes n > CH_STRIP_ROWS (n >= 5)");
#ifndef CH_STRIP_WAVES
#define CH_STRIP_WAVES 4         // waves per workgroup of the 2-D strip kernels
#endif
#define CH_STRIP_BLOCK (64 * CH_STRIP_WAVES)
#define CH_STRIP_HALO(vx) ((vx) >= 2 ? 1 : 2)
__host__ __device__ constexpr int strip_cols(int vx) { return (64 - 2 * CH_STRIP_HALO(vx)) * vx; }
__host__ __device__ constexpr long long strip_count(int n, int vx) {
    return (long long)((n + strip_cols(vx) - 1) / strip_cols(vx)) * ((n + CH_STRIP_ROWS - 1) / CH_STRIP_ROWS);
}

// Kinds of workgroup ranges that produce reduction partials.
enum PartKind { PK_STREAM = 0, PK_TILE = 1, PK_STRIP = 2 };

struct DevBuffers {
    void* V;            // Krylov basis: (m_max + 1) pooled columns of ldv elements (FP64 or FP32)
    size_t ldv;
    double* ybuf[2];    // FP64 state ping-pong (pooled)
    double* fcur;       // FP64 f(y^n) (start vector of the step, unnormalised)
    float* y32;         // FP32 copy of y^n (mixed precision only)
    double* zbuf;       // FP64 scratch (LIM stages)
    double* part;       // reduction partials: two slots of CH_NRED * CH_MAXB
    double* dots;       // DCGS2 dot-product partials: CH_DROWS rows of CH_MAXB
    int* lorder;        // LIM node order, CH_PMAX per slot
    double* lcoef;      // LIM stage coefficients (tau a_m, 1 / (1 + tau a_m)) by stage position, 2 CH_PMAX per slot
    Ctl* ctl;           // control blocks, one per slot
    int* dflag;         // device view of `hflag`, one word per slot
    const volatile int* hflag;   // pinned host words: `cyc` of the last finished Krylov cycle per slot
    int* dprog;         // device view of `hprog`
    const volatile int* hprog;   // pinned host word: sequence number of the last DCGS2 update launch begun
    int* hseq;          // host counter of the DCGS2 update launches issued
    int* dcount;        // device counter of the DCGS2 update launches begun (mirrors hseq)
    int* dlim;          // device view of `hlim`
    const volatile int* hlim;   // pinned host words, per slot: the LIM plan's order p (0: halted), then its tag
    void* phibig;       // per-slot device scratch of the phi of orders above 48 (phi_big_bytes each)
};

// Bytes of the device scratch one instance needs for the phi tests of Krylov
// dimensions above CH_MSMALL (ch_krylov.hip).
size_t phi_big_bytes();

// The instance table of one launch sequence (device pointers + host mirror sizes).
struct Table {
    const Inst* inst;   // ninst entries
    const int* sb2i;    // stencil (tile) workgroup -> instance
    const int* cb2i;    // streaming workgroup -> instance
    const int* wb2i;    // 2-D strip workgroup -> instance
    int ninst, sgrid, cgrid, dim;
    int wgrid;          // 2-D strip / 3-D marching workgroups
    const Inst* hinst;  // host copy
};


// Partials of the grid reductions alternate between two slots: a producer
// writes slot `par`, the next consumer reads the other one (written by the
// previous producer).  `stencil` records which workgroup ranges produced them.
struct PartSeq {
    double* base = nullptr;
    int par = 0;
    int stencil = PK_STREAM;   // PartKind of the last producer
    double* in() const { return base + (size_t)(par ^ 1) * CH_NRED * CH_MAXB; }
    double* out() const { return base + (size_t)par * CH_NRED * CH_MAXB; }
    void produced(int kind) {
        stencil = kind;
        par ^= 1;
    }
};

// Kernel launchers (ch_stencil.hip, ch_krylov.hip); all asynchronous on `s`.
// `dim` and `prec` are common to all instances of a table.  Field arguments
// are pooled FP64 arrays; each instance reads and writes its slice at `off`.
hipError_t launch_resid(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, const double* z,
                        bool write_f, bool write_y32, hipStream_t s);
hipError_t launch_after_resid(const Table& t, const DevBuffers& b, PartSeq& ps, bool begin_step, hipStream_t s);
hipError_t launch_cycle_begin(const Table& t, const DevBuffers& b, hipStream_t s);
// dots (MatvecDots): MV_DOTS_ONE to the next partials slot, MV_DOTS_DC to
// b.dots.  store_w: write w to column k + 1.
// timing: the instantiation used by the timing aid (same code, another symbol).
hipError_t launch_matvec(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int k,
                         int dots, bool store_w, hipStream_t s, bool timing = false);
// DCGS2 passes of Arnoldi iteration k (see ch_krylov.hip).
hipError_t launch_dots_reduce(const Table& t, const DevBuffers& b, int k, hipStream_t s);
// 2-D row-strip forms (ch_strip.hip); every 2-D launch uses them.
inline bool uses_strips(const Table& t) { return t.dim == 2; }
// A single 2-D grid with variable mobility (batches have constant mobility).
inline bool mobility(const Table& t) { return t.ninst == 1 && t.hinst[0].mob != 0; }
hipError_t launch_matvec_strip(const Table& t, int prec, const DevBuffers& b, const double* y, int k, int dots,
                               bool store_w, double* pout, bool timing, hipStream_t s);
hipError_t launch_lim_stage_strip(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                                  bool pairs, bool timing, hipStream_t s);
hipError_t launch_lim_stage2_strip(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                                   bool timing, hipStream_t s);
hipError_t launch_est_ee_strip(const Table& t, int prec, const DevBuffers& b, const double* y0, const double* y1,
                               double* pout, hipStream_t s);
// 3-D DCGS2 matvec on z-marching x-y tiles (ch_march.hip); its workgroups are
// the instance's wblk range, so its partials are of kind PK_STRIP too.
hipError_t launch_matvec_march(const Table& t, int prec, const DevBuffers& b, const double* y, int k, bool store_w,
                               double* pout, bool timing, hipStream_t s);
// with_phi: the same launch runs the phi test of Krylov dimension j (one
// extra workgroup per instance; padded orders up to 32).
hipError_t launch_dc_update(const Table& t, int prec, const DevBuffers& b, int j, hipStream_t s,
                            bool timing = false, bool with_phi = false);
// The DCGS2 phi test of Krylov dimension j rides in the update launch of
// iteration j when its padded order fits that launch's LDS (j + 1 <= 32).
inline bool phi_in_update(int j) { return j + 1 <= 32; }
hipError_t launch_dc_finish(const Table& t, const DevBuffers& b, int j, hipStream_t s);
hipError_t launch_mgs_pass(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, int k, int i, hipStream_t s);
// phi test of iteration k (MGS: dimension k + 1, from the norm
// partials; dc: DCGS2 iteration k -- dimension k, then the update coefficients).
// Phi tests: MGS iteration k (dc false), or DCGS2 dimensions k .. k_last.
hipError_t launch_phi(const Table& t, const DevBuffers& b, PartSeq& ps, int k, int k_last, bool dc, hipStream_t s);
// Launch environment of the Arnoldi iterations: a second stream for the
// DCGS2 phi tests too large for the update launch (each waits for its
// iteration's update through ev_main, then overlaps the next iterations; the
// last test and the cycle's end wait for them through ev_side).
// Captured Arnoldi iterations: a graph per run of iterations [k0, k1) of a
// cycle, keyed by every value its launches take as arguments.
struct GraphEntry {
    std::vector<unsigned long long> key;
    hipGraphExec_t exec;
    int updates;            // DCGS2 update launches in the graph
};
struct GraphCache {
    std::vector<GraphEntry> e;
    size_t next = 0;        // the entry replaced when the cache is full
};
struct LaunchEnv {
    hipStream_t side;
    hipEvent_t ev_main, ev_side;
    hipStream_t cap;        // capture stream (a caller's stream may be the null stream)
    int graph_chunk;        // > 0: issue DCGS2 iterations as graphs of this many
    GraphCache* graphs;
};
void destroy_graphs(GraphCache& g);
// Arnoldi iteration k: matvec, Gram-Schmidt passes (orth: ch_orth), phi and
// residual test.  side_used (DCGS2): set when a test went to the second
// stream and the main stream has not yet waited for it.
hipError_t launch_arnoldi_iter(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int k,
                               int orth, int m_max, const LaunchEnv* env, hipStream_t s, bool* side_used = nullptr);
// True when every instance has reported the current cycle finished:
// expected[slot] is the number of cycles the host has issued for that slot.
bool all_cycles_done(const Table& t, const DevBuffers& b, const int* expected);
// Issues the Arnoldi iterations of one Krylov cycle; stops issuing once every
// instance has reported the cycle finished (later launches would exit at once).
hipError_t launch_arnoldi(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int m_max,
                          int orth, const int* expected, const LaunchEnv* env, hipStream_t s);
// unit: the basis is stored normalised (DCGS2)
hipError_t launch_update(const Table& t, int prec, const DevBuffers& b, const double* y, double* ynew, bool unit,
                         hipStream_t s);
hipError_t launch_est_ee(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y0,
                         const double* y1, hipStream_t s);
hipError_t launch_step_end(const Table& t, const DevBuffers& b, PartSeq& ps, bool begin_next, hipStream_t s);
hipError_t launch_lim_begin(const Table& t, const DevBuffers& b, PartSeq& ps, const double* y, hipStream_t s);
// seq: the tag the plan writes beside each instance's order in the pinned
// words (when the buffers have them).
hipError_t launch_lim_plan(const Table& t, const DevBuffers& b, PartSeq& ps, int seq, hipStream_t s);
// Launch l of the stages of a LIM step whose Chebyshev order p each
// instance reads from its control block: single stages (pairs = 0: 2p - 1
// launches, stage l), or stage 0 alone and then two stages per launch
// (pairs = 1: p launches, stages 2l - 1 and 2l).  The launches ping-pong
// between zbuf and yout so that each instance's last launch writes yout;
// launch 0 reads y^n.  Launches past an instance's last do nothing for it,
// so one sequence serves a batch whose members have different p.
struct LimLaunch {
    int pos;            // first stage position of the launch
    const double* src;  // the previous stage (y^n for launch 0)
    double* dst;
    bool live;
};
__host__ __device__ inline LimLaunch lim_launch(int p, int l, bool pairs, const double* yin, double* yout,
                                                double* zbuf) {
    const int nl = pairs ? p : 2 * p - 1;
    LimLaunch L;
    L.live = l < nl;
    L.pos = pairs ? (l == 0 ? 0 : 2 * l - 1) : l;
    L.dst = ((nl - 1 - l) & 1) == 0 ? yout : zbuf;
    L.src = l == 0 ? yin : (((nl - l) & 1) == 0 ? yout : zbuf);
    return L;
}
// Launches of one LIM step of order p.
inline int lim_launches(int p, bool pairs) { return pairs ? p : 2 * p - 1; }
// Stage launch l (a single stage; with pairs only l = 0).
hipError_t launch_lim_stage(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l, bool pairs,
                            hipStream_t s, bool timing = false);
// Two stages per launch (2-D strips only: lim_stage_pairs), launch l >= 1.
inline bool lim_stage_pairs(const Table& t) { return uses_strips(t); }
hipError_t launch_lim_stage2(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                             hipStream_t s, bool timing = false);
hipError_t launch_est_lim(const Table& t, const DevBuffers& b, PartSeq& ps, const double* y0, const double* y1,
                          hipStream_t s);
hipError_t launch_lim_end(const Table& t, const DevBuffers& b, PartSeq& ps, hipStream_t s);
