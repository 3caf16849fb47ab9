// Internal declarations shared by the kernels and the host driver of libch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/ch.h"

#define CH_LDH (CH_MMAX + 1)     // leading dimension of the Hessenberg matrix
#define CH_MAXB 4096             // most workgroups of a reducing launch (partials per reduction)
#define CH_NRED 4                // most sums reduced by one launch
#define CH_BLOCK 256             // threads per workgroup of the streaming and stencil kernels

enum CtlMode { MODE_EE = 0, MODE_EE_CONST = 1, MODE_LIM = 2, MODE_LIM_CONST = 3, MODE_PHI = 4 };

// Device-resident control block: every scalar of the step controllers lives
// here, so a whole run is issued without host round trips (except where a
// launch count depends on device data: LIM's p and the number of restarted
// Krylov cycles).
struct Ctl {
    // run constants
    double T, tol, tol_phi_fixed, tau_min, tau_fixed;
    int mode, m_max, rec_cap, pad0;
    // run state
    double t, tau;
    int cur;         // ping-pong buffer holding the latest accepted state
    int halted;      // nothing more to do (t >= T or an error)
    int status;      // ch_status
    int steps;
    long long matvecs;
    int restarts, traces;
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
    double u[CH_MMAX];            // tau phi(-tau H) e_1
};

struct DevBuffers {
    void* V;            // Krylov basis, (m_max + 1) columns of ldv elements (FP64 or FP32)
    size_t ldv;
    double* ybuf[2];    // FP64 state ping-pong
    double* fcur;       // FP64 f(y^n) (start vector of the step, unnormalised)
    float* y32;         // FP32 copy of y^n (mixed precision only)
    double* zbuf;       // FP64 scratch (LIM stages)
    double* part;       // reduction partials: two slots of CH_NRED * CH_MAXB
    Ctl* ctl;
    ch_step_record* rec;
    int* dflag;                  // device view of `hflag`
    const volatile int* hflag;   // pinned host word: id of the last finished Krylov cycle
};

struct Grid {
    int dim, n;
    long long N;
    double eps2, inv_h2;
    int eyre;
};

// Partials of the grid reductions alternate between two slots: a producer
// writes slot `par`, the next consumer reads the other one (written by the
// previous producer).
struct PartSeq {
    double* base = nullptr;
    int par = 0;
    int np = 0;   // workgroups (partials) of the last producer
    double* in() const { return base + (size_t)(par ^ 1) * CH_NRED * CH_MAXB; }
    double* out() const { return base + (size_t)par * CH_NRED * CH_MAXB; }
    void produced(int G) {
        np = G;
        par ^= 1;
    }
};

// Kernel launchers (ch_stencil.hip, ch_krylov.hip); all asynchronous on `s`.
hipError_t launch_resid(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, const double* y, const double* z,
                        bool write_f, bool write_y32, hipStream_t s);
hipError_t launch_after_resid(const DevBuffers& b, PartSeq& ps, bool begin_step, hipStream_t s);
hipError_t launch_cycle_begin(const DevBuffers& b, hipStream_t s);
hipError_t launch_matvec(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int k,
                         hipStream_t s);
hipError_t launch_mgs_pass(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, int k, int i, hipStream_t s);
hipError_t launch_phi(const DevBuffers& b, PartSeq& ps, int k, int cycle_id, hipStream_t s);
// Issues the Arnoldi iterations of one Krylov cycle; stops issuing once the
// device has reported the cycle finished (those launches would exit at once).
hipError_t launch_arnoldi(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int m_max,
                          int cycle_id, hipStream_t s);
hipError_t launch_update(const Grid& g, int prec, const DevBuffers& b, const double* y, double* ynew, hipStream_t s);
hipError_t launch_est_ee(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, const double* y0,
                         const double* y1, hipStream_t s);
hipError_t launch_step_end(const DevBuffers& b, PartSeq& ps, bool begin_next, hipStream_t s);
hipError_t launch_lim_begin(const Grid& g, const DevBuffers& b, PartSeq& ps, const double* y, hipStream_t s);
hipError_t launch_lim_plan(const Grid& g, const DevBuffers& b, PartSeq& ps, hipStream_t s);
hipError_t launch_lim_stage(const Grid& g, const DevBuffers& b, const double* y, const double* z, double* out,
                            int m, hipStream_t s);
hipError_t launch_est_lim(const Grid& g, const DevBuffers& b, PartSeq& ps, const double* y0, const double* y1,
                          hipStream_t s);
hipError_t launch_lim_end(const DevBuffers& b, PartSeq& ps, hipStream_t s);
