// Arnoldi with modified Gram-Schmidt, the small-matrix phi with the
// residual-time restart, the solution update and the per-step controllers.
//
// Krylov algorithm of Fig. 3 (Section 4.1): for j = 1..m_max,
//   w = Ahat v_j;  h_ij = w^T v_i, w -= h_ij v_i (i = 1..j);  h_{j+1,j} = ||w||;
//   u = tau0 phi(-tau0 H_jj) e_1;  resnorm = h_{j+1,j} |e_j^T u|  (eq. rm);
//   converged if resnorm <= tol_phi, else at j = m_max shrink tau to the
//   largest step whose residual passes (eq. phi_stop);
// then y^{n+1} = y^n + V_j (beta u).
//
// Storage: column i of the basis is kept unnormalised, v_i = vscale[i] V(:,i),
// so the normalisation of line 21 is folded into the next reads.  One launch
// covers every instance of a batch; streaming kernels give each instance the
// workgroups [cblk0, cblk0 + cblk) (map cb2i), single-workgroup kernels one
// workgroup per instance.
#include "ch_common.h"

namespace {

// ---------------------------------------------------------------------------
// MGS pass i of Arnoldi iteration k (0-based columns):
//   h_{i-1,k} = <w, v_{i-1}> from the previous launch's partials;
//   w -= h_{i-1,k} v_{i-1};  partials of <w, v_i>  (or of ||w||^2 when FINAL).
// FP64 accumulation of the dot products in both precisions.
// ---------------------------------------------------------------------------
template <typename TV, bool FINAL, bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_mgs(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                  const int* __restrict__ cb2i, const Inst inst0, int ninst, TV* __restrict__ V, size_t ldv, int k,
                                                  int i, const double* __restrict__ pin, int pin_stencil,
                                                  double* __restrict__ pout) {
    const Inst I = SINGLE ? inst0 : insts[cb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    // the exit flag and the partials are fetched together (the partials of a
    // finished cycle are simply not used)
    const int finished = ctl->done | ctl->halted;
    using VT = typename Vec16<TV>::type;
    constexpr int VW = Vec16<TV>::W;
    TV* W = V + (size_t)(k + 1) * ldv + I.off;
    const TV* Vp = V + (size_t)(FINAL ? k : i - 1) * ldv + I.off;
    const TV* Vn = V + (size_t)i * ldv + I.off;
    double dot[1];
    sum_inst_partials<1, RED_SUM>(pin, I, pin_stencil, dot);
    if (finished) return;
    const double sp = ctl->vscale[i - 1];
    const double h = sp * dot[0];
    if (blockIdx.x == I.cblk0 && threadIdx.x == 0) ctl->H[(i - 1) + k * CH_LDH] = h;
    const TV c = TV(sp * h);
    double acc = 0.0;
    const long long N = I.N;
    const long long NV = N / VW;
    VT* W4 = reinterpret_cast<VT*>(W);
    const VT* P4 = reinterpret_cast<const VT*>(Vp);
    const VT* N4 = reinterpret_cast<const VT*>(Vn);
    const long long stride = (long long)I.cblk * CH_BLOCK;
    const long long first = (long long)(blockIdx.x - I.cblk0) * CH_BLOCK + threadIdx.x;
    for (long long q = first; q < NV; q += stride) {
        VT w = W4[q];
        const VT p = P4[q];
        TV* we = reinterpret_cast<TV*>(&w);
        const TV* pe = reinterpret_cast<const TV*>(&p);
#pragma unroll
        for (int e = 0; e < VW; ++e) we[e] = we[e] - c * pe[e];
        W4[q] = w;
        if (FINAL) {
#pragma unroll
            for (int e = 0; e < VW; ++e) acc += double(we[e]) * double(we[e]);
        } else {
            const VT nv = N4[q];
            const TV* ne = reinterpret_cast<const TV*>(&nv);
#pragma unroll
            for (int e = 0; e < VW; ++e) acc += double(we[e]) * double(ne[e]);
        }
    }
    for (long long q = NV * VW + first; q < N; q += stride) {
        const TV w = W[q] - c * Vp[q];
        W[q] = w;
        acc += FINAL ? double(w) * double(w) : double(w) * double(Vn[q]);
    }
    double x[1] = {acc};
    write_partials<1, RED_SUM>(x, pout);
}

// ---------------------------------------------------------------------------
// y^{n+1} = y^n + V_j (beta u)  (Fig. 3, line 23)
// ---------------------------------------------------------------------------
template <typename TV, bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_update(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                     const int* __restrict__ cb2i, const Inst inst0, int ninst, const double* ybase,
                                                     const TV* __restrict__ V, size_t ldv, double* ynewbase) {
    // ybase may alias ynewbase (restart cycles update the sub-step state in place)
    const Inst I = SINGLE ? inst0 : insts[cb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    __shared__ double cf[CH_MMAX];
    const int j = ctl->j;
    if ((int)threadIdx.x < j) cf[threadIdx.x] = ctl->beta * ctl->u[threadIdx.x] * ctl->vscale[threadIdx.x];
    __syncthreads();
    const double* y = ybase + I.off;
    double* ynew = ynewbase + I.off;
    const TV* Vi = V + I.off;
    const long long stride = (long long)I.cblk * CH_BLOCK;
    for (long long q = (long long)(blockIdx.x - I.cblk0) * CH_BLOCK + threadIdx.x; q < I.N; q += stride) {
        double acc = 0.0;
        for (int i = 0; i < j; ++i) acc += cf[i] * double(Vi[(size_t)i * ldv + q]);
        ynew[q] = y[q] + acc;
    }
}

// ---------------------------------------------------------------------------
// Small-matrix exponential.  exp([[X, b], [0, 0]]) = [[e^X, phi(X) b], [0, 1]]
// (phi of eq. phi), so with X = -s H_jj and b = s e_1 the last column holds
// u = s phi(-s H_jj) e_1 and the first column exp(-s H_jj) e_1 = du/ds.
// Evaluated by scaling and squaring with the diagonal [13/13] Pade
// approximant (Higham, SIAM J. Matrix Anal. Appl. 26 (2005) 1179-1193: degree
// 13, theta_13 = 5.371920351148152 for the 1-norm), all in FP64 LDS.
// ---------------------------------------------------------------------------
constexpr int PLD = CH_MMAX + 1;
constexpr double THETA13 = 5.371920351148152;
constexpr int NLVL = 80;

struct PhiShared {
    double B[6][PLD * PLD];
    double c[14];        // Pade coefficients
    double lvl[NLVL];    // lvl[kk] = resnorm at s 2^-kk from the squaring chain
    double red;
    int ired;
};

__device__ void mm(double* __restrict__ C, const double* __restrict__ A, const double* __restrict__ B, int n) {
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int r = idx / n, c = idx - r * n;
        const double* a = A + r * PLD;
        double acc = 0.0;
        for (int l = 0; l < n; ++l) acc = fma(a[l], B[l * PLD + c], acc);
        C[r * PLD + c] = acc;
    }
    __syncthreads();
}

// Solve Q X = P in place (X overwrites P) by Gaussian elimination with
// partial pivoting.
__device__ void lu_solve(PhiShared& S, double* Q, double* P, int n) {
    for (int col = 0; col < n; ++col) {
        if (threadIdx.x < 64) {
            const int r = col + threadIdx.x;
            double v = r < n ? fabs(Q[r * PLD + col]) : -1.0;
            int idx = r;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(v, off, 64);
                const int oi = __shfl_xor(idx, off, 64);
                if (ov > v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            if (threadIdx.x == 0) S.ired = idx;
        }
        __syncthreads();
        const int piv = S.ired;
        if (piv != col) {
            for (int c = threadIdx.x; c < 2 * n; c += CH_BLOCK) {
                double* Mx = c < n ? Q : P;
                const int cc = c < n ? c : c - n;
                const double tmp = Mx[col * PLD + cc];
                Mx[col * PLD + cc] = Mx[piv * PLD + cc];
                Mx[piv * PLD + cc] = tmp;
            }
        }
        __syncthreads();
        const double pv = Q[col * PLD + col];
        const int rows = n - col - 1, qc = n - col - 1, cols = qc + n;
        for (int idx = threadIdx.x; idx < rows * cols; idx += CH_BLOCK) {
            const int rr = col + 1 + idx / cols;
            const int kk = idx % cols;
            const double l = Q[rr * PLD + col] / pv;
            if (kk < qc) {
                const int cc = col + 1 + kk;
                Q[rr * PLD + cc] -= l * Q[col * PLD + cc];
            } else {
                const int cc = kk - qc;
                P[rr * PLD + cc] -= l * P[col * PLD + cc];
            }
        }
        __syncthreads();
    }
    for (int col = n - 1; col >= 0; --col) {
        const double pv = Q[col * PLD + col];
        for (int c = threadIdx.x; c < n; c += CH_BLOCK) P[col * PLD + c] /= pv;
        __syncthreads();
        for (int idx = threadIdx.x; idx < col * n; idx += CH_BLOCK) {
            const int rr = idx / n, c = idx - rr * n;
            P[rr * PLD + c] -= Q[rr * PLD + col] * P[col * PLD + c];
        }
        __syncthreads();
    }
}

// exp(s [[-H_jj, e_1], [0, 0]]); returns the LDS matrix holding it and the
// number of squarings in *nsq_out.  Records resnorm at every dyadic level of
// the squaring chain in S.lvl.
__device__ const double* expm_aug(PhiShared& S, const double* __restrict__ H, int j, double s, double hnext,
                                  int* nsq_out) {
    const int n = j + 1;
    double* M = S.B[0];
    double* A2 = S.B[1];
    double* A4 = S.B[2];
    double* A6 = S.B[3];
    double* T1 = S.B[4];
    double* T2 = S.B[5];
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int r = idx / n, c = idx - r * n;
        double v = 0.0;
        if (r < j && c < j) v = -s * H[r + c * CH_LDH];
        else if (r == 0 && c == j) v = s;
        M[r * PLD + c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double cs = 0.0;
        if ((int)threadIdx.x < n)
            for (int r = 0; r < n; ++r) cs += fabs(M[r * PLD + threadIdx.x]);
        cs = wave_max(cs);
        if (threadIdx.x == 0) S.red = cs;
    }
    __syncthreads();
    const double nrm = S.red;
    int nsq = 0;
    if (nrm > THETA13 && nrm < __builtin_inf()) nsq = (int)ceil(log2(nrm / THETA13));
    if (nsq > 1100) nsq = 1100;
    const double scale = ldexp(1.0, -nsq);
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int r = idx / n, c = idx - r * n;
        M[r * PLD + c] *= scale;
    }
    __syncthreads();
    const double* cf = S.c;
    mm(A2, M, M, n);
    mm(A4, A2, A2, n);
    mm(A6, A4, A2, n);
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int o = (idx / n) * PLD + idx % n;
        T1[o] = cf[13] * A6[o] + cf[11] * A4[o] + cf[9] * A2[o];
    }
    __syncthreads();
    mm(T2, A6, T1, n);
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int r = idx / n, c = idx - r * n, o = r * PLD + c;
        T2[o] += cf[7] * A6[o] + cf[5] * A4[o] + cf[3] * A2[o] + (r == c ? cf[1] : 0.0);
    }
    __syncthreads();
    mm(T1, M, T2, n);   // U (odd part)
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int o = (idx / n) * PLD + idx % n;
        T2[o] = cf[12] * A6[o] + cf[10] * A4[o] + cf[8] * A2[o];
    }
    __syncthreads();
    mm(M, A6, T2, n);
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int r = idx / n, c = idx - r * n, o = r * PLD + c;
        const double V = M[o] + cf[6] * A6[o] + cf[4] * A4[o] + cf[2] * A2[o] + (r == c ? cf[0] : 0.0);
        const double U = T1[o];
        A2[o] = V + U;   // numerator p(M)
        A4[o] = V - U;   // denominator q(M) = p(-M)
    }
    __syncthreads();
    lu_solve(S, A4, A2, n);
    double* X = A2;
    double* Y = A6;
    if (threadIdx.x == 0 && nsq < NLVL) S.lvl[nsq] = hnext * fabs(X[(j - 1) * PLD + j]);
    for (int i = 1; i <= nsq; ++i) {
        mm(Y, X, X, n);
        double* tmp = X;
        X = Y;
        Y = tmp;
        const int kk = nsq - i;
        if (threadIdx.x == 0 && kk < NLVL) S.lvl[kk] = hnext * fabs(X[(j - 1) * PLD + j]);
    }
    __syncthreads();
    *nsq_out = nsq;
    return X;
}

__device__ void store_u(Ctl* ctl, const double* E, int j) {
    for (int i = threadIdx.x; i < j; i += CH_BLOCK) ctl->u[i] = E[i * PLD + j];
}

// ---------------------------------------------------------------------------
// phi of the Hessenberg matrix after Arnoldi iteration k, convergence test and
// residual-time trace (Fig. 3, lines 10-20).  One workgroup.
//
// Trace: the squaring chain of the evaluation at tau0 gives resnorm at every
// s = tau0 2^-kk; the largest passing one brackets the crossing in
// [tau0 2^-kk, tau0 2^(1-kk)] (further halvings are evaluated if the chain is
// too short).  The crossing resnorm(s) = tol_phi is then located by Newton's
// method on log resnorm against log s, using d resnorm/ds =
// h_{j+1,j} |e_j^T exp(-s H) e_1| from the same exponential, safeguarded by the
// bracket, to a relative precision of about 1e-14.
// ---------------------------------------------------------------------------
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_phi(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst, int k,
                                                  const double* __restrict__ pin, int pin_stencil,
                                                  int* __restrict__ dflags) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];   // one workgroup per instance
    Ctl* ctl = ctls + I.slot;
    int* dflag = dflags ? dflags + I.slot : nullptr;
    if (ctl->done | ctl->halted) return;
    __shared__ PhiShared S;
    // h_{k+2,k+1} = ||w|| from the final Gram-Schmidt pass (Fig. 3, line 9)
    double nrm2[1];
    sum_inst_partials<1, RED_SUM>(pin, I, pin_stencil, nrm2);
    const double hnext = sqrt(nrm2[0]);
    if (threadIdx.x == 0) {
        ctl->H[(k + 1) + k * CH_LDH] = hnext;
        ctl->vscale[k + 1] = hnext > 0.0 ? 1.0 / hnext : 0.0;
    }
    if (threadIdx.x == 0) {
        // [13/13] Pade coefficients of exp: c_0 = 1, c_{i+1} = c_i (13 - i) / ((26 - i)(i + 1))
        double c = 1.0;
        S.c[0] = 1.0;
        for (int i = 0; i < 13; ++i) {
            c = c * double(13 - i) / (double(26 - i) * double(i + 1));
            S.c[i + 1] = c;
        }
    }
    __syncthreads();
    __syncthreads();   // H column k complete (written by the Gram-Schmidt launches and above)
    const int j = k + 1;
    const double* H = ctl->H;
    const double tau0 = ctl->tau0, tol = ctl->tol_phi;
    int nsq = 0;
    const double* E = expm_aug(S, H, j, tau0, hnext, &nsq);
    const double res0 = hnext * fabs(E[(j - 1) * PLD + j]);
    if (!(res0 < __builtin_inf())) {
        if (threadIdx.x == 0) {
            ctl->status = CH_ENONFINITE;
            ctl->halted = 1;
            ctl->done = 1;
            if (dflag) *dflag = ctl->cyc;
            ctl->j = 0;
        }
        return;
    }
    if (res0 <= tol) {
        store_u(ctl, E, j);
        if (threadIdx.x == 0) {
            ctl->tau_acc = tau0;
            ctl->resnorm = res0;
            ctl->converged = 1;
            ctl->done = 1;
            if (dflag) *dflag = ctl->cyc;
            ctl->j = j;
        }
        return;
    }
    if (j < ctl->m_max) {
        if (threadIdx.x == 0) ctl->resnorm = res0;
        return;
    }
    // ---- trace: largest passing dyadic step below tau0 ----
    const double tau_min = ctl->tau_min;
    double lo = -1.0, hi = 0.0, rlo = 0.0, rhi = 0.0;
    const int kmax = nsq < NLVL - 1 ? nsq : NLVL - 1;
    for (int kk = 1; kk <= kmax; ++kk) {
        if (S.lvl[kk] <= tol) {
            lo = ldexp(tau0, -kk);
            rlo = S.lvl[kk];
            hi = 2.0 * lo;
            rhi = S.lvl[kk - 1];
            break;
        }
    }
    bool underflow = false;
    if (lo < 0.0) {
        double prev = S.lvl[kmax];
        for (int kk = kmax + 1;; ++kk) {
            const double s = ldexp(tau0, -kk);
            if (kk > 1100 || s == 0.0 || s < tau_min) {
                underflow = true;
                break;
            }
            int nq;
            const double* Es = expm_aug(S, H, j, s, hnext, &nq);
            const double r = hnext * fabs(Es[(j - 1) * PLD + j]);
            if (r <= tol) {
                lo = s;
                rlo = r;
                hi = 2.0 * s;
                rhi = prev;
                break;
            }
            prev = r;
        }
    }
    if (!underflow && lo < tau_min) underflow = true;
    if (underflow) {
        if (threadIdx.x == 0) {
            ctl->status = CH_ETAU_UNDERFLOW;
            ctl->halted = 1;
            ctl->done = 1;
            if (dflag) *dflag = ctl->cyc;
            ctl->j = 0;
        }
        return;
    }
    // ---- refine the crossing inside [lo, hi] ----
    double s;
    if (rlo > 0.0 && rhi > rlo) s = lo * exp2(log2(tol / rlo) / log2(rhi / rlo));
    else s = 0.5 * (lo + hi);
    if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
    for (int it = 0; it < 60; ++it) {
        int nq;
        const double* Es = expm_aug(S, H, j, s, hnext, &nq);
        const double uj = Es[(j - 1) * PLD + j];
        const double r = hnext * fabs(uj);
        const double dr = hnext * (uj >= 0.0 ? 1.0 : -1.0) * Es[(j - 1) * PLD + 0];
        if (r <= tol) {
            lo = s;
            rlo = r;
        } else {
            hi = s;
            rhi = r;
        }
        if (hi - lo <= 0x1p-47 * lo) {
            s = lo;
            break;
        }
        double sn = -1.0;
        if (r > 0.0 && dr > 0.0) sn = s * exp(-log(r / tol) * r / (s * dr));
        if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        if (fabs(sn - s) <= 1e-14 * s) {
            s = sn;
            break;
        }
        s = sn;
    }
    int nq;
    const double* Ef = expm_aug(S, H, j, s, hnext, &nq);
    store_u(ctl, Ef, j);
    if (threadIdx.x == 0) {
        ctl->tau_acc = s;
        ctl->resnorm = hnext * fabs(Ef[(j - 1) * PLD + j]);
        ctl->converged = 0;
        ctl->traced = 1;
        ctl->done = 1;
            if (dflag) *dflag = ctl->cyc;
        ctl->j = j;
    }
}

// ---------------------------------------------------------------------------
// Step begin (Fig. 4, lines 3-7): final-time clip and tol_phi (eq. tol_phi).
// ---------------------------------------------------------------------------
__device__ void begin_step(Ctl* ctl) {
    if (ctl->halted) return;
    if (!(ctl->t < ctl->T) || (ctl->max_steps > 0 && ctl->steps >= ctl->max_steps)) {
        ctl->halted = 1;
        return;
    }
    double tau = ctl->tau;
    int clipped = 0;
    if (ctl->t + tau > ctl->T) {
        tau = ctl->T - ctl->t;
        clipped = 1;
    }
    ctl->cyc += 1;
    ctl->clipped = clipped;
    ctl->tau0 = tau;
    ctl->tau_step = tau;
    ctl->covered = 0.0;
    ctl->cycles = 1;
    ctl->mv_step = 0;
    if (ctl->tol_phi_fixed > 0.0) {
        ctl->tol_phi = ctl->tol_phi_fixed;
    } else {
        const double first = ctl->beta > 0.0 ? ctl->gnorm / (10.0 * ctl->beta) : __builtin_inf();
        ctl->tol_phi = fmax(fmin(fmin(first, 0.1), 10.0 * ctl->tol), 1e-7);
    }
    ctl->done = 0;
    ctl->j = 0;
    ctl->converged = 0;
    ctl->traced = 0;
    ctl->resnorm = 0.0;
    ctl->vscale[0] = ctl->beta > 0.0 ? 1.0 / ctl->beta : 0.0;
    if (ctl->beta == 0.0) {   // y^n is a steady state of the linearised problem
        ctl->done = 1;
        ctl->converged = 1;
        ctl->tau_acc = tau;
    }
}

// After a residual start vector: beta = ||v_1||, ||ghat||; then either the
// begin of a step or (restart cycles) the normalisation of the new start.
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_after_resid(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst,
                                                          const double* __restrict__ pin, int pin_stencil, int begin) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    double tot[2];
    sum_inst_partials<2, RED_SUM>(pin, I, pin_stencil, tot);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(tot[0]), gn = sqrt(tot[1]);
    if (!(beta < __builtin_inf()) || !(gn < __builtin_inf())) {
        ctl->status = CH_ENONFINITE;
        ctl->halted = 1;
        return;
    }
    ctl->beta = beta;
    if (begin) {
        ctl->gnorm = gn;
        begin_step(ctl);
        return;
    }
    ctl->vscale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    if (beta == 0.0) {
        ctl->done = 1;
        ctl->converged = 1;
        ctl->tau_acc = ctl->tau0;
    }
}

// Between linear RT restart cycles of a constant step: account for the cycle
// just finished and aim the next one at the remaining time.
template <bool SINGLE>
__global__ void k_cycle_begin(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst) {
    Ctl* ctl = ctls + (SINGLE ? inst0.slot : insts[blockIdx.x].slot);
    if (threadIdx.x != 0 || ctl->halted || ctl->converged) return;
    ctl->cyc += 1;
    ctl->covered += ctl->tau_acc;
    ctl->restarts += 1;
    ctl->mv_step += 1 + ctl->j;
    ctl->cycles += 1;
    ctl->tau0 = ctl->tau_step - ctl->covered;
    ctl->done = 0;
    ctl->j = 0;
    ctl->converged = 0;
    ctl->traced = 0;
}

// ---------------------------------------------------------------------------
// EE2 step end (Fig. 4, lines 8-10): est (eq. LIMest), t, tau_new (eq. EEdt);
// optionally the begin of the next step.
// ---------------------------------------------------------------------------
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_step_end(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst,
                                                       const double* __restrict__ pin, int pin_stencil,
                                                       int begin_next) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    double tot[4];
    sum_inst_partials<4, RED_SUM>(pin, I, pin_stencil, tot);
    if (threadIdx.x != 0) return;
    const double num = sqrt(tot[0]), den = sqrt(tot[1]);
    const double est = den > 0.0 ? num / den : 0.0;
    const double beta = sqrt(tot[2]), gn = sqrt(tot[3]);
    if (!(est < __builtin_inf()) || !(beta < __builtin_inf()) || !(gn < __builtin_inf())) {
        ctl->status = CH_ENONFINITE;
        ctl->halted = 1;
        return;
    }
    const bool constant = ctl->mode != MODE_EE;
    const double tau_used = constant ? ctl->tau_step : ctl->tau_acc;
    // the final-time clip lands exactly on T when the clipped step was taken in full
    const double t_new = (ctl->clipped && ctl->converged) ? ctl->T : ctl->t + tau_used;
    double tau_next;
    if (constant) {
        tau_next = ctl->tau_fixed;
    } else {
        const double grow = 1.25 * tau_used;   // eq. EEdt
        tau_next = est == 0.0 ? grow : fmin(grow, sqrt(ctl->tol / est) * tau_used);
    }
    const int mv = ctl->mv_step + 1 + ctl->j;
    ctl->last_j = ctl->j;
    if (ctl->rec && ctl->steps < ctl->rec_cap) {
        ch_step_record& r = ctl->rec[ctl->steps];
        r.t = t_new;
        r.tau = tau_used;
        r.tau_next = tau_next;
        r.est = est;
        r.tol_phi = ctl->tol_phi;
        r.beta = ctl->beta;
        r.resnorm = ctl->resnorm;
        r.lambda_max = 0.0;
        r.j = ctl->j;
        r.cycles = ctl->cycles;
        r.traced = ctl->traced;
        r.matvecs = mv;
    }
    ctl->est = est;
    ctl->t = t_new;
    ctl->tau = tau_next;
    ctl->beta = beta;
    ctl->gnorm = gn;
    ctl->matvecs += mv;
    ctl->traces += ctl->traced;
    ctl->steps += 1;
    ctl->cur ^= 1;
    if (!(t_new < ctl->T) || (ctl->max_steps > 0 && ctl->steps >= ctl->max_steps)) {
        ctl->halted = 1;
        return;
    }
    if (begin_next) begin_step(ctl);
}

// ---------------------------------------------------------------------------
// LIM step begin (Fig. 1, steps 1-2; Fig. 2, lines 3-5): partials of
// min/max y^2 (and a non-finite flag) ...
// ---------------------------------------------------------------------------
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_lim_begin(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                        const int* __restrict__ cb2i, const Inst inst0, int ninst, const double* __restrict__ ybase,
                                                        double* __restrict__ pout) {
    const Inst I = SINGLE ? inst0 : insts[cb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    const double* y = ybase + I.off;
    double mn = __builtin_inf(), mx = -__builtin_inf(), bad = 0.0;
    const long long stride = (long long)I.cblk * CH_BLOCK;
    for (long long q = (long long)(blockIdx.x - I.cblk0) * CH_BLOCK + threadIdx.x; q < I.N; q += stride) {
        const double v = y[q] * y[q];
        if (v < __builtin_inf()) {
            mn = fmin(mn, v);
            mx = fmax(mx, v);
        } else {
            bad = 1.0;
        }
    }
    double x[3] = {-mn, mx, bad};
    write_partials<3, RED_MAX>(x, pout);
}

// ... then the final-time clip, lambda_max = ||Ahat_n||_1 and p (eq. p).
// Column j of Ahat_n is d_j A e_j + eps^2 A^2 e_j; its absolute sum g(d_j) is
// convex and piecewise linear in d_j, so the largest column sum is
// max(g(d_min), g(d_max)):
//   2-D: g(d) = |4d/h^2 + 20e| + 4|d/h^2 + 8e| + 12e,      e = eps^2/h^4
//   3-D: g(d) = |6d/h^2 + 42e| + 6|d/h^2 + 12e| + 30e
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_lim_plan(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst,
                                                       const double* __restrict__ pin, int pin_stencil, int dim) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    double tot[3];
    sum_inst_partials<3, RED_MAX>(pin, I, pin_stencil, tot);
    if (threadIdx.x != 0) return;
    const double ymin2 = -tot[0], ymax2 = tot[1];
    if (tot[2] != 0.0) {
        ctl->status = CH_ENONFINITE;
        ctl->halted = 1;
        return;
    }
    if (!(ctl->t < ctl->T) || (ctl->max_steps > 0 && ctl->steps >= ctl->max_steps)) {
        ctl->halted = 1;
        return;
    }
    double tau = ctl->tau;
    int clipped = 0;
    if (ctl->t + tau > ctl->T) {
        tau = ctl->T - ctl->t;
        clipped = 1;
    }
    const double inv_h2 = I.inv_h2;
    const double e = I.eps2 * inv_h2 * inv_h2;
    const double dmin = 3.0 * ymin2 - 1.0 + I.eyre, dmax = 3.0 * ymax2 - 1.0 + I.eyre;
    double gmin, gmax;
    if (dim == 2) {
        gmin = fabs(4.0 * dmin * inv_h2 + 20.0 * e) + 4.0 * fabs(dmin * inv_h2 + 8.0 * e) + 12.0 * e;
        gmax = fabs(4.0 * dmax * inv_h2 + 20.0 * e) + 4.0 * fabs(dmax * inv_h2 + 8.0 * e) + 12.0 * e;
    } else {
        gmin = fabs(6.0 * dmin * inv_h2 + 42.0 * e) + 6.0 * fabs(dmin * inv_h2 + 12.0 * e) + 30.0 * e;
        gmax = fabs(6.0 * dmax * inv_h2 + 42.0 * e) + 6.0 * fabs(dmax * inv_h2 + 12.0 * e) + 30.0 * e;
    }
    const double lam = fmax(gmin, gmax);
    const double pi = 3.141592653589793;
    const double pr = ceil((pi / 4.0) / (pi / 2.0 - atan(sqrt(tau * lam))));
    if (!(pr <= double(CH_PMAX))) {
        ctl->status = CH_EINVAL;
        ctl->halted = 1;
        return;
    }
    ctl->clipped = clipped;
    ctl->tau0 = tau;
    ctl->lam = lam;
    ctl->p = (int)pr;
}

// LIM step end (Fig. 2, lines 8-10): est (eq. LIMest), t, tau_new (eq. LIMdt).
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_lim_end(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst,
                                                      const double* __restrict__ pin, int pin_stencil) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    double tot[2];
    sum_inst_partials<2, RED_SUM>(pin, I, pin_stencil, tot);
    if (threadIdx.x != 0) return;
    const double num = sqrt(tot[0]), den = sqrt(tot[1]);
    const double est = den > 0.0 ? num / den : 0.0;
    if (!(est < __builtin_inf())) {
        ctl->status = CH_ENONFINITE;
        ctl->halted = 1;
        return;
    }
    const double tau = ctl->tau0;
    const double t_new = ctl->clipped ? ctl->T : ctl->t + tau;
    double tau_next = tau;
    if (ctl->mode == MODE_LIM) tau_next = est == 0.0 ? tau : ctl->tol / est * tau;   // eq. LIMdt
    if (ctl->mode == MODE_LIM_CONST) tau_next = ctl->tau_fixed;
    const int mv = 2 * ctl->p - 1;
    if (ctl->rec && ctl->steps < ctl->rec_cap) {
        ch_step_record& r = ctl->rec[ctl->steps];
        r.t = t_new;
        r.tau = tau;
        r.tau_next = tau_next;
        r.est = est;
        r.tol_phi = 0.0;
        r.beta = 0.0;
        r.resnorm = 0.0;
        r.lambda_max = ctl->lam;
        r.j = ctl->p;
        r.cycles = 0;
        r.traced = 0;
        r.matvecs = mv;
    }
    ctl->est = est;
    ctl->t = t_new;
    ctl->tau = tau_next;
    ctl->matvecs += mv;
    ctl->steps += 1;
    ctl->cur ^= 1;
    if (!(t_new < ctl->T) || (ctl->max_steps > 0 && ctl->steps >= ctl->max_steps)) ctl->halted = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define CARGS dim3(t.cgrid), dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.cb2i, t.hinst[0], t.ninst
#define IARGS dim3(t.ninst), dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.hinst[0], t.ninst

hipError_t launch_mgs_pass(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, int k, int i, hipStream_t s) {
    const bool fin = i > k;
    if (prec == CH_FP64) {
        double* V = static_cast<double*>(b.V);
        if (fin)
            if (t.ninst == 1)
                hipLaunchKernelGGL((k_mgs<double, true, true>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
            else
                hipLaunchKernelGGL((k_mgs<double, true, false>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
        else
            if (t.ninst == 1)
                hipLaunchKernelGGL((k_mgs<double, false, true>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
            else
                hipLaunchKernelGGL((k_mgs<double, false, false>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
    } else {
        float* V = static_cast<float*>(b.V);
        if (fin)
            if (t.ninst == 1)
                hipLaunchKernelGGL((k_mgs<float, true, true>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
            else
                hipLaunchKernelGGL((k_mgs<float, true, false>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
        else
            if (t.ninst == 1)
                hipLaunchKernelGGL((k_mgs<float, false, true>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
            else
                hipLaunchKernelGGL((k_mgs<float, false, false>), CARGS, V, b.ldv, k, i, ps.in(), ps.stencil, ps.out());
    }
    ps.produced(false);
    return hipGetLastError();
}

hipError_t launch_phi(const Table& t, const DevBuffers& b, PartSeq& ps, int k, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_phi<true>), IARGS, k, ps.in(), ps.stencil, b.dflag);
    else
        hipLaunchKernelGGL((k_phi<false>), IARGS, k, ps.in(), ps.stencil, b.dflag);
    return hipGetLastError();
}

bool all_cycles_done(const Table& t, const DevBuffers& b, const int* expected) {
    if (!b.hflag || !expected) return false;
    for (int i = 0; i < t.ninst; ++i) {
        const int slot = t.hinst[i].slot;
        if (b.hflag[slot] != expected[slot]) return false;
    }
    return true;
}

hipError_t launch_arnoldi_iter(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int k,
                               hipStream_t s) {
    hipError_t e = launch_matvec(t, prec, b, ps, y, k, s);
    if (e != hipSuccess) return e;
    for (int i = 1; i <= k + 1; ++i)
        if ((e = launch_mgs_pass(t, prec, b, ps, k, i, s)) != hipSuccess) return e;
    return launch_phi(t, b, ps, k, s);
}

hipError_t launch_arnoldi(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int m_max,
                          const int* expected, hipStream_t s) {
    for (int k = 0; k < m_max; ++k) {
        if (k > 0 && all_cycles_done(t, b, expected)) break;
        hipError_t e = launch_arnoldi_iter(t, prec, b, ps, y, k, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_update(const Table& t, int prec, const DevBuffers& b, const double* y, double* ynew, hipStream_t s) {
    if (prec == CH_FP64)
        if (t.ninst == 1)
            hipLaunchKernelGGL((k_update<double, true>), CARGS, y, static_cast<const double*>(b.V), b.ldv, ynew);
        else
            hipLaunchKernelGGL((k_update<double, false>), CARGS, y, static_cast<const double*>(b.V), b.ldv, ynew);
    else
        if (t.ninst == 1)
            hipLaunchKernelGGL((k_update<float, true>), CARGS, y, static_cast<const float*>(b.V), b.ldv, ynew);
        else
            hipLaunchKernelGGL((k_update<float, false>), CARGS, y, static_cast<const float*>(b.V), b.ldv, ynew);
    return hipGetLastError();
}

hipError_t launch_after_resid(const Table& t, const DevBuffers& b, PartSeq& ps, bool begin_step, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_after_resid<true>), IARGS, ps.in(), ps.stencil, begin_step ? 1 : 0);
    else
        hipLaunchKernelGGL((k_after_resid<false>), IARGS, ps.in(), ps.stencil, begin_step ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_cycle_begin(const Table& t, const DevBuffers& b, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_cycle_begin<true>), dim3(t.ninst), dim3(64), 0, s, b.ctl, t.inst, t.hinst[0], t.ninst);
    else
        hipLaunchKernelGGL((k_cycle_begin<false>), dim3(t.ninst), dim3(64), 0, s, b.ctl, t.inst, t.hinst[0], t.ninst);
    return hipGetLastError();
}

hipError_t launch_step_end(const Table& t, const DevBuffers& b, PartSeq& ps, bool begin_next, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_step_end<true>), IARGS, ps.in(), ps.stencil, begin_next ? 1 : 0);
    else
        hipLaunchKernelGGL((k_step_end<false>), IARGS, ps.in(), ps.stencil, begin_next ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_lim_begin(const Table& t, const DevBuffers& b, PartSeq& ps, const double* y, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_lim_begin<true>), CARGS, y, ps.out());
    else
        hipLaunchKernelGGL((k_lim_begin<false>), CARGS, y, ps.out());
    ps.produced(false);
    return hipGetLastError();
}

hipError_t launch_lim_plan(const Table& t, const DevBuffers& b, PartSeq& ps, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_lim_plan<true>), IARGS, ps.in(), ps.stencil, t.dim);
    else
        hipLaunchKernelGGL((k_lim_plan<false>), IARGS, ps.in(), ps.stencil, t.dim);
    return hipGetLastError();
}

hipError_t launch_lim_end(const Table& t, const DevBuffers& b, PartSeq& ps, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_lim_end<true>), IARGS, ps.in(), ps.stencil);
    else
        hipLaunchKernelGGL((k_lim_end<false>), IARGS, ps.in(), ps.stencil);
    return hipGetLastError();
}
