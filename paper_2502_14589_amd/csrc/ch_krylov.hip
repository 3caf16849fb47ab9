// Arnoldi (delayed classical Gram-Schmidt twice, or modified Gram-Schmidt), the
// small-matrix phi with the residual-time restart, the solution update and
// the per-step controllers.
//
// Krylov algorithm of Fig. 3 (Section 4.1): for j = 1..m_max,
//   w = Ahat v_j;  h_ij = w^T v_i, w -= h_ij v_i (i = 1..j);  h_{j+1,j} = ||w||;
//   u = tau0 phi(-tau0 H_jj) e_1;  resnorm = h_{j+1,j} |e_j^T u|  (eq. rm);
//   converged if resnorm <= tol_phi, else at j = m_max shrink tau to the
//   largest step whose residual passes (eq. phi_stop);
// then y^{n+1} = y^n + V_j (beta u).
//
// Storage: column i of the basis is kept unnormalised, v_i = vscale[i] V(:,i),
// so the normalisation of each new basis vector is folded into the next reads.  One launch
// covers every instance of a batch; streaming kernels give each instance the
// workgroups [cblk0, cblk0 + cblk) (map cb2i), single-workgroup kernels one
// workgroup per instance.
#include "ch_common.h"
#include "ch_stream.h"

#include <algorithm>
#include <cstdint>

#include <chrono>

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
// DCGS2 for Arnoldi iteration j.  Column j holds u_j, the (j+1)-th vector
// after one classical projection on q_0..q_{j-1} (columns 0..j-1, stored
// normalised), not yet reorthogonalised nor normalised (u_0 is the start
// vector, scaled by vscale[0] = 1 / beta).
//   the matvec launch:    w = Ahat u_j into column j + 1; partials of
//                         sigma_i = <q_i, u_j>, tau_i = <q_i, w> (i < j),
//                         alpha = <u_j, u_j>, beta' = <u_j, w>
//   k_dots_reduce:        their totals
//   k_dc_update:          s = sigma, rho^2 = alpha - |s|^2 (Pythagoras: s is the
//                         reorthogonalisation of a vector already projected
//                         once, so no cancellation); h_{:,j-1} = h'_{:,j-1} + s
//                         and h_{j,j-1} = rho make column j - 1 of the
//                         Hessenberg matrix final.  From the Arnoldi relation
//                         A Q_{j-1} = Q_j H_j, A q_j = (w - Q_j H_j s) / rho, so
//                         the first projection of A q_j on Q_j follows from the
//                         same totals: with g = H_j s and t = tau,
//                           h'_i = (t_i - g_i) / rho                 (i < j),
//                           h'_j = ((beta' - s.t) / rho - g_j) / rho;
//                         then, in one pass over the basis,
//                           q_j = (u_j - Q_{j-1} s) / rho           -> column j,
//                           u_{j+1} = w / rho - Q_j (g / rho + h')  -> column j + 1.
//   the phi test:         dimension j on the final columns 0..j-1 (it reads
//                         only H): up to dimension 31 in extra workgroups of
//                         the update launch (k_dc_update_phi), which form
//                         column j - 1 themselves; beyond that in a launch of
//                         its own on a second stream, overlapping the next
//                         iteration.
// Every workgroup of the update forms the coefficients itself (same
// arithmetic, same order: identical in all of them); the first workgroup of
// an instance publishes column j - 1 and h'.  h' alternates between two
// buffers, so the publishing workgroup never overwrites what another still
// reads.  At j = m_max only column j - 1 is formed (FIN, one workgroup).
// ---------------------------------------------------------------------------
#ifndef CH_DCU_Q
#define CH_DCU_Q 2
#endif

struct DcCoef {
    double s[CH_MMAX + 1], t[CH_MMAX + 1], g[CH_MMAX + 1], hf[CH_MMAX + 1];
    double ca[CH_MMAX + 1], cb[CH_MMAX + 1];
    // H_j staged column by column, leading dimension j + 1 (j <= CH_MSMALL;
    // larger j read the control block directly)
    double hs[CH_MSMALL * (CH_MSMALL + 1)];
    double rho, st, cbw, cq;
};

// Coefficients of iteration j into LDS; `publish`: this workgroup writes
// column j - 1 of H and h' of column j.  Contains barriers: call from every
// thread of the workgroup.  Sums over i < j (j < 64) are wave-0 butterflies,
// the same in every workgroup.
__device__ void dc_prepare(DcCoef& C, Ctl* ctl, int j, bool fin, bool publish) {
    const double* dt = ctl->dt;
    const double* hprev = ctl->h1[j & 1];   // h' of column j - 1
    for (int i = threadIdx.x; i < j; i += CH_BLOCK) {
        C.s[i] = dt[i];
        C.t[i] = dt[j + i];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int i = threadIdx.x;
        const double si = i < j ? C.s[i] : 0.0, ti = i < j ? C.t[i] : 0.0;
        const double ss = wave_sum(si * si), st = wave_sum(si * ti);
        if (i == 0) {
            const double rho2 = dt[2 * j] - ss;
            C.rho = rho2 > 0.0 ? sqrt(rho2) : (rho2 <= 0.0 ? 0.0 : rho2);   // NaN stays NaN
            C.st = st;
        }
    }
    __syncthreads();
    const double rho = C.rho;
    for (int i = threadIdx.x; i <= j; i += CH_BLOCK) {
        const double h = i < j ? hprev[i] + C.s[i] : rho;
        C.hf[i] = h;
        if (publish && j >= 1) ctl->H[i + (j - 1) * CH_LDH] = h;
    }
    if (fin) return;
    __syncthreads();
    // H_j ((j + 1) x j, Hessenberg): columns 0..j-2 are final in ctl->H, column j - 1 is C.hf
    const int ld = j + 1;
    if (j <= CH_MSMALL) {
        for (int idx = threadIdx.x; idx < ld * j; idx += CH_BLOCK) {
            const int c = idx / ld, r = idx - c * ld;
            C.hs[idx] = r > c + 1 ? 0.0 : (c == j - 1 ? C.hf[r] : ctl->H[r + c * CH_LDH]);
        }
        __syncthreads();
        for (int r = threadIdx.x; r <= j; r += CH_BLOCK) {   // g = H_j s
            double g = 0.0;
            for (int c = r > 0 ? r - 1 : 0; c < j; ++c) g += C.hs[r + c * ld] * C.s[c];
            C.g[r] = g;
        }
    } else {
        for (int r = threadIdx.x; r <= j; r += CH_BLOCK) {   // g = H_j s, same order of terms
            double g = 0.0;
            for (int c = r > 0 ? r - 1 : 0; c < j; ++c) g += (c == j - 1 ? C.hf[r] : ctl->H[r + c * CH_LDH]) * C.s[c];
            C.g[r] = g;
        }
    }
    __syncthreads();
    const double ir = 1.0 / rho;
    const double qw = (dt[2 * j + 1] - C.st) * ir;   // q_j^T w
    double* hnew = ctl->h1[(j + 1) & 1];
    for (int i = threadIdx.x; i <= j; i += CH_BLOCK) {
        const double hp = ((i < j ? C.t[i] : qw) - C.g[i]) * ir;   // h'_i
        const double c = C.g[i] * ir + hp;
        if (publish) hnew[i] = hp;
        if (i < j) {
            C.ca[i] = -C.s[i] * ir;
            C.cb[i] = -c;
        } else {
            C.ca[j] = (j == 0 ? ctl->vscale[0] : 1.0) * ir;
            C.cq = -c;
        }
    }
    if (threadIdx.x == 0) C.cbw = ir;
    __syncthreads();
}

// 16-byte raw buffer accesses over one span of a column: reads past the
// span's end return zeros and stores there are dropped, so the pass below has
// no branch around a memory access (a branch would make the compiler wait for
// every outstanding load where it joins, prefetches included).
using u32x4v = unsigned __attribute__((ext_vector_type(4)));
constexpr unsigned DCU_OFF = 0x80000000u;   // an offset past any span

__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// AUX: the cache-policy bits of the load (2: non-temporal).
template <typename VT, int AUX = 0>
__device__ __forceinline__ VT load16(__amdgpu_buffer_rsrc_t r, unsigned bo) {
    return __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(r, bo, 0u, AUX));
}

template <typename VT>
__device__ __forceinline__ void store16(VT v, __amdgpu_buffer_rsrc_t r, unsigned bo) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4v, v), r, bo, 0u, 0);
}

// The update pass of one workgroup; bid: its index among the launch's
// streaming workgroups.  The instance's vectors (16 bytes) are taken in spans
// of cblk * CH_BLOCK * Q; thread t of the workgroups handles vectors t,
// t + cblk * CH_BLOCK, ... of each span.  Basis columns come in blocks of two
// through two buffers that alternate, so the loads of one block are in
// flight while the other is summed and no loaded value is copied.  NT: the
// basis columns are loaded with the streaming hint (stream_columns).
template <typename TV, bool SINGLE, int TAG, bool NT>
__device__ __forceinline__ void dc_update_wg(DcCoef& C, Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                             const int* __restrict__ cb2i, const Inst& inst0, int bid,
                                             TV* __restrict__ V, size_t ldv, int j) {
    const Inst I = SINGLE ? inst0 : insts[cb2i[bid]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    using VT = typename Vec16<TV>::type;
    constexpr int VW = Vec16<TV>::W, Q = CH_DCU_Q, RB = 2;
    const TV* Vi = V + I.off;
    TV* U = V + (size_t)j * ldv + I.off;
    TV* Wc = V + (size_t)(j + 1) * ldv + I.off;
    const long long NV = I.N / VW;
    const long long per = (long long)I.cblk * CH_BLOCK;
    const long long span = per * Q;   // vectors per span: at most 2^18 (4 MiB)
    const int lt = (bid - I.cblk0) * CH_BLOCK + threadIdx.x;
    unsigned rel[Q];   // byte offsets of this thread's vectors in a span
#pragma unroll
    for (int u = 0; u < Q; ++u) rel[u] = (unsigned)(lt + u * per) * 16u;
    auto vrs = [&](const TV* col, long long v0) {
        const long long left = NV - v0;
        const long long nv = left < span ? (left > 0 ? left : 0) : span;
        return span_rsrc(col + v0 * VW, (unsigned)nv * 16u);
    };
    VT uv[Q], wv[Q];
    auto load_uw = [&](long long v0) {
        const __amdgpu_buffer_rsrc_t ru = vrs(U, v0), rw = vrs(Wc, v0);
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            uv[u] = load16<VT>(ru, rel[u]);
            wv[u] = load16<VT>(rw, rel[u]);
        }
    };
    auto load_blk = [&](long long v0, int i0, VT (&b)[RB][Q]) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = i0 + r;
            const bool live = i < j;
            const __amdgpu_buffer_rsrc_t rc = vrs(Vi + (size_t)(live ? i : 0) * ldv, v0);
#pragma unroll
            for (int u = 0; u < Q; ++u) b[r][u] = load16<VT, NT ? 2 : 0>(rc, live ? rel[u] : DCU_OFF);
        }
    };
    // the first vectors and basis columns are requested before the
    // coefficients are formed, so the loads overlap that latency
    VT ba[RB][Q], bb[RB][Q];
    load_uw(0);
    load_blk(0, 0, ba);
    dc_prepare(C, ctl, j, false, TAG == 0 && bid == I.cblk0);   // timing launches publish nothing
    const double* ca = C.ca;
    const double* cb = C.cb;
    const double cbw = C.cbw, cq = C.cq;
    double xq[Q][VW], xu[Q][VW];
    auto acc = [&](const VT (&b)[RB][Q], int i0) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const bool live = i0 + r < j;
            const int i = live ? i0 + r : 0;
            const double a = live ? ca[i] : 0.0;
            const double c = live ? cb[i] : 0.0;
#pragma unroll
            for (int u = 0; u < Q; ++u) {
                const TV* ve = reinterpret_cast<const TV*>(&b[r][u]);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    xq[u][e] += a * double(ve[e]);
                    xu[u][e] += c * double(ve[e]);
                }
            }
        }
    };
    for (long long v0 = 0; v0 < NV; v0 += span) {
        if (v0 != 0) {
            load_uw(v0);
            load_blk(v0, 0, ba);
        }
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const TV* ue = reinterpret_cast<const TV*>(&uv[u]);
            const TV* we = reinterpret_cast<const TV*>(&wv[u]);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                xq[u][e] = ca[j] * double(ue[e]);
                xu[u][e] = cbw * double(we[e]);
            }
        }
        for (int i0 = 0; i0 < j; i0 += 2 * RB) {
            load_blk(v0, i0 + RB, bb);
            acc(ba, i0);
            load_blk(v0, i0 + 2 * RB, ba);
            acc(bb, i0 + RB);
        }
        const __amdgpu_buffer_rsrc_t ru = vrs(U, v0), rw = vrs(Wc, v0);
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            VT qv, nv;
            TV* qe = reinterpret_cast<TV*>(&qv);
            TV* ne = reinterpret_cast<TV*>(&nv);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                qe[e] = TV(xq[u][e]);
                ne[e] = TV(xu[u][e] + cq * double(qe[e]));   // with q_j as stored
            }
            store16<VT>(qv, ru, rel[u]);
            store16<VT>(nv, rw, rel[u]);
        }
    }
    // elements past the last whole vector
    for (long long e = NV * VW + lt; e < I.N; e += per) {
        double sq = ca[j] * double(U[e]), su = cbw * double(Wc[e]);
        for (int i = 0; i < j; ++i) {
            const double v = double(Vi[(size_t)i * ldv + e]);
            sq += ca[i] * v;
            su += cb[i] * v;
        }
        const TV qs = TV(sq);
        U[e] = qs;
        Wc[e] = TV(su + cq * double(qs));
    }
}

// Progress report of an update launch: workgroup 0 counts the launch on a
// device counter as the launch begins (whatever the state of its instances)
// and writes the count to a pinned host word, so the host, which counts the
// update launches it issues, can keep the number of iterations it has issued
// ahead of the device small.  The count lives on the device so that launches
// replayed from a graph number themselves.
__device__ __forceinline__ void report_launch(int* dprog, int* dcount) {
    if (dprog && blockIdx.x == 0 && threadIdx.x == 0)
        *dprog = __hip_atomic_fetch_add(dcount, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
}

template <typename TV, bool SINGLE, int TAG, bool NT>   // TAG: as for the matvec
__global__ __launch_bounds__(CH_BLOCK) void k_dc_update(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                        const int* __restrict__ cb2i, const Inst inst0, int ninst,
                                                        TV* __restrict__ V, size_t ldv, int j,
                                                        int* __restrict__ dprog, int* __restrict__ dcount) {
    report_launch(dprog, dcount);
    __shared__ DcCoef C;
    dc_update_wg<TV, SINGLE, TAG, NT>(C, ctls, insts, cb2i, inst0, blockIdx.x, V, ldv, j);
}

// Iteration j = m_max: column j - 1 of H only (one workgroup per instance).
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_dc_finish(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                        const Inst inst0, int ninst, int j) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    __shared__ DcCoef C;
    dc_prepare(C, ctl, j, true, true);
}

// One workgroup per (row i, instance): the total of the partials of row i of
// a DCGS2 matvec launch.
template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_dots_reduce(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                          const Inst inst0, int ninst,
                                                          const double* __restrict__ dots, int kind) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.y];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    const int r = blockIdx.x;
    double tot[1];
    sum_inst_partials<1, RED_SUM>(dots + (size_t)r * CH_MAXB, I, kind, tot);
    if (threadIdx.x == 0) ctl->dt[r] = tot[0];
}

// ---------------------------------------------------------------------------
// y^{n+1} = y^n + V_j (beta u)  (the solution update of Fig. 3)
// ---------------------------------------------------------------------------
template <typename TV, bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_update(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                     const int* __restrict__ cb2i, const Inst inst0, int ninst, const double* ybase,
                                                     const TV* __restrict__ V, size_t ldv, double* ynewbase,
                                                     int unit) {
    // ybase may alias ynewbase (restart cycles update the sub-step state in place);
    // unit: the basis is stored normalised (DCGS2), vscale is not used
    const Inst I = SINGLE ? inst0 : insts[cb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    __shared__ double cf[CH_MMAX];
    const int j = ctl->j;
    if ((int)threadIdx.x < j)
        cf[threadIdx.x] = ctl->beta * ctl->u[threadIdx.x] * (unit ? 1.0 : ctl->vscale[threadIdx.x]);
    const double* y = ybase + I.off;
    double* ynew = ynewbase + I.off;
    const TV* Vi = V + I.off;
    // 16-byte vectors of the basis (VW values), Q per thread, columns in
    // blocks of RB requested one block ahead; the state in FP64
    using VT = typename Vec16<TV>::type;
    constexpr int VW = Vec16<TV>::W, Q = 2, RB = 4;
    const long long NV = I.N / VW;
    const long long per = (long long)I.cblk * CH_BLOCK;
    const long long lt = (long long)(blockIdx.x - I.cblk0) * CH_BLOCK + threadIdx.x;
    __syncthreads();
    for (long long q0 = lt; q0 < NV; q0 += per * Q) {
        long long qq[Q];
        bool ok[Q];
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            qq[u] = q0 + u * per;
            ok[u] = qq[u] < NV;
        }
        auto load_cols = [&](int i0, VT (&v)[RB][Q]) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int u = 0; u < Q; ++u) {
                    if (ok[u] && i0 + r < j) {
                        v[r][u] = reinterpret_cast<const VT*>(Vi + (size_t)(i0 + r) * ldv)[qq[u]];
                    } else {
                        TV* ve = reinterpret_cast<TV*>(&v[r][u]);
#pragma unroll
                        for (int e = 0; e < VW; ++e) ve[e] = TV(0);
                    }
                }
        };
        double yv[Q][VW], acc[Q][VW];
#pragma unroll
        for (int u = 0; u < Q; ++u)
#pragma unroll
            for (int e = 0; e < VW; e += 2) {
                const double2 t2 = ok[u] ? reinterpret_cast<const double2*>(y)[(qq[u] * VW + e) / 2] : double2{0.0, 0.0};
                yv[u][e] = t2.x;
                yv[u][e + 1] = t2.y;
                acc[u][e] = acc[u][e + 1] = 0.0;
            }
        VT cur[RB][Q];
        load_cols(0, cur);
        for (int i0 = 0; i0 < j; i0 += RB) {
            VT nxt[RB][Q];
            load_cols(i0 + RB, nxt);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const double c = i0 + r < j ? cf[i0 + r] : 0.0;
#pragma unroll
                for (int u = 0; u < Q; ++u) {
                    const TV* ve = reinterpret_cast<const TV*>(&cur[r][u]);
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc[u][e] += c * double(ve[e]);
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int u = 0; u < Q; ++u) cur[r][u] = nxt[r][u];
        }
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int e = 0; e < VW; e += 2)
                reinterpret_cast<double2*>(ynew)[(qq[u] * VW + e) / 2] =
                    double2{yv[u][e] + acc[u][e], yv[u][e + 1] + acc[u][e + 1]};
        }
    }
    for (long long q = NV * VW + lt; q < I.N; q += per) {   // the last N mod VW points
        double a = 0.0;
        for (int i = 0; i < j; ++i) a += cf[i] * double(Vi[(size_t)i * ldv + q]);
        ynew[q] = y[q] + a;
    }
}

// ---------------------------------------------------------------------------
// Small-matrix exponential.  exp([[X, b], [0, 0]]) = [[e^X, phi(X) b], [0, 1]]
// (phi of eq. phi), so with X = -s H_jj and b = s e_1 the last column holds
// u = s phi(-s H_jj) e_1 and the first column exp(-s H_jj) e_1 = du/ds.
//
// Scaling and squaring with the degree-19 Taylor polynomial T_19: the
// argument is scaled by 2^-q so that its 1-norm is at most theta_19 =
// 1.2603811, the largest theta for which the relative backward error of T_19
// is at most 2^-53 (the power series of log(e^-x T_19(x)) has coefficients
// c_k, k >= 20, with sum_k |c_k| theta^(k-1) <= 2^-53; the backward-error
// analysis of Al-Mohy and Higham, SIAM J. Matrix Anal. Appl. 31 (2009)
// 970-989, applied to a Taylor instead of a Pade approximant).  T_19 is a
// polynomial, so the evaluation is matrix products only -- no linear solve --
// and all of them run on the FP64 matrix cores:
//   X^2, X^3, X^4, X^5;  T_19 = B_0 + X^5 (B_1 + X^5 (B_2 + X^5 B_3)),
//   B_i = sum_{q=0..4} X^q / (5i + q)!     (7 products),
// then q squarings.  Everything stays in LDS, in FP64.
// ---------------------------------------------------------------------------
// Orders are padded to a multiple of 16 for the matrix cores; the padding is
// a zero block of the argument, whose exponential is an identity block.
constexpr int NPMAX = 48;          // largest padded order in LDS
constexpr int NPBIG = 112;         // largest padded order (device scratch)
static_assert(CH_MSMALL + 1 <= NPMAX, "augmented matrix exceeds the padded LDS order");
static_assert(CH_MMAX + 1 <= NPBIG, "augmented matrix exceeds the padded order");
constexpr double THETA19 = 1.2603811;
constexpr int NLVL = 80;

// LDS of one phi evaluation for padded orders up to NPM; rows of stride
// LD = NPM + 1 (odd: rows fall in different banks).
template <int NPM>
struct PhiShared {
    static constexpr int LD = NPM + 1;
    double B[6][NPM * LD];      // X, X^2, X^3, X^4, two Horner / squaring buffers
    double c[20];               // 1 / k!
    double lvl[NLVL];           // lvl[kk] = resnorm at s 2^-kk from the squaring chain
    double red;
    int nsq;                    // squarings of the last evaluation (order-16 path)
    double hcol[NPM];           // column j - 1 of H when it is not yet in the control block
};

typedef double dbl4 __attribute__((ext_vector_type(4)));

// C = A B (+ epi(r, c) elementwise) for padded order np (a multiple of 16) on
// the FP64 matrix cores: 16x16 output tiles spread over the waves, K in steps
// of 4.  Lanes of the 16x16x4 instruction: lane l supplies A(l % 16, l / 16)
// and B(l / 16, l % 16) of its 16x4 and 4x16 slices and receives
// C(4 v + l / 16, l % 16) in element v.
struct NoEpi {
    __device__ double operator()(int, int) const { return 0.0; }
};

// NT = np / 16 tiles per direction.  The K loop is unrolled: every A and B
// operand of a tile is read from LDS before the first product, and even and
// odd K steps accumulate separately (two independent chains).
template <int NT, int PLD, typename Epi = NoEpi>
__device__ void mm_t(double* __restrict__ C, const double* __restrict__ A, const double* __restrict__ B,
                     Epi epi = Epi()) {
    constexpr int NP = 16 * NT, KS = NP / 4;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 1
    for (int t = wid; t < NT * NT; t += CH_BLOCK / 64) {
        const int ti = t / NT, tj = t - ti * NT;
        const double* a = A + (16 * ti + li) * PLD + lk;
        const double* b = B + lk * PLD + 16 * tj + li;
        double av[KS], bv[KS];
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            av[q] = a[4 * q];
            bv[q] = b[4 * q * PLD];
        }
        dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < KS; q += 2) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc0, 0, 0, 0);
            if (q + 1 < KS) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q + 1], bv[q + 1], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * ti + 4 * v + lk, c = 16 * tj + li;
            C[r * PLD + c] = (acc0[v] + acc1[v]) + epi(r, c);
        }
    }
    __syncthreads();
}

template <int NPM, typename Epi = NoEpi>
__device__ void mm(double* __restrict__ C, const double* __restrict__ A, const double* __restrict__ B, int np,
                   Epi epi = Epi()) {
    constexpr int PLD = NPM + 1;
    if (np <= 16) mm_t<1, PLD>(C, A, B, epi);
    else if (NPM >= 32 && np <= 32) mm_t<(NPM >= 32 ? 2 : 1), PLD>(C, A, B, epi);
    else if (NPM >= 48 && np <= 48) mm_t<(NPM >= 48 ? 3 : 1), PLD>(C, A, B, epi);
    else if (NPM >= 64 && np <= 64) mm_t<(NPM >= 64 ? 4 : 1), PLD>(C, A, B, epi);
    else if (NPM >= 80 && np <= 80) mm_t<(NPM >= 80 ? 5 : 1), PLD>(C, A, B, epi);
    else if (NPM >= 96 && np <= 96) mm_t<(NPM >= 96 ? 6 : 1), PLD>(C, A, B, epi);
    else if (NPM >= 112) mm_t<(NPM >= 112 ? 7 : 1), PLD>(C, A, B, epi);
}

// B_i(r, c) = sum_{q=0..3} X^q(r, c) / (4i + q)!
template <int PLD>
struct TaylorBlock {
    const double* X[4];   // X^1 .. X^3 in X[1..3]
    const double* cf;
    int i;
    __device__ double operator()(int r, int c) const {
        const int o = r * PLD + c;
        const double* f = cf + 4 * i;
        return (r == c ? f[0] : 0.0) + f[1] * X[1][o] + f[2] * X[2][o] + f[3] * X[3][o];
    }
};

// ---------------------------------------------------------------------------
// Padded order 16: the whole exponential in the registers of wave 0.  A
// 16 x 16 matrix M is held in the layout the matrix cores return it in
// ("C layout": lane l, element v holds M(4 v + l / 16, l % 16)), which is
// also the layout of a right operand's K slices; a left operand is wanted
// transposed ("A layout": lane l, element q holds M(l % 16, 4 q + l / 16)),
// made by a round trip through a block of LDS that only wave 0 touches (one
// wave's LDS accesses complete in order, so no barrier is needed).  Same
// products, epilogue and accumulation order as mm_t, without a workgroup
// barrier per product.
// ---------------------------------------------------------------------------
__device__ __forceinline__ dbl4 mm16(const dbl4& a, const dbl4& b) {
    dbl4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c1, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], c1, 0, 0, 0);
    return c0 + c1;
}

// C layout -> A layout through T (16 rows of stride 17)
__device__ __forceinline__ dbl4 to_a(const dbl4& c, double* T) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) T[(4 * v + lk) * 17 + li] = c[v];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    dbl4 a;
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = T[li * 17 + 4 * q + lk];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    return a;
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double elem(const dbl4& e, int v) {
    return v == 0 ? e[0] : (v == 1 ? e[1] : (v == 2 ? e[2] : e[3]));
}

// As expm_aug for n = j + 1 <= 16.  Call from every thread.
template <int NPM>
__device__ const double* expm16(PhiShared<NPM>& S, const double* __restrict__ H, const double* hlast, int j,
                                double s, double hnext, int* nsq_out) {
    constexpr int PLD = PhiShared<NPM>::LD;
    static_assert(16 * 17 <= NPM * PLD, "transpose block");
    double* E = S.B[4];
    __syncthreads();   // every wave's reads of the previous evaluation are done
    if (threadIdx.x < 64) {
        const int l = threadIdx.x, li = l & 15, lk = l >> 4;
        double* T = S.B[5];
        dbl4 x;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * v + lk, c = li;
            double val = 0.0;
            if (r < j && c < j) val = -s * (hlast && c == j - 1 ? hlast[r] : H[r + c * CH_LDH]);
            else if (r == 0 && c == j) val = s;
            x[v] = val;
        }
        // 1-norm: column sums (rows over v and the four lane groups), max over columns
        double cs = (fabs(x[0]) + fabs(x[1])) + (fabs(x[2]) + fabs(x[3]));
        cs += __shfl_xor(cs, 16, 64);
        cs += __shfl_xor(cs, 32, 64);
        const double nrm = wave_max(cs);
        int nsq = 0;
        if (nrm > THETA19 && nrm < __builtin_inf()) nsq = (int)ceil(log2(nrm / THETA19));
        if (nsq > 1100) nsq = 1100;
        const double scale = ldexp(1.0, -nsq);
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] *= scale;
        const dbl4 xa = to_a(x, T);
        const dbl4 x2 = mm16(xa, x);
        const dbl4 x2a = to_a(x2, T);
        const dbl4 x3 = mm16(x2a, x);
        const dbl4 x4a = to_a(mm16(x2a, x2), T);
        // T_19 = B_0 + X^4 (B_1 + X^4 (B_2 + X^4 (B_3 + X^4 B_4))),
        // B_i = sum_{q=0..3} X^q / (4i + q)!
        auto blk = [&](int i) {
            const double* f = S.c + 4 * i;
            dbl4 b;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                b[v] = ((4 * v + lk == li ? f[0] : 0.0) + f[1] * x[v] + f[2] * x2[v]) + f[3] * x3[v];
            return b;
        };
        dbl4 R = blk(4);
        for (int i = 3; i >= 0; --i) R = mm16(x4a, R) + blk(i);
        // resnorm at every dyadic level: element (j - 1, j)
        const int lr = j + 16 * ((j - 1) & 3), vr = (j - 1) >> 2;
        if (nsq < NLVL) {
            const double rv = hnext * fabs(readlane_d(elem(R, vr), lr));
            if (l == 0) S.lvl[nsq] = rv;
        }
        for (int i = 1; i <= nsq; ++i) {
            R = mm16(to_a(R, T), R);
            const int kk = nsq - i;
            if (kk < NLVL) {
                const double rv = hnext * fabs(readlane_d(elem(R, vr), lr));
                if (l == 0) S.lvl[kk] = rv;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) E[(4 * v + lk) * PLD + li] = R[v];
        if (l == 0) S.nsq = nsq;
    }
    __syncthreads();
    *nsq_out = S.nsq;
    return E;
}

// exp(s [[-H_jj, e_1], [0, 0]]); returns the LDS matrix holding it and the
// number of squarings in *nsq_out.  Records resnorm at every dyadic level of
// the squaring chain in S.lvl.  Column j - 1 of H comes from hlast when it is
// given (not yet in the control block), else from H.
template <int NPM>
__device__ const double* expm_aug(PhiShared<NPM>& S, const double* __restrict__ H, const double* hlast, int j,
                                  double s, double hnext, int* nsq_out) {
    constexpr int PLD = PhiShared<NPM>::LD;
    const int n = j + 1;
    if (n <= 16) return expm16<NPM>(S, H, hlast, j, s, hnext, nsq_out);
    const int np = (n + 15) & ~15;
    double* X1 = S.B[0];
    for (int idx = threadIdx.x; idx < np * np; idx += CH_BLOCK) {
        const int r = idx / np, c = idx - r * np;
        double v = 0.0;
        if (r < j && c < j) v = -s * (hlast && c == j - 1 ? hlast[r] : H[r + c * CH_LDH]);
        else if (r == 0 && c == j) v = s;
        X1[r * PLD + c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double cs = 0.0;
        if ((int)threadIdx.x < n)
            for (int r = 0; r < n; ++r) cs += fabs(X1[r * PLD + threadIdx.x]);
        cs = wave_max(cs);
        if (threadIdx.x == 0) S.red = cs;
    }
    __syncthreads();
    const double nrm = S.red;
    int nsq = 0;
    if (nrm > THETA19 && nrm < __builtin_inf()) nsq = (int)ceil(log2(nrm / THETA19));
    if (nsq > 1100) nsq = 1100;
    const double scale = ldexp(1.0, -nsq);
    for (int idx = threadIdx.x; idx < n * n; idx += CH_BLOCK) {
        const int r = idx / n, c = idx - r * n;
        X1[r * PLD + c] *= scale;
    }
    __syncthreads();
    mm<NPM>(S.B[1], X1, X1, np);         // X^2
    mm<NPM>(S.B[2], S.B[1], X1, np);     // X^3
    mm<NPM>(S.B[3], S.B[1], S.B[1], np); // X^4
    // T_19 = B_0 + X^4 (B_1 + X^4 (B_2 + X^4 (B_3 + X^4 B_4)))
    TaylorBlock<PLD> tb{{nullptr, S.B[0], S.B[1], S.B[2]}, S.c, 4};
    double* R = S.B[4];
    double* R2 = S.B[5];
    for (int idx = threadIdx.x; idx < np * np; idx += CH_BLOCK) {
        const int r = idx / np, c = idx - r * np;
        R[r * PLD + c] = tb(r, c);
    }
    __syncthreads();
    for (int i = 3; i >= 0; --i) {
        tb.i = i;
        mm<NPM>(R2, S.B[3], R, np, tb);
        double* t = R;
        R = R2;
        R2 = t;
    }
    double* X = R;
    double* Y = R2;
    if (threadIdx.x == 0 && nsq < NLVL) S.lvl[nsq] = hnext * fabs(X[(j - 1) * PLD + j]);
    for (int i = 1; i <= nsq; ++i) {
        mm<NPM>(Y, X, X, np);
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

template <int PLD>
__device__ void store_u(Ctl* ctl, const double* E, int j) {
    for (int i = threadIdx.x; i < j; i += CH_BLOCK) ctl->u[i] = E[i * PLD + j];
}

// ---------------------------------------------------------------------------
// phi of the Hessenberg matrix after an Arnoldi iteration, convergence test
// and residual-time trace (Fig. 3; eqs. rm, phi_stop).  One workgroup.
// MGS iteration k: dimension j = k + 1, h_{j+1,j} from the norm
// partials.  DCGS2 (DC) iteration k >= 1: dimension j = k, H final up to
// column j - 1 (written by the update launch of the same iteration).
//
// Trace: the squaring chain of the evaluation at tau0 gives resnorm at every
// s = tau0 2^-kk; the largest passing one brackets the crossing in
// [tau0 2^-kk, tau0 2^(1-kk)] (further halvings are evaluated if the chain is
// too short).  The crossing resnorm(s) = tol_phi is then located by Newton's
// method on log resnorm against log s, using d resnorm/ds =
// h_{j+1,j} |e_j^T exp(-s H) e_1| from the same exponential, safeguarded by the
// bracket, to a relative precision of about 1e-14.
// ---------------------------------------------------------------------------
// One phi test of Krylov dimension j (h_{j+1,j} = hnext, H columns 0..j-1
// final): returns true when the Krylov cycle is finished (converged, traced
// at the last dimension, or failed).
template <int NPM>
__device__ __forceinline__ bool phi_test(PhiShared<NPM>& S, Ctl* ctl, int* dflag, int j, double hnext, const double* hlast) {
    constexpr int PLD = PhiShared<NPM>::LD;
    // One exponential per pass of the loop below (a single call site keeps
    // the register footprint of one evaluation).  Phases: 0 the test at
    // tau0; 1 dyadic steps below the squaring chain, until one passes; 2
    // Newton inside the bracket; 3 the final evaluation at the chosen step.
    const double* H = ctl->H;
    const double tau0 = ctl->tau0, tol = ctl->tol_phi, tau_min = ctl->tau_min;
    int phase = 0, kk = 0, it = 0, kchain = 0;   // kchain: deepest level of the first squaring chain
    double s = tau0, lo = -1.0, hi = 0.0, rlo = 0.0, rhi = 0.0, prev = 0.0, step_prev = 1.0;
    int fail = 0;   // ch_status of a failed cycle
    auto finish = [&](const double* E, double sf, double res, int conv) {
        store_u<PLD>(ctl, E, j);
        if (threadIdx.x == 0) {
            ctl->tau_acc = sf;
            ctl->resnorm = res;
            ctl->converged = conv;
            if (!conv) ctl->traced = 1;
            ctl->done = 1;
            if (dflag) *dflag = ctl->cyc;
            ctl->j = j;
        }
    };
    // first Newton iterate inside [lo, hi]: log resnorm against log2(s / lo)
    // through the chain's values at lo / 2, lo and hi (quadratic) when they
    // are at hand, else through lo and hi
    auto first_guess = [&](bool chain) {
        double g = -1.0;
        if (rlo > 0.0 && rhi > rlo) {
            const double y0 = log(rlo), y1 = log(rhi), yt = log(tol);
            double x = (yt - y0) / (y1 - y0);
            const int kl = (int)lrint(log2(tau0 / lo));   // lo = tau0 2^-kl
            if (chain && kl + 1 <= kchain && S.lvl[kl + 1] > 0.0 && S.lvl[kl + 1] < rlo) {
                const double ym = log(S.lvl[kl + 1]);
                const double bq = 0.5 * (y1 - ym), cq = 0.5 * (y1 + ym) - y0;
                const double disc = bq * bq - 4.0 * cq * (y0 - yt);
                if (fabs(cq) > 1e-12 * fabs(bq) && disc >= 0.0) {
                    const double xq = (-bq + sqrt(disc)) / (2.0 * cq);
                    if (xq > 0.0 && xq < 1.0) x = xq;
                }
            }
            g = lo * exp2(x);
        }
        if (!(g > lo && g < hi)) g = 0.5 * (lo + hi);
        return g;
    };
    for (;;) {
        int nsq = 0;
        const double* E = expm_aug<NPM>(S, H, hlast, j, s, hnext, &nsq);
        const double uj = E[(j - 1) * PLD + j];
        const double r = hnext * fabs(uj);
        if (phase == 0) {
            if (!(r < __builtin_inf())) {
                fail = CH_ENONFINITE;
                break;
            }
            if (r <= tol) {
                finish(E, tau0, r, 1);
                return true;
            }
            if (j < ctl->m_max) {
                if (threadIdx.x == 0) ctl->resnorm = r;
                return false;
            }
            // ---- trace: largest passing dyadic step below tau0 ----
            const int kmax = nsq < NLVL - 1 ? nsq : NLVL - 1;
            kchain = kmax;
            for (int q = 1; q <= kmax; ++q) {
                if (S.lvl[q] <= tol) {
                    lo = ldexp(tau0, -q);
                    rlo = S.lvl[q];
                    hi = 2.0 * lo;
                    rhi = S.lvl[q - 1];
                    break;
                }
            }
            if (lo < 0.0) {   // below the chain: more halvings, one evaluation each
                prev = S.lvl[kmax];
                kk = kmax + 1;
                s = ldexp(tau0, -kk);
                if (kk > 1100 || s == 0.0 || s < tau_min) {
                    fail = CH_ETAU_UNDERFLOW;
                    break;
                }
                phase = 1;
                continue;
            }
            if (lo < tau_min) {
                fail = CH_ETAU_UNDERFLOW;
                break;
            }
            s = first_guess(true);
            phase = 2;
            continue;
        }
        if (phase == 1) {
            if (r <= tol) {
                lo = s;
                rlo = r;
                hi = 2.0 * s;
                rhi = prev;
                if (lo < tau_min) {
                    fail = CH_ETAU_UNDERFLOW;
                    break;
                }
                s = first_guess(false);
                phase = 2;
                continue;
            }
            prev = r;
            ++kk;
            s = ldexp(tau0, -kk);
            if (kk > 1100 || s == 0.0 || s < tau_min) {
                fail = CH_ETAU_UNDERFLOW;
                break;
            }
            continue;
        }
        if (phase == 2) {
            // Newton on log resnorm against log s, d resnorm / ds =
            // h_{j+1,j} |e_j^T exp(-s H) e_1| from the same exponential; it
            // converges quadratically, so a Newton step below 1e-7 s after
            // one below 1e-3 s leaves the next iterate within about 1e-14 of
            // the crossing.  Bisection steps (Newton iterate outside the
            // bracket) say nothing about convergence and reset that count.
            const double dr = hnext * (uj >= 0.0 ? 1.0 : -1.0) * E[(j - 1) * PLD + 0];
            if (r <= tol) {
                lo = s;
                rlo = r;
            } else {
                hi = s;
                rhi = r;
            }
            double sn = -1.0;
            if (r > 0.0 && dr > 0.0) sn = s * exp(-log(r / tol) * r / (s * dr));
            bool stop;
            if (hi - lo <= 0x1p-47 * lo) {
                sn = lo;
                stop = true;
            } else if (sn > 0.0 && fabs(sn - s) <= 1e-14 * s) {
                // s is the crossing to rounding (from the passing side the
                // Newton iterate may round onto lo itself); passing, it is
                // the step, and this exponential its result
                if (r <= tol) {
                    finish(E, s, r, 0);
                    return true;
                }
                stop = true;
            } else {
                const bool newton = sn > lo && sn < hi;
                if (!newton) sn = 0.5 * (lo + hi);
                const double step = fabs(sn - s) / s;
                stop = (newton && step <= 1e-7 && step_prev <= 1e-3) || ++it >= 60;
                step_prev = newton ? step : 1.0;
            }
            s = sn;
            if (stop) phase = 3;
            continue;
        }
        finish(E, s, r, 0);   // phase 3
        return true;
    }
    if (threadIdx.x == 0) {
        ctl->status = fail;
        ctl->halted = 1;
        ctl->done = 1;
        if (dflag) *dflag = ctl->cyc;
        ctl->j = 0;
    }
    return true;
}

// ---------------------------------------------------------------------------
// DCGS2 update pass of iteration j with the phi test of Krylov dimension j in
// the same launch (padded orders up to 32, j <= 31): workgroup w < ninst
// tests instance w, forming column j - 1 of H from its own copy of the
// iteration's coefficients; the others do the update pass.  The test then
// overlaps the update instead of needing a second stream.
// ---------------------------------------------------------------------------
constexpr int NPS = 32;
union DcPhiLds {
    DcCoef C;
    PhiShared<NPS> P;
};

__device__ void taylor_coefficients(double* c) {
    if (threadIdx.x == 0) {   // 1 / k!, k = 0..19
        double f = 1.0;
        c[0] = 1.0;
        for (int i = 1; i < 20; ++i) {
            f /= double(i);
            c[i] = f;
        }
    }
}

template <bool SINGLE>
__device__ __forceinline__ void dc_phi_wg(DcPhiLds& L, Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst& inst0,
                          int w, int j, int* __restrict__ dflags) {
    const Inst I = SINGLE ? inst0 : insts[w];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    int* dflag = dflags ? dflags + I.slot : nullptr;
    dc_prepare(L.C, ctl, j, true, false);   // column j - 1 of H, rho = h_{j+1,j} last
    __syncthreads();
    const double h = (int)threadIdx.x < j ? L.C.hf[threadIdx.x] : 0.0;
    const double hnext = L.C.hf[j];
    __syncthreads();                        // the coefficients are dead from here on
    if ((int)threadIdx.x < j) L.P.hcol[threadIdx.x] = h;
    taylor_coefficients(L.P.c);
    __syncthreads();
    phi_test<NPS>(L.P, ctl, dflag, j, hnext, L.P.hcol);
}

// Three workgroups per CU: the LDS of the phi part (about 51 KB) admits no
// more, and the matching register cap (168) keeps the update workgroups at
// three waves per SIMD instead of the one the unbounded phi code would leave.
// An update workgroup that starts after the test of its own launch has ended
// the cycle skips its share; the columns j and j + 1 it would write are not
// read by a finished cycle (its result uses columns 0..j-1 and u).
template <typename TV, bool SINGLE, bool NT>
__global__ __launch_bounds__(CH_BLOCK, 3) void k_dc_update_phi(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                            const int* __restrict__ cb2i, const Inst inst0, int ninst,
                                                            TV* __restrict__ V, size_t ldv, int j,
                                                            int* __restrict__ dflags, int* __restrict__ dprog,
                                                            int* __restrict__ dcount) {
    report_launch(dprog, dcount);
    __shared__ DcPhiLds L;
    if ((int)blockIdx.x < ninst) {
        dc_phi_wg<SINGLE>(L, ctls, insts, inst0, blockIdx.x, j, dflags);
        return;
    }
    dc_update_wg<TV, SINGLE, 0, NT>(L.C, ctls, insts, cb2i, inst0, blockIdx.x - ninst, V, ldv, j);
}

// MGS iteration k: dimension j = k + 1, h_{j+1,j} from the norm partials of
// the final Gram-Schmidt pass.  DCGS2 (DC): dimensions k .. k_last (>= 1),
// in order, until one ends the cycle; H is final up to column k_last - 1
// (written by the update launches of those iterations).
// BIG: orders above NPMAX, with the matrices in the instance's slot of the
// device scratch `big` (the workgroup's global writes are ordered for its
// other threads by the same barriers as LDS).
template <int NPM>
__device__ __forceinline__ void phi_tests(PhiShared<NPM>& S, Ctl* ctl, int* dflag, const Inst& I, bool dc, int k,
                                          int k_last, const double* __restrict__ pin, int pin_stencil) {
    taylor_coefficients(S.c);
    __syncthreads();
    if (dc) {
        for (int j = k; j <= k_last; ++j) {
            __syncthreads();   // the previous test's reads of ctl are complete
            if (phi_test<NPM>(S, ctl, dflag, j, ctl->H[j + (j - 1) * CH_LDH], nullptr)) return;
        }
        return;
    }
    // h_{k+2,k+1} = ||w|| from the final Gram-Schmidt pass (Fig. 3)
    double nrm2[1];
    sum_inst_partials<1, RED_SUM>(pin, I, pin_stencil, nrm2);
    const double hnext = sqrt(nrm2[0]);
    if (threadIdx.x == 0) {
        ctl->H[(k + 1) + k * CH_LDH] = hnext;
        ctl->vscale[k + 1] = hnext > 0.0 ? 1.0 / hnext : 0.0;
    }
    __syncthreads();   // H column k complete (written by the Gram-Schmidt launches and above)
    phi_test<NPM>(S, ctl, dflag, k + 1, hnext, nullptr);
}

template <bool SINGLE, bool DC, bool BIG>
__global__ __launch_bounds__(CH_BLOCK) void k_phi(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst, int k,
                                                  int k_last, const double* __restrict__ pin, int pin_stencil,
                                                  int* __restrict__ dflags, PhiShared<NPBIG>* __restrict__ big) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];   // one workgroup per instance
    Ctl* ctl = ctls + I.slot;
    int* dflag = dflags ? dflags + I.slot : nullptr;
    if (ctl->done | ctl->halted) return;
    if constexpr (BIG) {
        phi_tests<NPBIG>(big[I.slot], ctl, dflag, I, DC, k, k_last, pin, pin_stencil);
    } else {
        __shared__ PhiShared<NPMAX> S;
        phi_tests<NPMAX>(S, ctl, dflag, I, DC, k, k_last, pin, pin_stencil);
    }
}

// ---------------------------------------------------------------------------
// Step begin (Fig. 4): final-time clip and tol_phi (eq. tol_phi).
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
// EE2 step end (Fig. 4): est (eq. LIMest), t, tau_new (eq. EEdt);
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
// LIM step begin (Figs. 1 and 2: bounds of the spectrum): partials of
// min/max y^2 (and a non-finite flag) on periodic grids; with Neumann
// boundaries, of the largest absolute column sum of Ahat_n itself ...
// ---------------------------------------------------------------------------
// Absolute sum of column j = (ix, iy) of Ahat_n = A (J_n + eps^2 A) [+ A with
// the Eyre splitting] on the 2-D cell-centred Neumann grid, d = the diagonal
// of J_n at j, a = 1/h^2, e = eps^2/h^4.  A_jj = deg_j a and A_ij = -a for the
// existing neighbours i (deg: their number), so column j of Ahat_n = A D +
// eps^2 A^2 holds d deg_j a + e (deg_j^2 + deg_j) on the diagonal,
// -d a - e (deg_i + deg_j) at each neighbour, e at each point two steps away
// along an axis and 2 e at each diagonal point, where those exist.  On a
// periodic grid (deg = 4 everywhere) this is the closed form of k_lim_plan.
__device__ __forceinline__ double neumann_colsum(int ix, int iy, int n, double d, double a, double e) {
    auto deg = [n](int x, int y) { return (x > 0) + (x < n - 1) + (y > 0) + (y < n - 1); };
    const int dj = deg(ix, iy);
    double s = fabs(d * dj * a + e * double(dj * dj + dj));
    if (ix > 0) s += fabs(-d * a - e * double(deg(ix - 1, iy) + dj));
    if (ix < n - 1) s += fabs(-d * a - e * double(deg(ix + 1, iy) + dj));
    if (iy > 0) s += fabs(-d * a - e * double(deg(ix, iy - 1) + dj));
    if (iy < n - 1) s += fabs(-d * a - e * double(deg(ix, iy + 1) + dj));
    s += e * double((ix > 1) + (ix < n - 2) + (iy > 1) + (iy < n - 2));
    s += 2.0 * e * double((ix > 0 && iy > 0) + (ix > 0 && iy < n - 1) + (ix < n - 1 && iy > 0) +
                          (ix < n - 1 && iy < n - 1));
    return s;
}

// Absolute sum of column j = (ix, iy) of Ahat_n = A_M (D + eps^2 A) on the
// periodic grid with variable mobility (Section 2, Remark 1), a = 1/h^2,
// mu_ik = (M_i + M_k)/2 and S_i = sum of mu_ik over the four neighbours k of i:
//   row j:                    a S_j (d_j + 4 a eps^2) + a^2 eps^2 S_j
//   neighbour i of j:        -a mu_ij (d_j + 4 a eps^2) - a^2 eps^2 S_i
//   i = j +- 2 e_x, +- 2 e_y: a^2 eps^2 mu_(i, midpoint)
//   diagonal i = j + e_x + e_y (four): a^2 eps^2 (mu_(i, j + e_x) + mu_(i, j + e_y))
// The entries need M at the 13 points within distance 2 (in the 1-norm) of
// j; with M = 1 the sum is the closed form of k_lim_plan.
__device__ __forceinline__ double mobility_colsum(const double* __restrict__ y, int ix, int iy, int n, double d,
                                                  double a, double eps2, double m0, double m1) {
    const double ae = a * a * eps2;
    auto M = [&](int dx, int dy) {
        const int x = wrapi(ix + dx, n), yy = wrapi(iy + dy, n);
        return mobility_of(y[(size_t)yy * n + x], m0, m1);
    };
    const double mc = M(0, 0);
    const double mxp = M(1, 0), mxm = M(-1, 0), myp = M(0, 1), mym = M(0, -1);
    const double mpp = M(1, 1), mpm = M(1, -1), mmp = M(-1, 1), mmm = M(-1, -1);
    const double m2xp = M(2, 0), m2xm = M(-2, 0), m2yp = M(0, 2), m2ym = M(0, -2);
    const double uxp = 0.5 * (mc + mxp), uxm = 0.5 * (mc + mxm), uyp = 0.5 * (mc + myp), uym = 0.5 * (mc + mym);
    const double Sj = (uxp + uxm) + (uyp + uym);
    // S of the four neighbours (faces to j, the axis-2 point and two diagonals)
    const double Sxp = uxp + 0.5 * (mxp + m2xp) + 0.5 * (mxp + mpp) + 0.5 * (mxp + mpm);
    const double Sxm = uxm + 0.5 * (mxm + m2xm) + 0.5 * (mxm + mmp) + 0.5 * (mxm + mmm);
    const double Syp = uyp + 0.5 * (myp + m2yp) + 0.5 * (myp + mpp) + 0.5 * (myp + mmp);
    const double Sym = uym + 0.5 * (mym + m2ym) + 0.5 * (mym + mpm) + 0.5 * (mym + mmm);
    const double b = d + 4.0 * a * eps2;   // B_jj
    double s = fabs(a * Sj * b + ae * Sj);
    s += fabs(a * uxp * b + ae * Sxp) + fabs(a * uxm * b + ae * Sxm);
    s += fabs(a * uyp * b + ae * Syp) + fabs(a * uym * b + ae * Sym);
    // axis-2 points: the face between the point and the midpoint
    s += ae * (0.5 * (m2xp + mxp) + 0.5 * (m2xm + mxm) + 0.5 * (m2yp + myp) + 0.5 * (m2ym + mym));
    // diagonal points: their faces to the two common neighbours of j
    s += ae * ((0.5 * (mpp + mxp) + 0.5 * (mpp + myp)) + (0.5 * (mpm + mxp) + 0.5 * (mpm + mym)) +
               (0.5 * (mmp + mxm) + 0.5 * (mmp + myp)) + (0.5 * (mmm + mxm) + 0.5 * (mmm + mym)));
    return s;
}

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
    const bool neu = I.bc == CH_BC_NEUMANN;
    const double a = I.inv_h2, e = I.eps2 * I.inv_h2 * I.inv_h2;
    for (long long q = (long long)(blockIdx.x - I.cblk0) * CH_BLOCK + threadIdx.x; q < I.N; q += stride) {
        const double v = y[q] * y[q];
        if (v < __builtin_inf()) {
            if (neu) {   // the column sum itself (2-D: q = iy n + ix)
                const int iy = (int)(q / I.n), ix = (int)(q - (long long)iy * I.n);
                mx = fmax(mx, neumann_colsum(ix, iy, I.n, 3.0 * v - 1.0 + I.eyre, a, e));
            } else if (I.mob) {
                const int iy = (int)(q / I.n), ix = (int)(q - (long long)iy * I.n);
                mx = fmax(mx, mobility_colsum(y, ix, iy, I.n, 3.0 * v - 1.0 + I.eyre, a, I.eps2, ctl->mob0, ctl->mob1));
            } else {
                mn = fmin(mn, v);
                mx = fmax(mx, v);
            }
        } else {
            bad = 1.0;
        }
    }
    double x[3] = {-mn, mx, bad};
    write_partials<3, RED_MAX>(x, pout);
}

// Order of the Chebyshev nodes beta_i = cos(pi (2i - 1) / (2p)) in a LIM
// step (Fig. 1 fixes only beta_1 as the first): Leja order -- beta_1, then
// each time the node with the largest sum of log-distances to the nodes taken
// so far, the smallest index among those within 1e-9 (relative) of the
// largest.  Any order gives the same step in exact arithmetic; this one keeps
// the growth of intermediate stages, and so the amplification of rounding,
// small (below 10^7.2 up to p = 4096, against 10^105 at p = 209 for the
// order i = 1..p).  0-based indices into order[0..p); one workgroup.
// The log-distances come from one table: with theta_i = pi (2i + 1) / (2p),
// cos a - cos b = -2 sin((a + b)/2) sin((a - b)/2) gives
//   log|beta_i - beta_r| = log 2 + L[i + r + 1] + L[|i - r|],
//   L[k] = log sin(pi k / (2p)),  1 <= k <= 2p - 1,
// so a step costs two table reads per open node instead of a logarithm (and
// has no cancellation between nearby nodes).  The sums stay in registers; a
// pick costs two workgroup reductions.  order is in LDS.
// Wave-wide reduction with a uniform result: DPP within the four rows, then
// the four row results by readlane (no LDS permute on the critical path).
template <typename Op>
__device__ __forceinline__ double wave_reduce_rl(double x, Op op) {
    x = op(x, dpp_move<DPP_XOR1>(x));
    x = op(x, dpp_move<DPP_XOR2>(x));
    x = op(x, dpp_move<DPP_HMIR>(x));
    x = op(x, dpp_move<DPP_MIR>(x));
    return op(op(readlane_d(x, 0), readlane_d(x, 16)), op(readlane_d(x, 32), readlane_d(x, 48)));
}

__device__ __forceinline__ void lim_leja_order(int p, int* __restrict__ order) {
    constexpr int K = CH_PMAX / CH_BLOCK, G = 8, NW = CH_BLOCK / 64;
    __shared__ double L[2 * CH_PMAX];
    __shared__ double wmax[NW], wmin[NW];
    const double pi = 3.141592653589793, log2 = 0.6931471805599453;
    for (int k = threadIdx.x; k < 2 * CH_PMAX; k += CH_BLOCK)
        L[k] = (k == 0 || k >= 2 * p) ? 0.0 : log(sin(pi * double(k) / double(2 * p)));
    // Thread t owns nodes t + CH_BLOCK k, in groups of G whose table reads are
    // in flight together.  Taken nodes and nodes past p hold -inf, which no
    // update or comparison changes.
    const int tid = threadIdx.x, w = tid >> 6;
    const int gn = (p + CH_BLOCK * G - 1) / (CH_BLOCK * G);
    double sc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) sc[k] = tid + CH_BLOCK * k < p ? 0.0 : -__builtin_inf();
    __syncthreads();
    int r = 0;
    for (int s = 0; s < p; ++s) {
        if (tid == 0) order[s] = r;
        double best = -__builtin_inf();
#pragma unroll
        for (int g = 0; g < K / G; ++g) {
            if (g < gn) {
#pragma unroll
                for (int k = g * G; k < g * G + G; ++k) {
                    const int i = tid + CH_BLOCK * k, d = i - r;
                    const double t = log2 + (L[i + r + 1] + L[d < 0 ? -d : d]);
                    // the node just taken becomes -inf; an added mask (rather
                    // than a select) keeps the loop free of branches
                    sc[k] = (sc[k] + t) + (d == 0 ? -__builtin_inf() : 0.0);
                    best = fmax(best, sc[k]);
                }
            }
        }
        if (s == p - 1) break;
        best = wave_reduce_rl(best, [](double x, double y) { return fmax(x, y); });
        if ((tid & 63) == 0) wmax[w] = best;
        __syncthreads();
        best = wmax[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) best = fmax(best, wmax[q]);
        const double lim = best - 1e-9 * fmax(1.0, fabs(best));
        double c = double(p);
#pragma unroll
        for (int g = K / G - 1; g >= 0; --g) {
            if (g < gn) {
#pragma unroll
                for (int k = g * G + G - 1; k >= g * G; --k)
                    if (sc[k] >= lim) c = double(tid + CH_BLOCK * k);
            }
        }
        c = wave_reduce_rl(c, [](double x, double y) { return fmin(x, y); });
        if ((tid & 63) == 0) wmin[w] = c;
        __syncthreads();
        c = wmin[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) c = fmin(c, wmin[q]);
        r = (int)c;
    }
}

// ... then the final-time clip, lambda_max = ||Ahat_n||_1, p (eq. p) and the
// order of the nodes (lim_leja_order).
// Column j of Ahat_n is d_j A e_j + eps^2 A^2 e_j; its absolute sum g(d_j) is
// convex and piecewise linear in d_j, so the largest column sum is
// max(g(d_min), g(d_max)):
//   2-D: g(d) = |4d/h^2 + 20e| + 4|d/h^2 + 8e| + 12e,      e = eps^2/h^4
//   3-D: g(d) = |6d/h^2 + 42e| + 6|d/h^2 + 12e| + 30e
// The order of an instance's step (0: halted) to its pinned host words, then
// the tag of this plan launch, so that the host, which waits for the tags,
// sizes the stage launches without copying the control blocks back.
__device__ __forceinline__ void publish_order(int* dlim, int slot, int p, int seq) {
    if (dlim && threadIdx.x == 0) {
        dlim[2 * slot] = p;
        __threadfence_system();
        dlim[2 * slot + 1] = seq;
    }
}

template <bool SINGLE>
__global__ __launch_bounds__(CH_BLOCK) void k_lim_plan(Ctl* __restrict__ ctls, const Inst* __restrict__ insts, const Inst inst0, int ninst,
                                                       const double* __restrict__ pin, int pin_stencil, int dim,
                                                       int* __restrict__ orders, double* __restrict__ coefs,
                                                       int* __restrict__ dlim, int seq) {
    const Inst I = SINGLE ? inst0 : insts[blockIdx.x];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) {
        publish_order(dlim, I.slot, 0, seq);
        return;
    }
    double tot[3];
    sum_inst_partials<3, RED_MAX>(pin, I, pin_stencil, tot);
    __shared__ int sp;
    if (threadIdx.x == 0) {
        sp = 0;
        const double ymin2 = -tot[0], ymax2 = tot[1];
        if (tot[2] != 0.0) {
            ctl->status = CH_ENONFINITE;
            ctl->halted = 1;
        } else if (!(ctl->t < ctl->T) || (ctl->max_steps > 0 && ctl->steps >= ctl->max_steps)) {
            ctl->halted = 1;
        } else {
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
            if (I.bc == CH_BC_NEUMANN || I.mob) {   // the largest column sum, from the begin launch
                gmin = gmax = tot[1];
            } else if (dim == 2) {
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
            } else {
                ctl->clipped = clipped;
                ctl->tau0 = tau;
                ctl->lam = lam;
                ctl->p = (int)pr;
                sp = (int)pr;
            }
        }
    }
    __syncthreads();
    const int p = sp;
    publish_order(dlim, I.slot, p, seq);
    if (p == 0) return;
    __shared__ int order[CH_PMAX];
    lim_leja_order(p, order);
    __syncthreads();
    int* gorder = orders + (size_t)I.slot * CH_PMAX;
    for (int i = threadIdx.x; i < p; i += CH_BLOCK) gorder[i] = order[i];
    // Fig. 1: beta_i = cos(pi (2i - 1) / (2p)), z_1 = beta_1,
    // a_m = lambda_max (z_1 - beta_m) / (1 + z_1).  Stage position pos takes
    // the node order[pos] (first sweep, pos < p) or order[pos - p + 1]
    // (second sweep, without beta_1); its coefficients are
    // (tau a_m, 1 / (1 + tau a_m)).
    const double pi = 3.141592653589793;
    const double z1 = cos(pi / double(2 * p));
    const double lam = ctl->lam, tau = ctl->tau0;
    double* cf = coefs + (size_t)I.slot * 2 * CH_PMAX * 2;
    for (int pos = threadIdx.x; pos < 2 * p - 1; pos += CH_BLOCK) {
        const int m = 1 + order[pos < p ? pos : pos - p + 1];
        const double am = lam / (1.0 + z1) * (z1 - cos(pi * double(2 * m - 1) / double(2 * p)));
        const double ta = tau * am;
        cf[2 * pos] = ta;
        cf[2 * pos + 1] = 1.0 / (1.0 + ta);
    }
}

// LIM step end (Fig. 2): est (eq. LIMest), t, tau_new (eq. LIMdt).
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

size_t phi_big_bytes() { return sizeof(PhiShared<NPBIG>); }

template <bool DC, bool BIG>
static void launch_phi_t(const Table& t, const DevBuffers& b, PartSeq& ps, int k, int k_last, hipStream_t s) {
    auto* big = static_cast<PhiShared<NPBIG>*>(b.phibig);
    const double* pin = DC ? nullptr : ps.in();
    const int pk = DC ? 0 : ps.stencil;
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_phi<true, DC, BIG>), IARGS, k, k_last, pin, pk, b.dflag, big);
    else
        hipLaunchKernelGGL((k_phi<false, DC, BIG>), IARGS, k, k_last, pin, pk, b.dflag, big);
}

hipError_t launch_phi(const Table& t, const DevBuffers& b, PartSeq& ps, int k, int k_last, bool dc, hipStream_t s) {
    // the largest Krylov dimension tested: k_last (DCGS2) or k + 1 (MGS)
    const bool big = (dc ? k_last : k + 1) + 1 > NPMAX;
    if (big && !b.phibig) return hipErrorInvalidValue;
    if (dc) {
        if (big) launch_phi_t<true, true>(t, b, ps, k, k_last, s);
        else launch_phi_t<true, false>(t, b, ps, k, k_last, s);
    } else {
        if (big) launch_phi_t<false, true>(t, b, ps, k, k, s);
        else launch_phi_t<false, false>(t, b, ps, k, k, s);
    }
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

hipError_t launch_dots_reduce(const Table& t, const DevBuffers& b, int k, hipStream_t s) {
    const dim3 grid(2 * k + 2, t.ninst);
    const int kind = PK_STRIP;   // the DCGS2 matvec runs on strips (2-D) or marching tiles (3-D)
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_dots_reduce<true>), grid, dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.hinst[0], t.ninst,
                           b.dots, kind);
    else
        hipLaunchKernelGGL((k_dots_reduce<false>), grid, dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.hinst[0], t.ninst,
                           b.dots, kind);
    return hipGetLastError();
}

template <typename TV, bool NT>
static void launch_dc_update_nt(const Table& t, const DevBuffers& b, int j, bool timing, hipStream_t s) {
    TV* V = static_cast<TV*>(b.V);
    if (timing) {
        hipLaunchKernelGGL((k_dc_update<TV, true, 1, NT>), CARGS, V, b.ldv, j, nullptr, nullptr);
        return;
    }
    if (b.hseq) ++*b.hseq;
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_dc_update<TV, true, 0, NT>), CARGS, V, b.ldv, j, b.dprog, b.dcount);
    else
        hipLaunchKernelGGL((k_dc_update<TV, false, 0, NT>), CARGS, V, b.ldv, j, b.dprog, b.dcount);
}

template <typename TV>
static void launch_dc_update_t(const Table& t, const DevBuffers& b, int j, bool timing, hipStream_t s) {
    if (stream_columns(b.ldv, sizeof(TV), j)) launch_dc_update_nt<TV, true>(t, b, j, timing, s);
    else launch_dc_update_nt<TV, false>(t, b, j, timing, s);
}

template <typename TV, bool NT>
static void launch_dc_update_phi_nt(const Table& t, const DevBuffers& b, int j, hipStream_t s) {
    TV* V = static_cast<TV*>(b.V);
    const dim3 grid(t.ninst + t.cgrid);
    if (b.hseq) ++*b.hseq;
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_dc_update_phi<TV, true, NT>), grid, dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.cb2i,
                           t.hinst[0], t.ninst, V, b.ldv, j, b.dflag, b.dprog, b.dcount);
    else
        hipLaunchKernelGGL((k_dc_update_phi<TV, false, NT>), grid, dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.cb2i,
                           t.hinst[0], t.ninst, V, b.ldv, j, b.dflag, b.dprog, b.dcount);
}

template <typename TV>
static void launch_dc_update_phi_t(const Table& t, const DevBuffers& b, int j, hipStream_t s) {
    if (stream_columns(b.ldv, sizeof(TV), j)) launch_dc_update_phi_nt<TV, true>(t, b, j, s);
    else launch_dc_update_phi_nt<TV, false>(t, b, j, s);
}

hipError_t launch_dc_update(const Table& t, int prec, const DevBuffers& b, int j, hipStream_t s, bool timing,
                            bool with_phi) {
    if (with_phi) {
        if (prec == CH_FP64) launch_dc_update_phi_t<double>(t, b, j, s);
        else launch_dc_update_phi_t<float>(t, b, j, s);
    } else if (prec == CH_FP64) {
        launch_dc_update_t<double>(t, b, j, timing, s);
    } else {
        launch_dc_update_t<float>(t, b, j, timing, s);
    }
    return hipGetLastError();
}

hipError_t launch_dc_finish(const Table& t, const DevBuffers& b, int j, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_dc_finish<true>), dim3(t.ninst), dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.hinst[0],
                           t.ninst, j);
    else
        hipLaunchKernelGGL((k_dc_finish<false>), dim3(t.ninst), dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.hinst[0],
                           t.ninst, j);
    return hipGetLastError();
}

// One Arnoldi iteration.  MGS: iteration k makes column k + 1 and tests
// dimension k + 1.  DCGS2: iteration k (0..m_max) finishes column k - 1,
// tests dimension k and (k < m_max) makes columns k and k + 1.
hipError_t launch_arnoldi_iter(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int k,
                               int orth, int m_max, const LaunchEnv* env, hipStream_t s, bool* side_used) {
    hipError_t e;
    if (orth == CH_ORTH_DCGS2) {
        const bool store = k < m_max;
        if ((e = launch_matvec(t, prec, b, ps, y, k, MV_DOTS_DC, store, s)) != hipSuccess) return e;
        if ((e = launch_dots_reduce(t, b, k, s)) != hipSuccess) return e;
        if (store) {
            // the test of dimension k rides in the update launch when it fits
            if (k >= 1 && phi_in_update(k)) return launch_dc_update(t, prec, b, k, s, false, true);
            if ((e = launch_dc_update(t, prec, b, k, s)) != hipSuccess || k == 0) return e;
            if (!env) return launch_phi(t, b, ps, k, k, true, s);
            // a larger one on the second stream, overlapping the next iterations
            if ((e = hipEventRecord(env->ev_main, s)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(env->side, env->ev_main, 0)) != hipSuccess) return e;
            if (side_used) *side_used = true;
            return launch_phi(t, b, ps, k, k, true, env->side);
        }
        // the last test (and its residual-time trace) follows the final pass,
        // after every earlier test
        if ((e = launch_dc_finish(t, b, k, s)) != hipSuccess || k == 0) return e;
        if (env && side_used && *side_used) {
            if ((e = hipEventRecord(env->ev_side, env->side)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, env->ev_side, 0)) != hipSuccess) return e;
            *side_used = false;
        }
        return launch_phi(t, b, ps, k, k, true, s);
    }
    if ((e = launch_matvec(t, prec, b, ps, y, k, MV_DOTS_ONE, true, s)) != hipSuccess) return e;
    for (int i = 1; i <= k + 1; ++i)
        if ((e = launch_mgs_pass(t, prec, b, ps, k, i, s)) != hipSuccess) return e;
    return launch_phi(t, b, ps, k, k, false, s);
}

// Waits (a bounded time) until the update launch with sequence number `seq`
// has begun on the device, or every instance has finished its cycle.
static void wait_progress(const Table& t, const DevBuffers& b, const int* expected, int seq) {
    const auto t0 = std::chrono::steady_clock::now();
    for (long long spin = 0;; ++spin) {
        if (*b.hprog >= seq || all_cycles_done(t, b, expected)) return;
        if ((spin & 255) == 255 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > CH_LOOKAHEAD_WAIT_S)
            return;   // issue anyway: the launches are correct whenever they run
    }
}

void destroy_graphs(GraphCache& g) {
    for (GraphEntry& e : g.e) (void)hipGraphExecDestroy(e.exec);
    g.e.clear();
    g.next = 0;
}

// Every value the launches of DCGS2 iterations [k0, k1) take as arguments.
static std::vector<unsigned long long> graph_key(const Table& t, int prec, const DevBuffers& b, const double* y,
                                                 int m_max, int k0, int k1) {
    std::vector<unsigned long long> k;
    auto p = [&k](const void* q) { k.push_back((unsigned long long)(uintptr_t)q); };
    auto v = [&k](long long x) { k.push_back((unsigned long long)x); };
    auto d = [&k](double x) { k.push_back(__builtin_bit_cast(unsigned long long, x)); };
    v(prec), v(m_max), v(k0), v(k1), v(t.ninst), v(t.sgrid), v(t.cgrid), v(t.wgrid), v(t.dim);
    p(t.inst), p(t.sb2i), p(t.cb2i), p(t.wb2i);
    p(y), p(b.V), v((long long)b.ldv), p(b.ctl), p(b.dots), p(b.dflag), p(b.dprog), p(b.dcount), p(b.y32);
    p(b.phibig), p(b.part);
    const Inst& I = t.hinst[0];   // passed by value to single-instance launches
    v(I.off), v(I.N), v(I.n), v(I.slot), v(I.sblk0), v(I.sblk), v(I.cblk0), v(I.cblk), d(I.eps2), d(I.inv_h2);
    v(I.eyre), v(I.wblk0), v(I.wblk), v(I.vx), v(I.bc), v(I.mob);
    return k;
}

// The graph of DCGS2 iterations [k0, k1), captured on env.cap on first use.
static hipError_t iteration_graph(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y,
                                  int m_max, int k0, int k1, const LaunchEnv& env, hipStream_t s,
                                  const GraphEntry** out) {
    GraphCache& g = *env.graphs;
    std::vector<unsigned long long> key = graph_key(t, prec, b, y, m_max, k0, k1);
    for (const GraphEntry& e : g.e)
        if (e.key == key) {
            *out = &e;
            return hipSuccess;
        }
    hipError_t e = hipStreamBeginCapture(env.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const int seq0 = b.hseq ? *b.hseq : 0;
    for (int k = k0; k < k1 && e == hipSuccess; ++k)
        e = launch_arnoldi_iter(t, prec, b, ps, y, k, CH_ORTH_DCGS2, m_max, nullptr, env.cap);
    const int updates = b.hseq ? *b.hseq - seq0 : 0;
    if (b.hseq) *b.hseq = seq0;   // counted again at each replay
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(env.cap, &graph);
    if (e == hipSuccess) e = ec;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    constexpr size_t CAP = 256;
    GraphEntry ne{std::move(key), exec, updates};
    if (g.e.size() < CAP) {
        g.e.push_back(std::move(ne));
        *out = &g.e.back();
    } else {   // replace the oldest, once no launch of it can still be running
        if ((e = hipStreamSynchronize(s)) != hipSuccess) {
            (void)hipGraphExecDestroy(exec);
            return e;
        }
        GraphEntry& old = g.e[g.next];
        (void)hipGraphExecDestroy(old.exec);
        old = std::move(ne);
        *out = &old;
        g.next = (g.next + 1) % CAP;
    }
    return hipSuccess;
}

// The DCGS2 iterations of a cycle as replayed graphs of env.graph_chunk
// iterations, with the same lookahead as direct issue (in whole graphs).  The
// tests of every iteration run on the main stream (no second stream).
static hipError_t launch_arnoldi_graphs(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y,
                                        int m_max, const int* expected, const LaunchEnv& env, hipStream_t s) {
    const int iters = m_max + 1, C = env.graph_chunk;
    int useq[CH_MMAX + 2];
    for (int k0 = 0; k0 < iters; k0 += C) {
        const int k1 = std::min(iters, k0 + C);
        if (b.hprog && b.hseq && expected && k0 > CH_LOOKAHEAD) wait_progress(t, b, expected, useq[k0 - 1 - CH_LOOKAHEAD]);
        if (k0 > 0 && all_cycles_done(t, b, expected)) break;
        const GraphEntry* g = nullptr;
        hipError_t e = iteration_graph(t, prec, b, ps, y, m_max, k0, k1, env, s, &g);
        if (e != hipSuccess) return e;
        if ((e = hipGraphLaunch(g->exec, s)) != hipSuccess) return e;
        // iteration k < m_max has one update launch, in order
        int q = b.hseq ? *b.hseq : 0;
        for (int k = k0; k < k1; ++k) useq[k] = k < m_max ? ++q : q;
        if (b.hseq) *b.hseq += g->updates;
    }
    return hipSuccess;
}

hipError_t launch_arnoldi(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int m_max,
                          int orth, const int* expected, const LaunchEnv* env, hipStream_t s) {
    const bool dc = orth == CH_ORTH_DCGS2;
    if (dc && env && env->graph_chunk > 0 && env->graphs && env->cap)
        return launch_arnoldi_graphs(t, prec, b, ps, y, m_max, expected, *env, s);
    const int iters = dc ? m_max + 1 : m_max;
    bool side_used = false;
    int useq[CH_MMAX + 2];   // sequence number of each iteration's update launch
    for (int k = 0; k < iters; ++k) {
        // the host issues at most CH_LOOKAHEAD iterations ahead of the
        // device's update launches: once a test ends the cycle, few launches
        // are left that only find it finished and exit
        if (dc && b.hprog && b.hseq && expected && k > CH_LOOKAHEAD)
            wait_progress(t, b, expected, useq[k - 1 - CH_LOOKAHEAD]);
        if (k > 0 && all_cycles_done(t, b, expected)) break;
        hipError_t e = launch_arnoldi_iter(t, prec, b, ps, y, k, orth, m_max, env, s, &side_used);
        if (e != hipSuccess) return e;
        useq[k] = b.hseq ? *b.hseq : 0;
    }
    if (side_used) {   // a cycle stopped early: its result may be a test still on the second stream
        hipError_t e = hipEventRecord(env->ev_side, env->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, env->ev_side, 0);
        return e;
    }
    return hipSuccess;
}

hipError_t launch_update(const Table& t, int prec, const DevBuffers& b, const double* y, double* ynew, bool unit,
                         hipStream_t s) {
    const int u = unit ? 1 : 0;
    if (prec == CH_FP64)
        if (t.ninst == 1)
            hipLaunchKernelGGL((k_update<double, true>), CARGS, y, static_cast<const double*>(b.V), b.ldv, ynew, u);
        else
            hipLaunchKernelGGL((k_update<double, false>), CARGS, y, static_cast<const double*>(b.V), b.ldv, ynew, u);
    else
        if (t.ninst == 1)
            hipLaunchKernelGGL((k_update<float, true>), CARGS, y, static_cast<const float*>(b.V), b.ldv, ynew, u);
        else
            hipLaunchKernelGGL((k_update<float, false>), CARGS, y, static_cast<const float*>(b.V), b.ldv, ynew, u);
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

hipError_t launch_lim_plan(const Table& t, const DevBuffers& b, PartSeq& ps, int seq, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_lim_plan<true>), IARGS, ps.in(), ps.stencil, t.dim, b.lorder, b.lcoef, b.dlim, seq);
    else
        hipLaunchKernelGGL((k_lim_plan<false>), IARGS, ps.in(), ps.stencil, t.dim, b.lorder, b.lcoef, b.dlim, seq);
    return hipGetLastError();
}

hipError_t launch_lim_end(const Table& t, const DevBuffers& b, PartSeq& ps, hipStream_t s) {
    if (t.ninst == 1)
        hipLaunchKernelGGL((k_lim_end<true>), IARGS, ps.in(), ps.stencil);
    else
        hipLaunchKernelGGL((k_lim_end<false>), IARGS, ps.in(), ps.stencil);
    return hipGetLastError();
}
