// Fused stencil kernels: Jacobian matvec with its Gram-Schmidt dot products,
// residual / right-hand side, LIM stage and the two error-estimate passes.
//
// Operators (Section 2, eq. IVP; Section 3.1, eqs. J, A_g; Section 3.3,
// eq. A_g_cs): -A is the (2 dim + 1)-point periodic Laplacian, d = 3 y^2 - 1
// (+1 with the Eyre splitting) is the diagonal of J_n (+I), and
//     Ahat v        = A (d v + eps^2 A v)
//     ghat - Ahat z = A (c - d z - eps^2 A z),   c = 2 y^3 (+ y with Eyre),
// since J_n y - F'(y) = 2 y^3.  Every kernel evaluates the inner expression on
// the halo-1 region in LDS and applies the outer A from LDS, so A^2 is never
// formed and each operand is read from HBM once per tile.
//
// One launch covers every instance of a batch: workgroup b works on instance
// sb2i[b], on the tiles lb, lb + sblk, ... of that instance (lb = b - sblk0).
#include "ch_common.h"
#include "ch_march.h"

namespace {

template <typename T>
__device__ __forceinline__ T dcoef(T y, int eyre) {
    return T(3) * y * y - T(1) + T(eyre);
}
template <typename T>
__device__ __forceinline__ T ccoef(T y, int eyre) {
    return T(2) * y * y * y + (eyre ? y : T(0));
}

// ---------------------------------------------------------------------------
// w = Ahat u, u = vscale[k] V_k (the matvec of Fig. 3), stored in column k + 1
// (unless store_w is 0), with the partials of its dot products:
//   DM_ONE  <w, V_0>                                   (the first MGS dot)
//   DM_DC   rows i < k: <u, V_i>; rows k + i: <w, V_i>;
//           row 2k: <u, u>; row 2k + 1: <u, w>          (DCGS2)
// ---------------------------------------------------------------------------
enum DotMode { DM_ONE = 0, DM_DC = 1 };

// TAG distinguishes the launches of the timing aid (same code, another symbol).
template <int DIM, typename TV, typename TY, bool SINGLE, int DM, int TAG>
__global__ __launch_bounds__(CH_BLOCK) void k_matvec(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                     const int* __restrict__ sb2i, const Inst inst0, int ninst, TV* __restrict__ V, size_t ldv,
                                                     int k, int store_w, const TY* __restrict__ ybase,
                                                     double* __restrict__ pout) {
    const Inst I = SINGLE ? inst0 : insts[sb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    constexpr int TX = Geo<DIM>::TX, TY_ = Geo<DIM>::TY;
    constexpr int PPT = tile_points<DIM>() / CH_BLOCK;   // output points per thread and tile
    static_assert(PPT * CH_BLOCK == tile_points<DIM>(), "tile size");
    static_assert(PPT == 2, "the dot phase takes two points per thread");
    constexpr int NW = CH_BLOCK / 64;
    constexpr bool MANY = DM != DM_ONE;
    __shared__ TV sv[R2::SIZE];
    __shared__ TV sd[R1::SIZE];
    __shared__ TV sq[R1::SIZE];
    __shared__ double red[DM == DM_DC ? CH_DROWS : 1][NW];
    __shared__ TV sw[MANY ? tile_points<DIM>() : 1];
    using VT = typename Vec16<TV>::type;
    constexpr int PD = Vec16<TV>::W;                                   // dot-phase points per thread
    constexpr int CG = PD * CH_BLOCK / tile_points<DIM>();             // column groups
    static_assert(CG * tile_points<DIM>() == PD * CH_BLOCK && (CH_BLOCK / CG) % 64 == 0, "dot-phase split");
    static_assert(Geo<DIM>::TX % PD == 0, "dot-phase points stay in one row");
    const TV* Vk = V + (size_t)k * ldv + I.off;
    TV* W = V + (size_t)(k + 1) * ldv + I.off;
    const TV* V0 = V + I.off;
    const TY* y = ybase + I.off;
    const int n = I.n, eyre = I.eyre;
    // DCGS2 keeps its columns normalised, except the start vector
    const TV sc = TV(DM == DM_DC && k > 0 ? 1.0 : ctl->vscale[k]);
    const TV ih2 = TV(I.inv_h2), e2ih2 = TV(I.eps2 * I.inv_h2);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nrows = 2 * k + 2;
    if (MANY)
        for (int i = threadIdx.x; i < nrows * NW; i += CH_BLOCK) red[i / NW][i % NW] = 0.0;
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    const int lb = blockIdx.x - I.sblk0;
    double dot = 0.0;
    for (int t = xcd_remap(lb, I.sblk); t < nt; t += I.sblk) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_regions<DIM, 2, 1>(o, n, I.bc, Vk, [&](int i, TV v) { sv[i] = sc * v; },
                                y, [&](int i, TY v) { sd[i] = dcoef(TV(v), eyre); });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += CH_BLOCK)
            sq[i] = sd[i] * sv[r1_to_r2<DIM>(i)] + e2ih2 * lap2_at_r1<DIM>(sv, i);
        __syncthreads();
        TV wv[PPT];
        size_t gv[PPT];
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            int i1;
            size_t gi;
            wv[m] = TV(0);
            gv[m] = 0;
            if (out_point<DIM>(threadIdx.x + m * CH_BLOCK, o, n, i1, gi)) {
                const TV w = ih2 * lap1_at<DIM>(sq, i1);
                if (store_w) W[gi] = w;
                wv[m] = w;
                gv[m] = gi;
            }
        }
        if (MANY) {
            // Through LDS, each thread takes PD consecutive tile-linear points
            // (x-neighbours), so a column is read with one 16-byte load per
            // thread where all are in the grid and aligned.  FP32 (PD = 4)
            // splits the columns between two thread groups, each covering the
            // whole tile.  Points outside the grid carry w = u = 0.
#pragma unroll
            for (int m = 0; m < PPT; ++m) sw[threadIdx.x + m * CH_BLOCK] = wv[m];
            __syncthreads();
            constexpr int GT = CH_BLOCK / CG;   // threads per column group
            const int grp = threadIdx.x / GT, p0 = PD * (threadIdx.x % GT);
            const int cx = p0 % TX, rr = p0 / TX, cy = rr % TY_, cz = rr / TY_;
            const int gx = o.x0 + cx, gy = o.y0 + cy, gz = o.z0 + cz;
            const bool rowin = gy < n && (DIM == 2 || gz < n);
            bool in[PD];
#pragma unroll
            for (int e = 0; e < PD; ++e) in[e] = rowin && gx + e < n;
            const size_t g0 = in[0] ? ((size_t)gz * n + gy) * n + gx : 0;
            const bool vec = in[PD - 1] && g0 % PD == 0;
            const int c2 = ((cz + (DIM == 3 ? 2 : 0)) * R2::Y + (cy + 2)) * R2::X + (cx + 2);
            double wd[PD], ud[PD];
#pragma unroll
            for (int e = 0; e < PD; ++e) {
                wd[e] = double(sw[p0 + e]);
                ud[e] = in[e] ? double(sv[c2 + e]) : 0.0;
            }
            auto loadv = [&](int i, TV (&v)[PD]) {
                const TV* col = V + (size_t)i * ldv + I.off;
                if (vec) {
                    const VT q = *reinterpret_cast<const VT*>(col + g0);
                    const TV* qe = reinterpret_cast<const TV*>(&q);
#pragma unroll
                    for (int e = 0; e < PD; ++e) v[e] = qe[e];
                } else {
#pragma unroll
                    for (int e = 0; e < PD; ++e) v[e] = in[e] ? col[g0 + e] : TV(0);
                }
            };
            {
                // four of the group's columns per wave_sum8 (two sums each);
                // the loads of the next four are in flight while this block
                // is summed
                constexpr int RB = 4;
                const int hv = wave_sum8_holder(lane);
                const int kg = (k - grp + CG - 1) / CG;   // columns grp, grp + CG, ... below k
                auto fetch = [&](int l0, TV (&v)[RB][PD]) {
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        if (l0 + r < kg) loadv(grp + CG * (l0 + r), v[r]);
                        else
#pragma unroll
                            for (int e = 0; e < PD; ++e) v[r][e] = TV(0);
                    }
                };
                TV cur[RB][PD];
                fetch(0, cur);
                for (int l0 = 0; l0 < kg; l0 += RB) {
                    TV nxt[RB][PD];
                    fetch(l0 + RB, nxt);
                    double a[8];
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        a[2 * r] = a[2 * r + 1] = 0.0;
#pragma unroll
                        for (int e = 0; e < PD; ++e) {
                            a[2 * r] += ud[e] * double(cur[r][e]);
                            a[2 * r + 1] += wd[e] * double(cur[r][e]);
                            cur[r][e] = nxt[r][e];
                        }
                    }
                    const double tot = wave_sum8(a);
                    const int l = l0 + (hv >> 1);
                    if (hv >= 0 && l < kg) {
                        const int c = grp + CG * l;
                        red[(hv & 1) ? k + c : c][wid] += tot;
                    }
                }
                double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int e = 0; e < PD; ++e) {
                    a[0] += ud[e] * ud[e];
                    a[1] += ud[e] * wd[e];
                }
                const double tot = wave_sum8(a);
                if (grp == 0 && (hv == 0 || hv == 1)) red[2 * k + hv][wid] += tot;
            }
        } else {
#pragma unroll
            for (int m = 0; m < PPT; ++m) dot += double(wv[m]) * double(V0[gv[m]]);
        }
        __syncthreads();
    }
    if (MANY) {
        for (int i = threadIdx.x; i < nrows; i += CH_BLOCK) {
            double a = red[i][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) a += red[i][w];
            pout[(size_t)i * CH_MAXB + blockIdx.x] = a;
        }
    } else {
        double x[1] = {dot};
        write_partials<1, RED_SUM>(x, pout);
    }
}

// ---------------------------------------------------------------------------
// Residual of the frozen linear problem at state z:
//     r = ghat - Ahat z = A (c(y) - d(y) z - eps^2 A z)
// With z = y this is f(y) (eq. IVP), the EE2 start vector of Fig. 3.
// Writes r to V_0 (and FP64 to fcur when write_f), optionally the FP32 copy
// of y; partials of ||r||^2 and ||A c(y)||^2 = ||ghat||^2 (eq. tol_phi).
// MOB: the outer operator is A_M(y) (variable mobility, Section 2, Remark 1;
// 2-D single grids).
// ---------------------------------------------------------------------------
template <int DIM, typename TV, bool SINGLE, bool MOB = false>
__global__ __launch_bounds__(CH_BLOCK) void k_resid(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                    const int* __restrict__ sb2i, const Inst inst0, int ninst, const double* __restrict__ ybase,
                                                    const double* __restrict__ zbase, double* __restrict__ fbase,
                                                    TV* __restrict__ V0base, float* __restrict__ y32base,
                                                    double* __restrict__ pout) {
    const Inst I = SINGLE ? inst0 : insts[sb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    __shared__ double sz[R2::SIZE];
    __shared__ double sdq[R1::SIZE];   // d(y), then the inner expression
    __shared__ double sc[R1::SIZE];
    __shared__ double sm[MOB ? R1::SIZE : 1];
    const double* y = ybase + I.off;
    const double* z = zbase + I.off;
    double* fout = fbase ? fbase + I.off : nullptr;
    TV* V0 = V0base + I.off;
    float* y32 = y32base ? y32base + I.off : nullptr;
    const int n = I.n, eyre = I.eyre;
    const double inv_h2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    const int lb = blockIdx.x - I.sblk0;
    double acc_r = 0.0, acc_g = 0.0;
    for (int t = xcd_remap(lb, I.sblk); t < nt; t += I.sblk) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_regions<DIM, 2, 1>(o, n, I.bc, z, [&](int i, double v) { sz[i] = v; }, y, [&](int i, double v) {
            sdq[i] = dcoef(v, eyre);
            sc[i] = ccoef(v, eyre);
            if constexpr (MOB) sm[i] = mobility_of(v, ctl->mob0, ctl->mob1);
        });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += CH_BLOCK)
            sdq[i] = sdq[i] * sz[r1_to_r2<DIM>(i)] + e2ih2 * lap2_at_r1<DIM>(sz, i) - sc[i];
        __syncthreads();
        for (int i = threadIdx.x; i < tile_points<DIM>(); i += CH_BLOCK) {
            int i1;
            size_t gi;
            if (out_point<DIM>(i, o, n, i1, gi)) {
                double r, g;
                if constexpr (MOB) {
                    r = -inv_h2 * lap1m_at(sdq, sm, i1);
                    g = inv_h2 * lap1m_at(sc, sm, i1);
                } else {
                    r = -inv_h2 * lap1_at<DIM>(sdq, i1);
                    g = inv_h2 * lap1_at<DIM>(sc, i1);
                }
                V0[gi] = TV(r);
                if (fout) fout[gi] = r;
                if (y32) y32[gi] = float(y[gi]);
                acc_r += r * r;
                acc_g += g * g;
            }
        }
        __syncthreads();
    }
    double x[2] = {acc_r, acc_g};
    write_partials<2, RED_SUM>(x, pout);
}

// ---------------------------------------------------------------------------
// LIM estimate (Fig. 2; eq. LIMest):
//   y_PC = y^n - tau/2 A (F'(y^n) + F'(y^{n+1}) + eps^2 A (y^n + y^{n+1}));
// partials of ||y^{n+1} - y_PC||^2 and ||y_PC||^2 go to the controller.
// MOB: y_PC = y^n + tau/2 (f(y^n) + f(y^{n+1})) with the variable-mobility
// right-hand side f(y) = -A_M(y) (F'(y) + eps^2 A y), whose outer operator
// differs between the two states (2-D single grids).
// ---------------------------------------------------------------------------
template <int DIM, bool SINGLE, bool MOB = false>
__global__ __launch_bounds__(CH_BLOCK) void k_est_lim(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                      const int* __restrict__ sb2i, const Inst inst0, int ninst, const double* __restrict__ y0base,
                                                      const double* __restrict__ y1base, double* __restrict__ pout) {
    const Inst I = SINGLE ? inst0 : insts[sb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    __shared__ double s0[R2::SIZE];
    __shared__ double s1[R2::SIZE];
    __shared__ double sq[R1::SIZE];
    __shared__ double sq1[MOB ? R1::SIZE : 1];
    __shared__ double sm0[MOB ? R1::SIZE : 1];
    __shared__ double sm1[MOB ? R1::SIZE : 1];
    const double* y0 = y0base + I.off;
    const double* y1 = y1base + I.off;
    const int n = I.n;
    const double inv_h2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    const double tau = ctl->tau0;
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    const int lb = blockIdx.x - I.sblk0;
    double a_err = 0.0, a_pc = 0.0;
    for (int t = xcd_remap(lb, I.sblk); t < nt; t += I.sblk) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_regions<DIM, 2, 2>(o, n, I.bc, y0, [&](int i, double v) { s0[i] = v; }, y1, [&](int i, double v) { s1[i] = v; });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += CH_BLOCK) {
            const int c = r1_to_r2<DIM>(i);
            const double a = s0[c], b = s1[c];
            if constexpr (MOB) {
                sq[i] = a * (a * a - 1.0) + e2ih2 * lap2_at_r1<DIM>(s0, i);
                sq1[i] = b * (b * b - 1.0) + e2ih2 * lap2_at_r1<DIM>(s1, i);
                sm0[i] = mobility_of(a, ctl->mob0, ctl->mob1);
                sm1[i] = mobility_of(b, ctl->mob0, ctl->mob1);
            } else {
                sq[i] = a * (a * a - 1.0) + b * (b * b - 1.0) +
                        e2ih2 * (lap2_at_r1<DIM>(s0, i) + lap2_at_r1<DIM>(s1, i));
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < tile_points<DIM>(); i += CH_BLOCK) {
            int i1;
            size_t gi;
            if (out_point<DIM>(i, o, n, i1, gi)) {
                const int c = r1_to_r2<DIM>(i1);
                double ypc;
                if constexpr (MOB)
                    ypc = s0[c] - 0.5 * tau * inv_h2 * (lap1m_at(sq, sm0, i1) + lap1m_at(sq1, sm1, i1));
                else
                    ypc = s0[c] - 0.5 * tau * inv_h2 * lap1_at<DIM>(sq, i1);
                const double e = s1[c] - ypc;
                a_err += e * e;
                a_pc += ypc * ypc;
            }
        }
        __syncthreads();
    }
    double x[2] = {a_err, a_pc};
    write_partials<2, RED_SUM>(x, pout);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define SARGS dim3(t.sgrid), dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.sb2i, t.hinst[0], t.ninst

template <int DIM, typename TV, typename TY, int DM>
static void launch_matvec_k(const Table& t, const DevBuffers& b, const TY* y, int k, int store_w, double* pout,
                            bool timing, hipStream_t s) {
    TV* V = static_cast<TV*>(b.V);
    if (timing)
        hipLaunchKernelGGL((k_matvec<DIM, TV, TY, true, DM, 1>), SARGS, V, b.ldv, k, store_w, y, pout);
    else if (t.ninst == 1)
        hipLaunchKernelGGL((k_matvec<DIM, TV, TY, true, DM, 0>), SARGS, V, b.ldv, k, store_w, y, pout);
    else
        hipLaunchKernelGGL((k_matvec<DIM, TV, TY, false, DM, 0>), SARGS, V, b.ldv, k, store_w, y, pout);
}

// FP64 basis: FP64 state; FP32 basis: the FP32 copy of the state.
template <int DIM, typename TV>
static hipError_t launch_matvec_t(const Table& t, const DevBuffers& b, PartSeq& ps, const void* y, int k,
                                  int dots, bool store_w, bool timing, hipStream_t s) {
    using TY = TV;
    const TY* yy = static_cast<const TY*>(y);
    const int sw = store_w ? 1 : 0;
    if (dots == MV_DOTS_DC) {
        launch_matvec_k<DIM, TV, TY, DM_DC>(t, b, yy, k, sw, b.dots, timing, s);
    } else {
        launch_matvec_k<DIM, TV, TY, DM_ONE>(t, b, yy, k, sw, ps.out(), false, s);
        ps.produced(PK_TILE);
    }
    return hipGetLastError();
}

hipError_t launch_matvec(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int k,
                         int dots, bool store_w, hipStream_t s, bool timing) {
    if (t.dim == 3 && dots == MV_DOTS_DC) return launch_matvec_march(t, prec, b, y, k, store_w, b.dots, timing, s);
    if (uses_strips(t)) {
        if (dots == MV_DOTS_DC) return launch_matvec_strip(t, prec, b, y, k, dots, store_w, b.dots, timing, s);
        const hipError_t e = launch_matvec_strip(t, prec, b, y, k, dots, store_w, ps.out(), false, s);
        ps.produced(PK_STRIP);
        return e;
    }
    if (prec == CH_FP64)
        return t.dim == 2 ? launch_matvec_t<2, double>(t, b, ps, y, k, dots, store_w, timing, s)
                          : launch_matvec_t<3, double>(t, b, ps, y, k, dots, store_w, timing, s);
    return t.dim == 2 ? launch_matvec_t<2, float>(t, b, ps, b.y32, k, dots, store_w, timing, s)
                      : launch_matvec_t<3, float>(t, b, ps, b.y32, k, dots, store_w, timing, s);
}

template <int DIM, typename TV>
static hipError_t launch_resid_t(const Table& t, const DevBuffers& b, PartSeq& ps, const double* y, const double* z,
                                 bool write_f, bool write_y32, hipStream_t s) {
    if (DIM == 2 && mobility(t))
        hipLaunchKernelGGL((k_resid<2, TV, true, true>), SARGS, y, z, write_f ? b.fcur : nullptr, static_cast<TV*>(b.V),
                           write_y32 ? b.y32 : nullptr, ps.out());
    else if (t.ninst == 1)
        hipLaunchKernelGGL((k_resid<DIM, TV, true>), SARGS, y, z, write_f ? b.fcur : nullptr, static_cast<TV*>(b.V),
                       write_y32 ? b.y32 : nullptr, ps.out());
    else
        hipLaunchKernelGGL((k_resid<DIM, TV, false>), SARGS, y, z, write_f ? b.fcur : nullptr, static_cast<TV*>(b.V),
                       write_y32 ? b.y32 : nullptr, ps.out());
    ps.produced(PK_TILE);
    return hipGetLastError();
}

hipError_t launch_resid(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y, const double* z,
                        bool write_f, bool write_y32, hipStream_t s) {
    if (prec == CH_FP64)
        return t.dim == 2 ? launch_resid_t<2, double>(t, b, ps, y, z, write_f, false, s)
                          : launch_resid_t<3, double>(t, b, ps, y, z, write_f, false, s);
    return t.dim == 2 ? launch_resid_t<2, float>(t, b, ps, y, z, write_f, write_y32, s)
                      : launch_resid_t<3, float>(t, b, ps, y, z, write_f, write_y32, s);
}

hipError_t launch_est_ee(const Table& t, int prec, const DevBuffers& b, PartSeq& ps, const double* y0,
                         const double* y1, hipStream_t s) {
    if (uses_strips(t)) {
        const hipError_t e = launch_est_ee_strip(t, prec, b, y0, y1, ps.out(), s);
        ps.produced(PK_STRIP);
        return e;
    }
    const hipError_t e = launch_est_march(t, prec, b, y0, y1, ps.out(), s);   // 3-D
    ps.produced(PK_STRIP);
    return e;
}

hipError_t launch_lim_stage2(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                             hipStream_t s, bool timing) {
    if (!lim_stage_pairs(t)) return hipErrorInvalidValue;
    return launch_lim_stage2_strip(t, b, yin, yout, l, timing, s);
}

hipError_t launch_lim_stage(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l, bool pairs,
                            hipStream_t s, bool timing) {
    if (uses_strips(t)) return launch_lim_stage_strip(t, b, yin, yout, l, pairs, timing, s);
    if (pairs) return hipErrorInvalidValue;
    return launch_lim_stage_march(t, b, yin, yout, l, timing, s);   // 3-D
}

hipError_t launch_est_lim(const Table& t, const DevBuffers& b, PartSeq& ps, const double* y0, const double* y1,
                          hipStream_t s) {
    if (t.dim == 2)
        if (mobility(t))
            hipLaunchKernelGGL((k_est_lim<2, true, true>), SARGS, y0, y1, ps.out());
        else if (t.ninst == 1)
            hipLaunchKernelGGL((k_est_lim<2, true>), SARGS, y0, y1, ps.out());
        else
            hipLaunchKernelGGL((k_est_lim<2, false>), SARGS, y0, y1, ps.out());
    else {   // 3-D: the marching tiles
        const hipError_t e = launch_est_lim_march(t, b, y0, y1, ps.out(), s);
        ps.produced(PK_STRIP);
        return e;
    }
    ps.produced(PK_TILE);
    return hipGetLastError();
}
