// 3-D DCGS2 Jacobian matvec by z-marching x-y tiles.
//
// Same operator as the tile kernels (Section 2, eq. IVP; Section 3.1,
// eqs. J, A_g; Section 3.3, eq. A_g_cs):
//     w = Ahat u = A (d u + eps^2 A u),   d = 3 y^2 - 1 (+1 Eyre),
// -A the 7-point periodic Laplacian, with the dot products of the DCGS2
// iteration (rows i < k: <u, V_i>; k + i: <w, V_i>; 2k: <u, u>; 2k + 1:
// <u, w>).
//
// Layout.  A workgroup owns an MX x MY block of (x, y) columns and a run of
// up to CH_MARCH_L planes in z.  It walks the run plane by plane keeping three
// operand planes (halo 2 in x and y), two planes of d and three planes of the
// inner expression q = d u + eps^2 A u (halo 1) in LDS, as rings: each step
// reads one new operand plane and one plane of the state, forms q on one
// plane and w on the plane below it.  An operand plane region is read
// (L + 4) / L times per run, (MX + 4)(MY + 4) / (MX MY) = 1.6 times the tile,
// against (TX + 4)(TY + 4)(TZ + 4) / (TX TY TZ) = 4.5 for a 32 x 4 x 4 tile
// staged whole; the next step's loads are issued before the current step's
// arithmetic.
#include "ch_common.h"

#include <type_traits>

namespace {

// x-y tile of a workgroup: MX x MY outputs per plane, two per thread.
template <typename TV>
struct MGeo {
    static constexpr int MX = 64, MY = 8;
    static constexpr int MVX = MX + 4, MVY = MY + 4;   // operand plane region (halo 2)
    static constexpr int MQX = MX + 2, MQY = MY + 2;   // inner-expression plane region (halo 1)
    static constexpr int MVP = MVX * MVY, MQP = MQX * MQY;
    static constexpr int NVL = (MVP + CH_BLOCK - 1) / CH_BLOCK;   // operand values per thread and plane
    static constexpr int NQL = (MQP + CH_BLOCK - 1) / CH_BLOCK;   // q values per thread and plane
    static constexpr int MPTS = MX * MY;
    static constexpr int MPPT = MPTS / CH_BLOCK;
    static_assert(MPPT * CH_BLOCK == MPTS, "plane outputs per thread");
    // the q pass's reads stay in the operand plane region
    static_assert(MQY * MVX + MQX + MVX < MVP, "q pass reads");
};

template <typename T>
__device__ __forceinline__ T mdcoef(T y, int eyre) {
    return T(3) * y * y - T(1) + T(eyre);
}

// Every load and store below is branch-free: raw buffer accesses over one
// plane, where a lane that has nothing to read or write passes an offset past
// the plane (the load returns zero, the store is dropped).  Divergent branches
// around memory operations would make the compiler wait for every
// outstanding load where they join, including the prefetches.
constexpr unsigned MOFF = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned bo) {
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, bo, 0u, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, bo, 0u, 0));
}

// NPT consecutive values of 16 bytes in all (one buffer load).
template <typename T, int NPT>
__device__ __forceinline__ void bload16(__amdgpu_buffer_rsrc_t r, unsigned bo, T (&v)[NPT]) {
    static_assert(NPT * sizeof(T) == 16, "16-byte vector");
    struct P { T e[NPT]; };
    const P p = __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b128(r, bo, 0u, 0));
#pragma unroll
    for (int e = 0; e < NPT; ++e) v[e] = p.e[e];
}

template <typename T>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, unsigned bo) {
    using u32x2 = unsigned __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, bo, 0u, 0);
    else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, bo, 0u, 0);
}

// Work item it of an instance: x-y tile and run of planes.
struct MarchItem {
    int x0, y0, z0, zl;
};

template <int MX, int MY>
__device__ __forceinline__ MarchItem march_item(int it, int n) {
    const int ntx = (n + MX - 1) / MX, nty = (n + MY - 1) / MY;
    const int nxy = ntx * nty;
    const int c = it / nxy, t = it - c * nxy;
    MarchItem m;
    m.x0 = (t % ntx) * MX;
    m.y0 = (t / ntx) * MY;
    m.z0 = c * CH_MARCH_L;
    m.zl = min(CH_MARCH_L, n - m.z0);
    return m;
}

// Step p of a run (planes p - 1, p, p + 1 of the operand and d(p) in LDS):
//   issue the loads of operand plane p + 2 and state plane p + 1;
//   q(p) on the halo-1 region;                         barrier
//   w(p - 1) = A q on the tile, stored; first basis columns of the dot
//   phase issued (FP64: at the start of the step);     barrier
//   dot products of plane p - 1;
//   the loaded planes into the rings;                  barrier.
// The step's loads have its whole arithmetic to arrive, and nothing is carried
// from one step to the next in registers.  Rings: operand plane z in slot
// (z - z0 + 2) mod 3, d in (z - z0 + 1) mod 2, q in (z - z0 + 1) mod 3.
// Operand plane p + 2 takes the slot of plane p - 1, whose last reads (the q
// pass and the dot phase's operand values) come before the step's first
// barrier.
// FP32: four workgroups per CU (128 registers); FP64: three (LDS-bound).
// DV: the dot-phase form -- 1: 16-byte vectors (n a multiple of NPT), 0:
// scalar points, 2: chosen per instance at run time (batches).  BIGK: room
// for the dot rows of iterations k > CH_MSMALL (the LDS of the small form
// keeps FP64 at three workgroups per CU).
template <typename TV, typename TY, bool SINGLE, int TAG, int DV, bool BIGK>
__global__ __launch_bounds__(CH_BLOCK, sizeof(TV) == 4 ? 4 : 3) void k_matvec_m(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                       const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                       TV* __restrict__ V, size_t ldv, int k, int store_w,
                                                       const TY* __restrict__ ybase, double* __restrict__ pout) {
    using G = MGeo<TV>;
    constexpr int MX = G::MX, MY = G::MY, MVX = G::MVX, MVP = G::MVP, MQX = G::MQX, MQP = G::MQP;
    constexpr int NVL = G::NVL, NQL = G::NQL, MPTS = G::MPTS, MPPT = G::MPPT;
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    constexpr int NW = CH_BLOCK / 64;
    // The region passes run over whole passes of the workgroup with no
    // bounds test: lanes past a region's end repeat its last point, so they
    // load, compute and store the same value as the lane that owns it.
    __shared__ TV sv[3][MVP];
    __shared__ TV sd[2][MQP];
    __shared__ TV sq[3][MQP];
    __shared__ TV sw[MPTS];
    __shared__ double red[BIGK ? CH_DROWS : CH_DROWS_SMALL][NW];
    // dot phase: thread t of column group g takes plane points t + GT e, so
    // the lanes of a wave read consecutive x; the columns are split over CG
    // groups (FP32: two, FP64: one)
    constexpr int CG = sizeof(TV) == 4 ? 2 : 1;
    constexpr int GT = CH_BLOCK / CG;
    constexpr int NPT = MPTS / GT;
    static_assert(GT % 64 == 0 && (MX % 64 == 0 || 64 % MX == 0) && NPT * GT == MPTS, "dot-phase split");
    constexpr unsigned ES = sizeof(TV);
    const TV* Vk = V + (size_t)k * ldv + I.off;
    TV* W = V + (size_t)(k + 1) * ldv + I.off;
    const TY* y = ybase + I.off;
    const int n = I.n, eyre = I.eyre;
    const size_t n2 = (size_t)n * n;
    const unsigned pv = (unsigned)n2 * ES, py = (unsigned)n2 * (unsigned)sizeof(TY);   // plane bytes
    // DCGS2 keeps its columns normalised, except the start vector
    const TV sc = TV(k > 0 ? 1.0 : ctl->vscale[0]);
    const TV ih2 = TV(I.inv_h2), e2ih2 = TV(I.eps2 * I.inv_h2);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nrows = 2 * k + 2;
    for (int i = tid; i < nrows * NW; i += CH_BLOCK) red[i / NW][i % NW] = 0.0;
    const int hv = wave_sum8_holder(lane);
    // GT is a multiple of 64, so grp is wave-uniform; saying so keeps the
    // column resources in scalar registers
    const int grp = __builtin_amdgcn_readfirstlane(tid / GT), gt = tid % GT;
    const int kg = (k - grp + CG - 1) / CG;       // dot columns grp, grp + CG, ... below k
    const int ntx = (n + MX - 1) / MX, nty = (n + MY - 1) / MY;
    const int nitems = ntx * nty * ((n + CH_MARCH_L - 1) / CH_MARCH_L);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    constexpr int RB = 4;   // columns per wave_sum8 (two sums each)
    static_assert(NPT * sizeof(TV) == 16, "dot-phase points of a thread: one 16-byte vector");
    // Dot-phase points of thread gt: the NPT consecutive x of vector gt of the
    // plane tile (one 16-byte load per basis column) when n is a multiple of
    // NPT, else the scalar points gt + GT e.  Every grid of the same n takes
    // the same form, so batched and separate runs sum in the same order.
    // FP64 requests the first block of basis columns of a step before the
    // next planes (loads complete in issue order, so the dot phase then waits
    // for its columns but not for the prefetch); in FP32 that was slower (the
    // registers held across the stencil passes).
    constexpr bool EARLY = sizeof(TV) == 8;
    auto items = [&](auto vec_c) {
    constexpr bool VEC = decltype(vec_c)::value;
    for (int it = lb; it < nitems; it += I.wblk) {
        const MarchItem m = march_item<MX, MY>(it, n);
        // byte offsets in a plane of this thread's operand and state values
        // (periodic wrap; the region may extend past the grid, whose outputs
        // are masked below)
        unsigned vo[NVL], qo[NQL];
#pragma unroll
        for (int l = 0; l < NVL; ++l) {
            const int i = min(tid + l * CH_BLOCK, MVP - 1);
            const int ry = i / MVX, rx = i - ry * MVX;
            vo[l] = (unsigned)(wrapi(m.y0 - 2 + ry, n) * n + wrapi(m.x0 - 2 + rx, n)) * ES;
        }
#pragma unroll
        for (int l = 0; l < NQL; ++l) {
            const int i = min(tid + l * CH_BLOCK, MQP - 1);
            const int ry = i / MQX, rx = i - ry * MQX;
            qo[l] = (unsigned)(wrapi(m.y0 - 1 + ry, n) * n + wrapi(m.x0 - 1 + rx, n)) * (unsigned)sizeof(TY);
        }
        // this thread's dot-phase points: plane offsets (MOFF outside the
        // grid) and operand-ring indices
        unsigned dof[NPT];
        int dsv[NPT];
        bool din[NPT];
        int dsw[NPT];
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int j = VEC ? NPT * gt + e : gt + GT * e;
            dsw[e] = j;
            const int cy = j / MX, cx = j - cy * MX;
            const int gx = m.x0 + cx, gy = m.y0 + cy;
            din[e] = gx < n && gy < n;
            dof[e] = din[e] ? (unsigned)(gy * n + gx) * ES : MOFF;
            dsv[e] = (cy + 2) * MVX + (cx + 2);
        }
        auto load_v = [&](int z, TV (&r)[NVL]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(Vk + (size_t)wrapi(z, n) * n2, pv);
#pragma unroll
            for (int l = 0; l < NVL; ++l) r[l] = bload<TV>(rs, vo[l]);
        };
        auto load_y = [&](int z, TY (&r)[NQL]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(y + (size_t)wrapi(z, n) * n2, py);
#pragma unroll
            for (int l = 0; l < NQL; ++l) r[l] = bload<TY>(rs, qo[l]);
        };
        auto store_v = [&](int z, const TV (&r)[NVL]) {
            TV* d = sv[(z - m.z0 + 2) % 3];
#pragma unroll
            for (int l = 0; l < NVL; ++l) d[min(tid + l * CH_BLOCK, MVP - 1)] = sc * r[l];
        };
        auto store_d = [&](int z, const TY (&r)[NQL]) {
            TV* d = sd[(z - m.z0 + 1) & 1];
#pragma unroll
            for (int l = 0; l < NQL; ++l) d[min(tid + l * CH_BLOCK, MQP - 1)] = mdcoef(TV(r[l]), eyre);
        };
        const int z0 = m.z0;
        {
            TV a[NVL], b[NVL], c[NVL];
            TY yy[NQL];
            load_v(z0 - 2, a);
            load_v(z0 - 1, b);
            load_v(z0, c);
            load_y(z0 - 1, yy);
            __syncthreads();   // the previous item's readers of the rings are done
            store_v(z0 - 2, a);
            store_v(z0 - 1, b);
            store_v(z0, c);
            store_d(z0 - 1, yy);
            __syncthreads();
        }
        for (int p = z0 - 1; p <= z0 + m.zl; ++p) {
            const int zo = p - 1;   // plane of this step's w
            const bool more = p + 1 <= z0 + m.zl;
            // the basis columns of the dot phase (plane p - 1), in blocks of RB
            const TV* colbase = V + I.off + (size_t)(zo >= z0 ? zo : z0) * n2;
            auto fetch = [&](int l0, TV (&v)[RB][NPT]) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const bool live = zo >= z0 && l0 + r < kg;
                    const int c = live ? grp + CG * (l0 + r) : 0;
                    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(colbase + (size_t)c * ldv, pv);
                    if constexpr (VEC) {
                        bload16<TV, NPT>(rs, live ? dof[0] : MOFF, v[r]);
                    } else {
#pragma unroll
                        for (int e = 0; e < NPT; ++e) v[r][e] = bload<TV>(rs, live ? dof[e] : MOFF);
                    }
                }
            };
            TV cur[RB][NPT];
            if constexpr (EARLY) fetch(0, cur);
            TV nv[NVL];
            TY ny[NQL];
            if (more) {   // the next step's planes, in flight during this one
                load_v(p + 2, nv);
                load_y(p + 1, ny);
            }
            // q(p) on the halo-1 region
            const int qs = (p - z0 + 1) % 3;
            {
                const TV* v0 = sv[(p - z0 + 2) % 3];
                const TV* vm = sv[(p - z0 + 1) % 3];
                const TV* vp = sv[(p - z0 + 3) % 3];
                const TV* dp = sd[(p - z0 + 1) & 1];
#pragma unroll
                for (int l = 0; l < NQL; ++l) {
                    const int i = min(tid + l * CH_BLOCK, MQP - 1);
                    const int ry = i / MQX, rx = i - ry * MQX;
                    const int c = (ry + 1) * MVX + (rx + 1);
                    TV nb = (v0[c - 1] + v0[c + 1]) + (v0[c - MVX] + v0[c + MVX]);
                    nb += vm[c] + vp[c];
                    sq[qs][i] = dp[i] * v0[c] + e2ih2 * (TV(6) * v0[c] - nb);
                }
            }
            if (zo >= z0) {
                // the dot phase's operand values (plane p - 1), read before
                // the barrier after which plane p + 2 may take their slot
                const TV* um = sv[(p - z0 + 1) % 3];
                double ud[NPT];
#pragma unroll
                for (int e = 0; e < NPT; ++e) ud[e] = din[e] ? double(um[dsv[e]]) : 0.0;
                __syncthreads();
                // w(p - 1) on the tile: A q from q planes p - 2, p - 1, p
                const TV* qlo = sq[(p - z0 + 2) % 3];    // plane p - 2
                const TV* qmid = sq[(p - z0) % 3];       // plane p - 1
                const TV* qhi = sq[qs];                  // plane p
                const __amdgpu_buffer_rsrc_t rw = plane_rsrc(W + (size_t)zo * n2, pv);
#pragma unroll
                for (int mm = 0; mm < MPPT; ++mm) {
                    const int i0 = tid + mm * CH_BLOCK;
                    const int cy = i0 / MX, cx = i0 - cy * MX;
                    const int gx = m.x0 + cx, gy = m.y0 + cy;
                    const bool inb = gx < n && gy < n;
                    const int c = (cy + 1) * MQX + (cx + 1);
                    TV nb = (qmid[c - 1] + qmid[c + 1]) + (qmid[c - MQX] + qmid[c + MQX]);
                    nb += qlo[c] + qhi[c];
                    const TV w = inb ? ih2 * (TV(6) * qmid[c] - nb) : TV(0);
                    bstore<TV>(w, rw, inb && store_w ? (unsigned)(gy * n + gx) * ES : MOFF);
                    sw[i0] = w;
                }
                if constexpr (!EARLY) fetch(0, cur);   // the first basis columns, in flight during the barrier
                __syncthreads();
                double wd[NPT];
#pragma unroll
                for (int e = 0; e < NPT; ++e) wd[e] = double(sw[dsw[e]]);
                // the loads of the next four columns are in flight while this
                // block is summed
                for (int l0 = 0; l0 < kg; l0 += RB) {
                    TV nxt[RB][NPT];
                    fetch(l0 + RB, nxt);
                    double a[8];
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        a[2 * r] = a[2 * r + 1] = 0.0;
#pragma unroll
                        for (int e = 0; e < NPT; ++e) {
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
                for (int e = 0; e < NPT; ++e) {
                    a[0] += ud[e] * ud[e];
                    a[1] += ud[e] * wd[e];
                }
                const double tot = wave_sum8(a);
                if (grp == 0 && (hv == 0 || hv == 1)) red[2 * k + hv][wid] += tot;
            } else {
                __syncthreads();   // the q pass's reads of plane p - 1 are done
            }
            // the loaded planes into their slots: operand p + 2 replaces
            // p - 1, d(p + 1) replaces d(p - 1) (last read in the previous step)
            if (more) {
                store_v(p + 2, nv);
                store_d(p + 1, ny);
            }
            __syncthreads();
        }
    }
    };
    if (DV == 1 || (DV == 2 && n % NPT == 0)) items(std::true_type{});
    else items(std::false_type{});
    __syncthreads();
    for (int i = tid; i < nrows; i += CH_BLOCK) {
        double a = red[i][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) a += red[i][w];
        pout[(size_t)i * CH_MAXB + blockIdx.x] = a;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------
#define MARGS dim3(t.wgrid), dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.wb2i, t.hinst[0], t.ninst

template <typename TV, typename TY>
static void launch_matvec_m(const Table& t, const DevBuffers& b, const TY* y, int k, int store_w, double* pout,
                            bool timing, hipStream_t s) {
    TV* V = static_cast<TV*>(b.V);
    constexpr int NPT = 16 / (int)sizeof(TV);   // dot-phase points per thread
    const bool vec = t.hinst[0].n % NPT == 0;
    if (k > CH_MSMALL) {
        if (timing) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 1, 2, true>), MARGS, V, b.ldv, k, store_w, y, pout);
        else if (t.ninst == 1) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 0, 2, true>), MARGS, V, b.ldv, k, store_w, y, pout);
        else hipLaunchKernelGGL((k_matvec_m<TV, TY, false, 0, 2, true>), MARGS, V, b.ldv, k, store_w, y, pout);
    } else if (timing) {
        if (vec) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 1, 1, false>), MARGS, V, b.ldv, k, store_w, y, pout);
        else hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 1, 0, false>), MARGS, V, b.ldv, k, store_w, y, pout);
    } else if (t.ninst == 1) {
        if (vec) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 0, 1, false>), MARGS, V, b.ldv, k, store_w, y, pout);
        else hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 0, 0, false>), MARGS, V, b.ldv, k, store_w, y, pout);
    } else {
        hipLaunchKernelGGL((k_matvec_m<TV, TY, false, 0, 2, false>), MARGS, V, b.ldv, k, store_w, y, pout);
    }
}

hipError_t launch_matvec_march(const Table& t, int prec, const DevBuffers& b, const double* y, int k, bool store_w,
                               double* pout, bool timing, hipStream_t s) {
    const int sw = store_w ? 1 : 0;
    if (prec == CH_FP64) launch_matvec_m<double, double>(t, b, y, k, sw, pout, timing, s);
    else launch_matvec_m<float, float>(t, b, b.y32, k, sw, pout, timing, s);
    return hipGetLastError();
}
