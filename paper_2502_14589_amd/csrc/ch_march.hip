// 3-D kernels on z-marching x-y tiles: the DCGS2 Jacobian matvec (below),
// the EE2 estimate pass, the LIM stage and the LIM estimate (further down,
// each with its own comment).
//
// Same operator as the tile kernels (Section 2, eq. IVP; Section 3.1,
// eqs. J, A_g; Section 3.3, eq. A_g_cs):
//     w = Ahat u = A (d u + eps^2 A u),   d = 3 y^2 - 1 (+1 Eyre),
// -A the 7-point periodic Laplacian, with the dot products of the DCGS2
// iteration (rows i < k: <u, V_i>; k + i: <w, V_i>; 2k: <u, u>; 2k + 1:
// <u, w>).
//
// Layout.  A workgroup owns an MX x MY block of (x, y) columns and a run of
// up to CH_MARCH_L planes in z (in the FP32 matvec, the length march_len_fp32
// picks for the grid), which it walks plane by plane.  Thread t owns the same
// 16 bytes of consecutive-x columns of the block in every pass (the stencil
// passes and the dot phase: two x in FP64, four in FP32), plus one column of
// the halo-1 ring around the block.  In LDS: a ring of three operand planes
// (halo 2 in x and y) and two planes of the inner expression
// q = d u + eps^2 A u (halo 1); what the stencils take from the planes above
// and below a point -- the operand and q at the point itself -- stays in the
// owning thread's registers, and so do
// d = 3 y^2 - 1 at its points and the w and u values of its dot products.  A
// plane step has one barrier: it reads one operand plane and the state at the
// thread's points (requested a step ahead), forms q on one plane and w on the
// plane below it, and runs that plane's dot phase.  An operand plane region
// is read (L + 4) / L times per run, (MX + 4)(MY + 4) / (MX MY) = 1.6 times
// the tile in FP64 (64 x 8) and 1.3 in FP32 (64 x 16), against
// (TX + 4)(TY + 4)(TZ + 4) / (TX TY TZ) = 4.5 for a 32 x 4 x 4 tile staged
// whole.
#include "ch_common.h"
#include "ch_stream.h"
#include "ch_march.h"

#include <type_traits>

namespace {

static_assert(march_rows(CH_FP64) == 8 && march_rows(CH_FP32_MIXED) == 16, "block heights of MGeo");

// x-y tile of a workgroup: MX x MY outputs per plane, NPT consecutive x per
// thread (one 16-byte vector: FP64 pairs in a 64 x 8 block, FP32 quads in a
// 64 x 16 block); the halo-1 ring of the q region is spread over the threads.
// In LDS each region row has a leading pad and a stride that put every
// thread's first point on a multiple of NPT, so its NPT values are one
// aligned access.
template <typename TV>
struct MGeo {
    static constexpr int NPT = 16 / (int)sizeof(TV);              // tile points per thread
    static constexpr int MX = 64, TXT = MX / NPT, MY = CH_BLOCK / TXT;
    static constexpr int MVX = MX + 4, MVY = MY + 4;   // operand plane region (halo 2)
    static constexpr int MQX = MX + 2, MQY = MY + 2;   // inner-expression plane region (halo 1)
    static constexpr int PV = (NPT - 2 % NPT) % NPT;   // leading pad of an operand row in LDS
    static constexpr int PQ = (NPT - 1 % NPT) % NPT;   // leading pad of a q row in LDS
    static constexpr int MVS = (MVX + PV + NPT - 1) / NPT * NPT;   // operand row stride in LDS
    static constexpr int MQS = (MQX + PQ + NPT - 1) / NPT * NPT;   // q row stride in LDS
    static constexpr int MVP = MVX * MVY, MQP = MQX * MQY;          // region points
    static constexpr int MVPS = MVY * MVS, MQPS = MQY * MQS;        // LDS plane sizes
    static constexpr int NVL = (MVP + CH_BLOCK - 1) / CH_BLOCK;   // operand values per thread and plane
    static constexpr int NRING = MQP - MX * MY;                   // halo-1 ring of the q region
    static constexpr int NRL = (NRING + CH_BLOCK - 1) / CH_BLOCK; // ring points per thread
    static constexpr int NQL = NPT + NRL;                         // q points per thread
    static_assert(TXT * MY == CH_BLOCK, "one thread per point group of the tile");
    static_assert(MVS % NPT == 0 && MQS % NPT == 0 && MVPS % NPT == 0 && MQPS % NPT == 0, "aligned LDS vectors");
};

// NPT consecutive LDS values at a multiple of NPT, as one 16-byte access.
template <typename T, int NPT>
struct alignas(16) LVec {
    T e[NPT];
};
template <typename T, int NPT>
__device__ __forceinline__ LVec<T, NPT> lds_vec(const T* p) {
    return *reinterpret_cast<const LVec<T, NPT>*>(p);
}

// Two consecutive LDS values at an even index, as one access.
template <typename T>
struct alignas(2 * sizeof(T)) LPair {
    T a, b;
};
template <typename T>
__device__ __forceinline__ LPair<T> lds_pair(const T* p) {
    return *reinterpret_cast<const LPair<T>*>(p);
}

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

// AUX: the cache-policy bits of the load (2: non-temporal).
template <typename T, int AUX = 0>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned bo) {
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, bo, 0u, AUX));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, bo, 0u, AUX));
}

// 16 bytes of consecutive values (NPT of them) as one buffer load.
template <typename T, int NPT, int AUX = 0>
__device__ __forceinline__ void bload16(__amdgpu_buffer_rsrc_t r, unsigned bo, T (&v)[NPT]) {
    static_assert(NPT * sizeof(T) == 16, "16-byte vector");
    struct P { T e[NPT]; };
    const P p = __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b128(r, bo, 0u, AUX));
#pragma unroll
    for (int e = 0; e < NPT; ++e) v[e] = p.e[e];
}

// Two consecutive values (one buffer load of 16 bytes in FP64, 8 in FP32).
template <typename T, int AUX = 0>
__device__ __forceinline__ void bload2(__amdgpu_buffer_rsrc_t r, unsigned bo, T (&v)[2]) {
    struct P { T e[2]; };
    P p;
    if constexpr (sizeof(T) == 8) p = __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b128(r, bo, 0u, AUX));
    else p = __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b64(r, bo, 0u, AUX));
    v[0] = p.e[0];
    v[1] = p.e[1];
}

template <typename T, int AUX = 0>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, unsigned bo) {
    using u32x2 = unsigned __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, bo, 0u, AUX);
    else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, bo, 0u, AUX);
}

template <typename T, int AUX = 0>
__device__ __forceinline__ void bstore2(const T (&v)[2], __amdgpu_buffer_rsrc_t r, unsigned bo) {
    struct P { T e[2]; };
    const P p{{v[0], v[1]}};
    using u32x2 = unsigned __attribute__((ext_vector_type(2)));
    using u32x4 = unsigned __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 8) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, p), r, bo, 0u, AUX);
    else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, p), r, bo, 0u, AUX);
}

template <typename T, int NPT, int AUX = 0>
__device__ __forceinline__ void bstore16(const T (&v)[NPT], __amdgpu_buffer_rsrc_t r, unsigned bo) {
    static_assert(NPT * sizeof(T) == 16, "16-byte vector");
    struct P { T e[NPT]; };
    P p;
#pragma unroll
    for (int e = 0; e < NPT; ++e) p.e[e] = v[e];
    using u32x4 = unsigned __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, p), r, bo, 0u, AUX);
}

// Work item it of an instance: x-y tile and run of planes.
struct MarchItem {
    int x0, y0, z0, zl;
};

template <int MX, int MY>
__device__ __forceinline__ MarchItem march_item(int it, int n, int len = CH_MARCH_L) {
    const int ntx = (n + MX - 1) / MX, nty = (n + MY - 1) / MY;
    const int nxy = ntx * nty;
    const int c = it / nxy, t = it - c * nxy;
    MarchItem m;
    m.x0 = (t % ntx) * MX;
    m.y0 = (t / ntx) * MY;
    m.z0 = c * len;
    m.zl = min(len, n - m.z0);
    return m;
}

// Step p of a run (operand planes p and p + 1 and q(p - 1) in LDS; in
// registers at the thread's points: the operand of plane p - 1, d(p), and
// q(p - 2), q(p - 1) at its tile pair):
//   request the first basis columns of the dot phase (FP64), then operand
//   plane p + 2 and the state of plane p + 1 at the thread's q points;
//   q(p) at the thread's q points, stored to the free q plane;
//   w(p - 1) at its tile pair from q(p - 1) in LDS and q(p - 2), q(p) in
//   registers, stored; the dot phase of plane p - 1 (its u and w values in
//   registers);
//   operand plane p + 2 into the ring slot of plane p - 1, d(p + 1) from the
//   state;                                            barrier.
// Rings: operand plane z in slot (z - z0 + 2) mod 3, q(z) in (z - z0 + 1) mod
// 2.  Operand plane p + 2 takes the slot of plane p - 1, which no thread reads
// in step p (its values at each thread's points are in registers); q(p)
// takes the buffer of q(p - 2), last read in step p - 1.
// DV: the dot-phase form -- 1: the tile pair as one vector (n even), 0: two
// scalar points, 2: chosen per instance at run time (batches).  BIGK: room
// for the dot rows of iterations k > CH_MSMALL.  NT: the basis columns are
// loaded with the streaming hint (stream_columns); NTW: w is stored with it
// (stream_store).
template <typename TV, typename TY, bool SINGLE, int TAG, int DV, bool BIGK, bool NT, bool NTW>
__global__ __launch_bounds__(CH_BLOCK) void k_matvec_m(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                       const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                       TV* __restrict__ V, size_t ldv, int k, int store_w,
                                                       const TY* __restrict__ ybase, double* __restrict__ pout,
                                                       int zlen0) {
    using G = MGeo<TV>;
    constexpr int MX = G::MX, MY = G::MY, MVX = G::MVX, MVP = G::MVP, MQX = G::MQX, MQY = G::MQY, MQS = G::MQS,
                  MQPS = G::MQPS, MVS = G::MVS, MVPS = G::MVPS, PV = G::PV, PQ = G::PQ;
    constexpr int NVL = G::NVL, NPT = G::NPT, TXT = G::TXT, NRING = G::NRING, NQL = G::NQL;
    static_assert(G::MQP == MQX * MQY, "q region");
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    constexpr int NW = CH_BLOCK / 64;
    // The operand pass runs over whole passes of the workgroup with no bounds
    // test: lanes past the region's end repeat its last point, so they load
    // and store the same value as the lane that owns it.
    __shared__ __attribute__((aligned(16))) TV sv[3][MVPS];   // operand (x, y) at y * MVS + x + PV
    __shared__ __attribute__((aligned(16))) TV sq[2][MQPS];   // q(x, y) at y * MQS + x + PQ
    __shared__ double red[BIGK ? CH_DROWS : CH_DROWS_SMALL][NW];
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
    const int ntx = (n + MX - 1) / MX, nty = (n + MY - 1) / MY;
    // planes per run: from the host for a single grid, else per instance
    const int zlen = SINGLE ? zlen0 : (sizeof(TV) == 4 ? march_len_fp32(n) : CH_MARCH_L);
    const int nitems = ntx * nty * ((n + zlen - 1) / zlen);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    constexpr int RB = 4;   // columns per wave_sum8 (two sums each)
    // the thread's q points in the q region: its tile points, then its ring point
    // (lanes past the ring's end repeat its last point)
    int qrx[NQL], qry[NQL];
    const int cx = NPT * (tid % TXT), cy = tid / TXT;
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
        qrx[e] = cx + 1 + e;
        qry[e] = cy + 1;
    }
#pragma unroll
    for (int l = NPT; l < NQL; ++l) {
        const int r = min(tid + (l - NPT) * CH_BLOCK, NRING - 1);
        if (r < MQX) {
            qrx[l] = r;
            qry[l] = 0;
        } else if (r < 2 * MQX) {
            qrx[l] = r - MQX;
            qry[l] = MQY - 1;
        } else if (r < 2 * MQX + MY) {
            qrx[l] = 0;
            qry[l] = 1 + r - 2 * MQX;
        } else {
            qrx[l] = MQX - 1;
            qry[l] = 1 + r - 2 * MQX - MY;
        }
    }
    // FP64 requests the first block of basis columns of a step before the
    // next planes (loads complete in issue order, so the dot phase then waits
    // for its columns but not for the prefetch)
    constexpr bool EARLY = sizeof(TV) == 8;
    auto items = [&](auto vec_c) {
    constexpr bool VEC = decltype(vec_c)::value;
    for (int it = lb; it < nitems; it += I.wblk) {
        const MarchItem m = march_item<MX, MY>(it, n, zlen);
        // byte offsets in a plane of the thread's operand-region values and
        // of its q points (periodic wrap; the region may extend past the
        // grid, whose outputs are masked below)
        unsigned vo[NVL], qpos[NQL];
#pragma unroll
        for (int l = 0; l < NVL; ++l) {
            const int i = min(tid + l * CH_BLOCK, MVP - 1);
            const int ry = i / MVX, rx = i - ry * MVX;
            vo[l] = (unsigned)(wrapi(m.y0 - 2 + ry, n) * n + wrapi(m.x0 - 2 + rx, n)) * ES;
        }
#pragma unroll
        for (int l = 0; l < NQL; ++l)
            qpos[l] = (unsigned)(wrapi(m.y0 - 1 + qry[l], n) * n + wrapi(m.x0 - 1 + qrx[l], n));
        // the tile pair: plane offset (MOFF outside the grid) and which
        // points are in the grid
        const int gx = m.x0 + cx, gy = m.y0 + cy;
        bool din[NPT];
        unsigned dof[NPT];
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            din[e] = gx + e < n && gy < n;
            dof[e] = din[e] ? (unsigned)(gy * n + gx + e) * ES : MOFF;
        }
        auto load_v = [&](int z, TV (&r)[NVL]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(Vk + (size_t)wrapi(z, n) * n2, pv);
#pragma unroll
            for (int l = 0; l < NVL; ++l) r[l] = bload<TV>(rs, vo[l]);
        };
        auto store_v = [&](int z, const TV (&r)[NVL]) {
            TV* d = sv[(z - m.z0 + 2) % 3];
#pragma unroll
            for (int l = 0; l < NVL; ++l) {
                const int i = min(tid + l * CH_BLOCK, MVP - 1);
                const int ry = i / MVX, rx = i - ry * MVX;
                d[ry * MVS + rx + PV] = sc * r[l];
            }
        };
        auto load_y = [&](int z, TY (&r)[NQL]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(y + (size_t)wrapi(z, n) * n2, py);
#pragma unroll
            for (int l = 0; l < NQL; ++l) r[l] = bload<TY>(rs, qpos[l] * (unsigned)sizeof(TY));
        };
        const int z0 = m.z0;
        // registers carried between steps: operand of the plane below and
        // d of the current plane at the q points; q two planes and one plane
        // below at the tile pair
        TV vm[NQL], dr[NQL], qm2[NPT], qm1[NPT];
        {
            TV a[NVL], b[NVL];
            TY yy[NQL];
            load_v(z0 - 1, a);
            load_v(z0, b);
            {
                const __amdgpu_buffer_rsrc_t rs = plane_rsrc(Vk + (size_t)wrapi(z0 - 2, n) * n2, pv);
#pragma unroll
                for (int l = 0; l < NQL; ++l) vm[l] = sc * bload<TV>(rs, qpos[l] * ES);
            }
            load_y(z0 - 1, yy);
            // the previous item's last step ended with a barrier after its
            // last reads of the rings
            store_v(z0 - 1, a);
            store_v(z0, b);
#pragma unroll
            for (int l = 0; l < NQL; ++l) dr[l] = mdcoef(TV(yy[l]), eyre);
#pragma unroll
            for (int e = 0; e < NPT; ++e) qm2[e] = qm1[e] = TV(0);
            __syncthreads();
        }
        for (int p = z0 - 1; p <= z0 + m.zl; ++p) {
            const int zo = p - 1;   // plane of this step's w
            const bool more = p + 1 <= z0 + m.zl;
            const bool dots = zo >= z0;
            // the basis columns of the dot phase (plane p - 1), in blocks of RB
            const TV* colbase = V + I.off + (size_t)(dots ? zo : z0) * n2;
            auto fetch = [&](int l0, TV (&v)[RB][NPT]) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const bool live = dots && l0 + r < k;
                    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(colbase + (size_t)(live ? l0 + r : 0) * ldv, pv);
                    if constexpr (VEC) {
                        bload16<TV, NPT, NT ? 2 : 0>(rs, live ? dof[0] : MOFF, v[r]);
                    } else {
#pragma unroll
                        for (int e = 0; e < NPT; ++e) v[r][e] = bload<TV, NT ? 2 : 0>(rs, live ? dof[e] : MOFF);
                    }
                }
            };
            TV cur[RB][NPT];
            if constexpr (EARLY) fetch(0, cur);
            TV nv[NVL];
            TY ny[NQL];
            if (more) {   // the next step's operand plane and state, in flight during this one
                load_v(p + 2, nv);
                load_y(p + 1, ny);
            }
            // q(p) at the q points, into the free q plane
            TV vc[NQL], qn[NQL];
            {
                const TV* v0 = sv[(p - z0 + 2) % 3];
                const TV* vp = sv[(p - z0 + 3) % 3];
                TV* qd = sq[(p - z0 + 1) & 1];
                {   // the tile points: every operand value as part of an aligned vector
                    const int c = (qry[0] + 1) * MVS + (qrx[0] + 1) + PV;
                    const LVec<TV, NPT> lft = lds_vec<TV, NPT>(v0 + c - NPT), mid = lds_vec<TV, NPT>(v0 + c),
                                        rgt = lds_vec<TV, NPT>(v0 + c + NPT);
                    const LVec<TV, NPT> up = lds_vec<TV, NPT>(v0 + c - MVS), dn = lds_vec<TV, NPT>(v0 + c + MVS),
                                        ab = lds_vec<TV, NPT>(vp + c);
                    LVec<TV, NPT> qv;
#pragma unroll
                    for (int e = 0; e < NPT; ++e) {
                        vc[e] = mid.e[e];
                        const TV left = e == 0 ? lft.e[NPT - 1] : mid.e[e - 1];
                        const TV right = e == NPT - 1 ? rgt.e[0] : mid.e[e + 1];
                        TV nb = (left + right) + (up.e[e] + dn.e[e]);
                        nb += vm[e] + ab.e[e];
                        qn[e] = dr[e] * vc[e] + e2ih2 * (TV(6) * vc[e] - nb);
                        qv.e[e] = qn[e];
                    }
                    *reinterpret_cast<LVec<TV, NPT>*>(qd + qry[0] * MQS + qrx[0] + PQ) = qv;
                }
#pragma unroll
                for (int l = NPT; l < NQL; ++l) {
                    const int c = (qry[l] + 1) * MVS + (qrx[l] + 1) + PV;
                    vc[l] = v0[c];
                    TV nb = (v0[c - 1] + v0[c + 1]) + (v0[c - MVS] + v0[c + MVS]);
                    nb += vm[l] + vp[c];
                    qn[l] = dr[l] * vc[l] + e2ih2 * (TV(6) * vc[l] - nb);
                    qd[qry[l] * MQS + qrx[l] + PQ] = qn[l];
                }
            }
            if (dots) {
                // w(p - 1) at the tile pair: A q from q(p - 1) in LDS (written
                // in the previous step) and q(p - 2), q(p) in registers
                const TV* qmid = sq[(p - z0) & 1];
                TV w[NPT];
                double ud[NPT], wd[NPT];
                {   // q(p - 1) of the thread's own points is in registers
                    const int c = qry[0] * MQS + qrx[0] + PQ;
                    const LVec<TV, NPT> lft = lds_vec<TV, NPT>(qmid + c - NPT), rgt = lds_vec<TV, NPT>(qmid + c + NPT);
                    const LVec<TV, NPT> up = lds_vec<TV, NPT>(qmid + c - MQS), dn = lds_vec<TV, NPT>(qmid + c + MQS);
#pragma unroll
                    for (int e = 0; e < NPT; ++e) {
                        const TV left = e == 0 ? lft.e[NPT - 1] : qm1[e - 1];
                        const TV right = e == NPT - 1 ? rgt.e[0] : qm1[e + 1];
                        TV nb = (left + right) + (up.e[e] + dn.e[e]);
                        nb += qm2[e] + qn[e];
                        w[e] = din[e] ? ih2 * (TV(6) * qm1[e] - nb) : TV(0);
                        ud[e] = din[e] ? double(vm[e]) : 0.0;
                        wd[e] = double(w[e]);
                    }
                }
                const __amdgpu_buffer_rsrc_t rw = plane_rsrc(W + (size_t)zo * n2, pv);
                if constexpr (VEC) {
                    bstore16<TV, NPT, NTW ? 2 : 0>(w, rw, store_w ? dof[0] : MOFF);
                } else {
#pragma unroll
                    for (int e = 0; e < NPT; ++e) bstore<TV, NTW ? 2 : 0>(w[e], rw, store_w ? dof[e] : MOFF);
                }
                if constexpr (!EARLY) fetch(0, cur);
                // the loads of the next four columns are in flight while this
                // block is summed
                for (int l0 = 0; l0 < k; l0 += RB) {
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
                    if (hv >= 0 && l < k) red[(hv & 1) ? k + l : l][wid] += tot;
                }
                double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int e = 0; e < NPT; ++e) {
                    a[0] += ud[e] * ud[e];
                    a[1] += ud[e] * wd[e];
                }
                const double tot = wave_sum8(a);
                if (hv == 0 || hv == 1) red[2 * k + hv][wid] += tot;
            }
            // operand plane p + 2 into the slot of plane p - 1; d(p + 1)
            if (more) {
                store_v(p + 2, nv);
#pragma unroll
                for (int l = 0; l < NQL; ++l) dr[l] = mdcoef(TV(ny[l]), eyre);
            }
#pragma unroll
            for (int l = 0; l < NQL; ++l) vm[l] = vc[l];
#pragma unroll
            for (int e = 0; e < NPT; ++e) {
                qm2[e] = qm1[e];
                qm1[e] = qn[e];
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


// ---------------------------------------------------------------------------
// 3-D estimate pass of EE2 (Fig. 4; eq. LIMest with the EE2 step in place of
// the LIM step; eqs. IVP, A_g, tol_phi) on the same z-marching tiles: at every
// point of the grid
//   f1 = f(y^{n+1}) = -A q,  q = F'(y^{n+1}) + eps^2 A y^{n+1},
//   g1 = A c,  c = 2 y^3 (+ y with the Eyre splitting)      (ghat at y^{n+1}),
//   y_PC = y^n + tau/2 (f(y^n) + f1),
// with the sums of (y^{n+1} - y_PC)^2, y_PC^2, f1^2 and g1^2 as the
// workgroup's partials.  f1 replaces f(y^n) and becomes the next start vector
// (basis column 0, in TV); the mixed form also writes the FP32 copy of
// y^{n+1}.  The operand y^{n+1} keeps a ring of four planes, so that plane p - 1
// is still there while step p forms g1 on it from c of its in-plane
// neighbours; the thread's own y of planes p - 2 .. p give c above and below.
// DV as for the matvec.
template <typename TV, bool SINGLE, int DV>
__global__ __launch_bounds__(CH_BLOCK) void k_est_m(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                    const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                    const double* __restrict__ y0base, const double* __restrict__ y1base,
                                                    double* __restrict__ fbase, TV* __restrict__ V0base,
                                                    float* __restrict__ y32base, double* __restrict__ pout, int zlen0) {
    using G = MGeo<double>;
    constexpr int MX = G::MX, MY = G::MY, MVX = G::MVX, MVP = G::MVP, MQX = G::MQX, MQY = G::MQY, MQS = G::MQS,
                  MQPS = G::MQPS;
    constexpr int NVL = G::NVL, NPT = G::NPT, TXT = G::TXT, NRING = G::NRING, NQL = G::NQL;
    static_assert(NPT == 2 && G::MVS == MVX && G::PV == 0 && G::PQ == 1 && G::MVPS == MVP, "FP64 pair layout");
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    __shared__ __attribute__((aligned(16))) double sv[4][MVP];
    __shared__ __attribute__((aligned(16))) double sq[2][MQPS];   // q(x, y) at y * MQS + x + 1
    const double* y0 = y0base + I.off;
    const double* y1 = y1base + I.off;
    double* fcur = fbase + I.off;
    TV* V0 = V0base + I.off;
    float* y32 = y32base ? y32base + I.off : nullptr;
    const int n = I.n, eyre = I.eyre;
    const size_t n2 = (size_t)n * n;
    const unsigned pb = (unsigned)n2 * 8u, pt = (unsigned)n2 * (unsigned)sizeof(TV), pf = (unsigned)n2 * 4u;
    const double ih2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    const double half_tau = 0.5 * (ctl->mode == MODE_EE ? ctl->tau_acc : ctl->tau_step);
    const int tid = threadIdx.x;
    const int ntx = (n + MX - 1) / MX, nty = (n + MY - 1) / MY;
    // planes per run: the FP32 matvec's in the mixed form (its workgroup
    // count is sized for them); from the host for a single grid
    const int zlen = SINGLE ? zlen0 : (sizeof(TV) == 4 ? march_len_fp32(n) : CH_MARCH_L);
    const int nitems = ntx * nty * ((n + zlen - 1) / zlen);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    int qrx[NQL], qry[NQL];
    const int cx = NPT * (tid % TXT), cy = tid / TXT;
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
        qrx[e] = cx + 1 + e;
        qry[e] = cy + 1;
    }
#pragma unroll
    for (int l = NPT; l < NQL; ++l) {
        const int r = min(tid + (l - NPT) * CH_BLOCK, NRING - 1);
        if (r < MQX) {
            qrx[l] = r;
            qry[l] = 0;
        } else if (r < 2 * MQX) {
            qrx[l] = r - MQX;
            qry[l] = MQY - 1;
        } else if (r < 2 * MQX + MY) {
            qrx[l] = 0;
            qry[l] = 1 + r - 2 * MQX;
        } else {
            qrx[l] = MQX - 1;
            qry[l] = 1 + r - 2 * MQX - MY;
        }
    }
    auto cc = [eyre](double v) { return 2.0 * v * v * v + (eyre ? v : 0.0); };
    double a_err = 0.0, a_pc = 0.0, a_f = 0.0, a_g = 0.0;
    auto items = [&](auto vec_c) {
    constexpr bool VEC = decltype(vec_c)::value;
    for (int it = lb; it < nitems; it += I.wblk) {
        const MarchItem m = march_item<MX, MY>(it, n, zlen);
        unsigned vo[NVL], qpos[NQL];
#pragma unroll
        for (int l = 0; l < NVL; ++l) {
            const int i = min(tid + l * CH_BLOCK, MVP - 1);
            const int ry = i / MVX, rx = i - ry * MVX;
            vo[l] = (unsigned)(wrapi(m.y0 - 2 + ry, n) * n + wrapi(m.x0 - 2 + rx, n)) * 8u;
        }
#pragma unroll
        for (int l = 0; l < NQL; ++l)
            qpos[l] = (unsigned)(wrapi(m.y0 - 1 + qry[l], n) * n + wrapi(m.x0 - 1 + qrx[l], n));
        const int gx = m.x0 + cx, gy = m.y0 + cy;
        bool din[NPT];
        unsigned pidx[NPT];   // plane index of the pair's points (MOFF / 8 outside the grid)
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            din[e] = gx + e < n && gy < n;
            pidx[e] = din[e] ? (unsigned)(gy * n + gx + e) : (MOFF >> 3);
        }
        auto load_v = [&](int z, double (&r)[NVL]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(y1 + (size_t)wrapi(z, n) * n2, pb);
#pragma unroll
            for (int l = 0; l < NVL; ++l) r[l] = bload<double>(rs, vo[l]);
        };
        auto store_v = [&](int z, const double (&r)[NVL]) {
            double* d = sv[(z - m.z0 + 2) & 3];
#pragma unroll
            for (int l = 0; l < NVL; ++l) d[min(tid + l * CH_BLOCK, MVP - 1)] = r[l];
        };
        // the pair's values of a field plane (y^n, f(y^n)): one 16-byte load, or two
        auto load_pair = [&](const double* base, int z, double (&v)[NPT]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(base + (size_t)z * n2, pb);
            if constexpr (VEC) {
                bload2<double>(rs, pidx[0] * 8u, v);
            } else {
#pragma unroll
                for (int e = 0; e < NPT; ++e) v[e] = bload<double>(rs, pidx[e] * 8u);
            }
        };
        const int z0 = m.z0;
        // carried between steps: y of the plane below at the q points, y two
        // planes below and q one and two planes below at the tile pair
        double vm[NQL], ym2[NPT], qm2[NPT], qm1[NPT];
        {
            double a[NVL], b[NVL];
            load_v(z0 - 1, a);
            load_v(z0, b);
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(y1 + (size_t)wrapi(z0 - 2, n) * n2, pb);
#pragma unroll
            for (int l = 0; l < NQL; ++l) vm[l] = bload<double>(rs, qpos[l] * 8u);
            store_v(z0 - 1, a);
            store_v(z0, b);
#pragma unroll
            for (int e = 0; e < NPT; ++e) ym2[e] = qm2[e] = qm1[e] = 0.0;
            __syncthreads();
        }
        for (int p = z0 - 1; p <= z0 + m.zl; ++p) {
            const int zo = p - 1;   // plane of this step's f1, g1 and sums
            const bool more = p + 1 <= z0 + m.zl;
            const bool outp = zo >= z0;
            double o0[NPT], of[NPT];
            if (outp) {   // y^n and f(y^n) at the pair, in flight during the q pass
                load_pair(y0, zo, o0);
                load_pair(fcur, zo, of);
            }
            double nv[NVL];
            if (more) load_v(p + 2, nv);
            double vc[NQL], qn[NQL];
            {
                const double* v0 = sv[(p - z0 + 2) & 3];
                const double* vp = sv[(p - z0 + 3) & 3];
                double* qd = sq[(p - z0 + 1) & 1];
                const int c = (qry[0] + 1) * MVX + (qrx[0] + 1);
                const LPair<double> lft = lds_pair(v0 + c - 2), mid = lds_pair(v0 + c), rgt = lds_pair(v0 + c + 2);
                const LPair<double> up = lds_pair(v0 + c - MVX), dn = lds_pair(v0 + c + MVX), ab = lds_pair(vp + c);
                vc[0] = mid.a;
                vc[1] = mid.b;
                double nb0 = (lft.b + mid.b) + (up.a + dn.a);
                double nb1 = (mid.a + rgt.a) + (up.b + dn.b);
                nb0 += vm[0] + ab.a;
                nb1 += vm[1] + ab.b;
                qn[0] = vc[0] * (vc[0] * vc[0] - 1.0) + e2ih2 * (6.0 * vc[0] - nb0);
                qn[1] = vc[1] * (vc[1] * vc[1] - 1.0) + e2ih2 * (6.0 * vc[1] - nb1);
                *reinterpret_cast<LPair<double>*>(qd + qry[0] * MQS + qrx[0] + 1) = LPair<double>{qn[0], qn[1]};
#pragma unroll
                for (int l = NPT; l < NQL; ++l) {
                    const int cr = (qry[l] + 1) * MVX + (qrx[l] + 1);
                    vc[l] = v0[cr];
                    double nb = (v0[cr - 1] + v0[cr + 1]) + (v0[cr - MVX] + v0[cr + MVX]);
                    nb += vm[l] + vp[cr];
                    qn[l] = vc[l] * (vc[l] * vc[l] - 1.0) + e2ih2 * (6.0 * vc[l] - nb);
                    qd[qry[l] * MQS + qrx[l] + 1] = qn[l];
                }
            }
            if (outp) {
                // f1 = -A q and g1 = A c on plane p - 1 at the pair
                const double* qmid = sq[(p - z0) & 1];
                const double* ym = sv[(p - z0 + 1) & 3];   // y of plane p - 1
                const int c = qry[0] * MQS + qrx[0] + 1;
                const LPair<double> lft = lds_pair(qmid + c - 2), rgt = lds_pair(qmid + c + 2);
                const LPair<double> up = lds_pair(qmid + c - MQS), dn = lds_pair(qmid + c + MQS);
                double nb[NPT] = {(lft.b + qm1[1]) + (up.a + dn.a), (qm1[0] + rgt.a) + (up.b + dn.b)};
                const int cv = (qry[0] + 1) * MVX + (qrx[0] + 1);
                const LPair<double> yl = lds_pair(ym + cv - 2), yr = lds_pair(ym + cv + 2);
                const LPair<double> yu = lds_pair(ym + cv - MVX), yd = lds_pair(ym + cv + MVX);
                const double c0 = cc(vm[0]), c1 = cc(vm[1]);
                double gb[NPT] = {(cc(yl.b) + c1) + (cc(yu.a) + cc(yd.a)), (c0 + cc(yr.a)) + (cc(yu.b) + cc(yd.b))};
                const double cown[NPT] = {c0, c1};
                double f1[NPT];
                TV ft[NPT];
                float yf[NPT];
#pragma unroll
                for (int e = 0; e < NPT; ++e) {
                    nb[e] += qm2[e] + qn[e];
                    gb[e] += cc(ym2[e]) + cc(vc[e]);
                    f1[e] = -ih2 * (6.0 * qm1[e] - nb[e]);
                    const double g1 = ih2 * (6.0 * cown[e] - gb[e]);
                    const double ypc = o0[e] + half_tau * (of[e] + f1[e]);
                    const double er = vm[e] - ypc;
                    if (din[e]) {
                        a_err += er * er;
                        a_pc += ypc * ypc;
                        a_f += f1[e] * f1[e];
                        a_g += g1 * g1;
                    }
                    ft[e] = TV(f1[e]);
                    yf[e] = float(vm[e]);
                }
                const __amdgpu_buffer_rsrc_t rf = plane_rsrc(fcur + (size_t)zo * n2, pb);
                const __amdgpu_buffer_rsrc_t rt = plane_rsrc(V0 + (size_t)zo * n2, pt);
                if constexpr (VEC) {
                    bstore2<double>(f1, rf, pidx[0] * 8u);
                    bstore2<TV>(ft, rt, pidx[0] * (unsigned)sizeof(TV));
                    if (y32) bstore2<float>(yf, plane_rsrc(y32 + (size_t)zo * n2, pf), pidx[0] * 4u);
                } else {
#pragma unroll
                    for (int e = 0; e < NPT; ++e) {
                        bstore<double>(f1[e], rf, pidx[e] * 8u);
                        bstore<TV>(ft[e], rt, pidx[e] * (unsigned)sizeof(TV));
                        if (y32) bstore<float>(yf[e], plane_rsrc(y32 + (size_t)zo * n2, pf), pidx[e] * 4u);
                    }
                }
            }
            if (more) store_v(p + 2, nv);   // into the slot of plane p - 2
#pragma unroll
            for (int e = 0; e < NPT; ++e) {
                ym2[e] = vm[e];
                qm2[e] = qm1[e];
                qm1[e] = qn[e];
            }
#pragma unroll
            for (int l = 0; l < NQL; ++l) vm[l] = vc[l];
            __syncthreads();
        }
    }
    };
    if (DV == 1 || (DV == 2 && n % NPT == 0)) items(std::true_type{});
    else items(std::false_type{});
    double x[4] = {a_err, a_pc, a_f, a_g};
    write_partials<4, RED_SUM>(x, pout);
}


// ---------------------------------------------------------------------------
// 3-D LIM stage (one iteration of Fig. 1) on the same z-marching tiles:
//   y_next = (y^n + tau a_m z + tau (ghat - Ahat z)) / (1 + tau a_m),
//   ghat - Ahat z = -A q,  q = d z + eps^2 A z - c,  d = 3 y^2 - 1 (+1),
//   c = 2 y^3 (+ y)  (eqs. A_g, J; eq. A_g_cs with the Eyre splitting),
// with d and c of y^n at the thread's points.  The operand z (the previous
// stage; y^n for the first) keeps a ring of three planes, q two planes, as in
// the matvec.  (tau a_m, 1 / (1 + tau a_m)) of the launch's stage position
// come from the plan launch; launches past the instance's 2p - 1 stages do
// nothing.
template <bool SINGLE, int TAG, int DV>
__global__ __launch_bounds__(CH_BLOCK) void k_lim_stage_m(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                          const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                          const double* __restrict__ ybase, double* youtbase,
                                                          double* zbufbase, const double* __restrict__ coefs, int l) {
    using G = MGeo<double>;
    constexpr int MX = G::MX, MY = G::MY, MVX = G::MVX, MVP = G::MVP, MQX = G::MQX, MQY = G::MQY, MQS = G::MQS,
                  MQPS = G::MQPS;
    constexpr int NVL = G::NVL, NPT = G::NPT, TXT = G::TXT, NRING = G::NRING, NQL = G::NQL;
    static_assert(NPT == 2 && G::MVS == MVX && G::PV == 0 && G::PQ == 1 && G::MVPS == MVP, "FP64 pair layout");
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    const LimLaunch L = lim_launch(ctl->p, l, false, ybase, youtbase, zbufbase);
    if (!L.live) return;
    __shared__ __attribute__((aligned(16))) double sv[3][MVP];
    __shared__ __attribute__((aligned(16))) double sq[2][MQPS];   // q(x, y) at y * MQS + x + 1
    const double* yn = ybase + I.off;
    const double* zs = L.src + I.off;
    double* out = L.dst + I.off;
    const int n = I.n, eyre = I.eyre;
    const size_t n2 = (size_t)n * n;
    const unsigned pb = (unsigned)n2 * 8u;
    const double ih2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    const double tau = ctl->tau0;
    const double* cf = coefs + ((size_t)I.slot * 2 * CH_PMAX + L.pos) * 2;
    const double ta = cf[0], inv = cf[1];
    const int tid = threadIdx.x;
    const int ntx = (n + MX - 1) / MX, nty = (n + MY - 1) / MY;
    const int nitems = ntx * nty * ((n + CH_MARCH_L - 1) / CH_MARCH_L);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    int qrx[NQL], qry[NQL];
    const int cx = NPT * (tid % TXT), cy = tid / TXT;
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
        qrx[e] = cx + 1 + e;
        qry[e] = cy + 1;
    }
#pragma unroll
    for (int m = NPT; m < NQL; ++m) {
        const int r = min(tid + (m - NPT) * CH_BLOCK, NRING - 1);
        if (r < MQX) {
            qrx[m] = r;
            qry[m] = 0;
        } else if (r < 2 * MQX) {
            qrx[m] = r - MQX;
            qry[m] = MQY - 1;
        } else if (r < 2 * MQX + MY) {
            qrx[m] = 0;
            qry[m] = 1 + r - 2 * MQX;
        } else {
            qrx[m] = MQX - 1;
            qry[m] = 1 + r - 2 * MQX - MY;
        }
    }
    auto items = [&](auto vec_c) {
    constexpr bool VEC = decltype(vec_c)::value;
    for (int it = lb; it < nitems; it += I.wblk) {
        const MarchItem m = march_item<MX, MY>(it, n);
        unsigned vo[NVL], qpos[NQL];
#pragma unroll
        for (int q = 0; q < NVL; ++q) {
            const int i = min(tid + q * CH_BLOCK, MVP - 1);
            const int ry = i / MVX, rx = i - ry * MVX;
            vo[q] = (unsigned)(wrapi(m.y0 - 2 + ry, n) * n + wrapi(m.x0 - 2 + rx, n)) * 8u;
        }
#pragma unroll
        for (int q = 0; q < NQL; ++q)
            qpos[q] = (unsigned)(wrapi(m.y0 - 1 + qry[q], n) * n + wrapi(m.x0 - 1 + qrx[q], n)) * 8u;
        const int gx = m.x0 + cx, gy = m.y0 + cy;
        unsigned dof[NPT];   // byte offsets of the pair in a plane (MOFF outside the grid)
#pragma unroll
        for (int e = 0; e < NPT; ++e) dof[e] = gx + e < n && gy < n ? (unsigned)(gy * n + gx + e) * 8u : MOFF;
        auto load_v = [&](int z, double (&r)[NVL]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(zs + (size_t)wrapi(z, n) * n2, pb);
#pragma unroll
            for (int q = 0; q < NVL; ++q) r[q] = bload<double>(rs, vo[q]);
        };
        auto store_v = [&](int z, const double (&r)[NVL]) {
            double* d = sv[(z - m.z0 + 2) % 3];
#pragma unroll
            for (int q = 0; q < NVL; ++q) d[min(tid + q * CH_BLOCK, MVP - 1)] = r[q];
        };
        auto load_y = [&](int z, double (&r)[NQL]) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(yn + (size_t)wrapi(z, n) * n2, pb);
#pragma unroll
            for (int q = 0; q < NQL; ++q) r[q] = bload<double>(rs, qpos[q]);
        };
        const int z0 = m.z0;
        // carried between steps: z of the plane below and d, c of the current
        // plane at the q points; y^n of the current plane and of the plane
        // below and q one and two planes below at the tile pair
        double vm[NQL], dr[NQL], cr[NQL], yp[NPT], ym[NPT], qm2[NPT], qm1[NPT];
        {
            double a[NVL], b[NVL], yy[NQL];
            load_v(z0 - 1, a);
            load_v(z0, b);
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(zs + (size_t)wrapi(z0 - 2, n) * n2, pb);
#pragma unroll
            for (int q = 0; q < NQL; ++q) vm[q] = bload<double>(rs, qpos[q]);
            load_y(z0 - 1, yy);
            store_v(z0 - 1, a);
            store_v(z0, b);
#pragma unroll
            for (int q = 0; q < NQL; ++q) {
                dr[q] = 3.0 * yy[q] * yy[q] - 1.0 + double(eyre);
                cr[q] = 2.0 * yy[q] * yy[q] * yy[q] + (eyre ? yy[q] : 0.0);
            }
#pragma unroll
            for (int e = 0; e < NPT; ++e) {
                yp[e] = yy[e];
                ym[e] = qm2[e] = qm1[e] = 0.0;
            }
            __syncthreads();
        }
        for (int p = z0 - 1; p <= z0 + m.zl; ++p) {
            const int zo = p - 1;
            const bool more = p + 1 <= z0 + m.zl;
            double nv[NVL], ny[NQL];
            if (more) {   // the next step's operand plane and state, in flight during this one
                load_v(p + 2, nv);
                load_y(p + 1, ny);
            }
            double vc[NQL], qn[NQL];
            {
                const double* v0 = sv[(p - z0 + 2) % 3];
                const double* vp = sv[(p - z0 + 3) % 3];
                double* qd = sq[(p - z0 + 1) & 1];
                const int c = (qry[0] + 1) * MVX + (qrx[0] + 1);
                const LPair<double> lft = lds_pair(v0 + c - 2), mid = lds_pair(v0 + c), rgt = lds_pair(v0 + c + 2);
                const LPair<double> up = lds_pair(v0 + c - MVX), dn = lds_pair(v0 + c + MVX), ab = lds_pair(vp + c);
                vc[0] = mid.a;
                vc[1] = mid.b;
                double nb0 = (lft.b + mid.b) + (up.a + dn.a);
                double nb1 = (mid.a + rgt.a) + (up.b + dn.b);
                nb0 += vm[0] + ab.a;
                nb1 += vm[1] + ab.b;
                qn[0] = dr[0] * vc[0] + e2ih2 * (6.0 * vc[0] - nb0) - cr[0];
                qn[1] = dr[1] * vc[1] + e2ih2 * (6.0 * vc[1] - nb1) - cr[1];
                *reinterpret_cast<LPair<double>*>(qd + qry[0] * MQS + qrx[0] + 1) = LPair<double>{qn[0], qn[1]};
#pragma unroll
                for (int q = NPT; q < NQL; ++q) {
                    const int cc = (qry[q] + 1) * MVX + (qrx[q] + 1);
                    vc[q] = v0[cc];
                    double nb = (v0[cc - 1] + v0[cc + 1]) + (v0[cc - MVX] + v0[cc + MVX]);
                    nb += vm[q] + vp[cc];
                    qn[q] = dr[q] * vc[q] + e2ih2 * (6.0 * vc[q] - nb) - cr[q];
                    qd[qry[q] * MQS + qrx[q] + 1] = qn[q];
                }
            }
            if (zo >= z0) {   // the stage on plane p - 1 at the pair
                const double* qmid = sq[(p - z0) & 1];
                const int c = qry[0] * MQS + qrx[0] + 1;
                const LPair<double> lft = lds_pair(qmid + c - 2), rgt = lds_pair(qmid + c + 2);
                const LPair<double> up = lds_pair(qmid + c - MQS), dn = lds_pair(qmid + c + MQS);
                double nb[NPT] = {(lft.b + qm1[1]) + (up.a + dn.a), (qm1[0] + rgt.a) + (up.b + dn.b)};
                double o[NPT];
#pragma unroll
                for (int e = 0; e < NPT; ++e) {
                    nb[e] += qm2[e] + qn[e];
                    const double r = -ih2 * (6.0 * qm1[e] - nb[e]);
                    o[e] = (ym[e] + ta * vm[e] + tau * r) * inv;
                }
                const __amdgpu_buffer_rsrc_t ro = plane_rsrc(out + (size_t)zo * n2, pb);
                if constexpr (VEC) {
                    bstore2<double>(o, ro, dof[0]);
                } else {
#pragma unroll
                    for (int e = 0; e < NPT; ++e) bstore<double>(o[e], ro, dof[e]);
                }
            }
            // y^n of plane p at the pair serves the stage on plane p next step
#pragma unroll
            for (int e = 0; e < NPT; ++e) ym[e] = yp[e];
            if (more) {
                store_v(p + 2, nv);
#pragma unroll
                for (int q = 0; q < NQL; ++q) {
                    dr[q] = 3.0 * ny[q] * ny[q] - 1.0 + double(eyre);
                    cr[q] = 2.0 * ny[q] * ny[q] * ny[q] + (eyre ? ny[q] : 0.0);
                }
#pragma unroll
                for (int e = 0; e < NPT; ++e) yp[e] = ny[e];
            }
#pragma unroll
            for (int e = 0; e < NPT; ++e) {
                qm2[e] = qm1[e];
                qm1[e] = qn[e];
            }
#pragma unroll
            for (int q = 0; q < NQL; ++q) vm[q] = vc[q];
            __syncthreads();
        }
    }
    };
    if (DV == 1 || (DV == 2 && n % NPT == 0)) items(std::true_type{});
    else items(std::false_type{});
}


// ---------------------------------------------------------------------------
// 3-D LIM estimate (Fig. 2; eq. LIMest) on the same z-marching tiles:
//   y_PC = y^n - tau/2 A (F'(y^n) + F'(y^{n+1}) + eps^2 A (y^n + y^{n+1})),
// partials of ||y^{n+1} - y_PC||^2 and ||y_PC||^2.  A is linear, so the
// operand ring holds s = y^n + y^{n+1}; the two states themselves are loaded
// at the thread's points for the cubic terms and the sums.
template <bool SINGLE, int DV>
__global__ __launch_bounds__(CH_BLOCK) void k_est_lim_m(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                        const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                        const double* __restrict__ y0base,
                                                        const double* __restrict__ y1base, double* __restrict__ pout) {
    using G = MGeo<double>;
    constexpr int MX = G::MX, MY = G::MY, MVX = G::MVX, MVP = G::MVP, MQX = G::MQX, MQY = G::MQY, MQS = G::MQS,
                  MQPS = G::MQPS;
    constexpr int NVL = G::NVL, NPT = G::NPT, TXT = G::TXT, NRING = G::NRING, NQL = G::NQL;
    static_assert(NPT == 2 && G::MVS == MVX && G::PV == 0 && G::PQ == 1 && G::MVPS == MVP, "FP64 pair layout");
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    __shared__ __attribute__((aligned(16))) double sv[3][MVP];
    __shared__ __attribute__((aligned(16))) double sq[2][MQPS];   // q(x, y) at y * MQS + x + 1
    const double* ya = y0base + I.off;
    const double* yb = y1base + I.off;
    const int n = I.n;
    const size_t n2 = (size_t)n * n;
    const unsigned pb = (unsigned)n2 * 8u;
    const double ih2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    const double half_tau = 0.5 * ctl->tau0;
    const int tid = threadIdx.x;
    const int ntx = (n + MX - 1) / MX, nty = (n + MY - 1) / MY;
    const int nitems = ntx * nty * ((n + CH_MARCH_L - 1) / CH_MARCH_L);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    int qrx[NQL], qry[NQL];
    const int cx = NPT * (tid % TXT), cy = tid / TXT;
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
        qrx[e] = cx + 1 + e;
        qry[e] = cy + 1;
    }
#pragma unroll
    for (int m = NPT; m < NQL; ++m) {
        const int r = min(tid + (m - NPT) * CH_BLOCK, NRING - 1);
        if (r < MQX) {
            qrx[m] = r;
            qry[m] = 0;
        } else if (r < 2 * MQX) {
            qrx[m] = r - MQX;
            qry[m] = MQY - 1;
        } else if (r < 2 * MQX + MY) {
            qrx[m] = 0;
            qry[m] = 1 + r - 2 * MQX;
        } else {
            qrx[m] = MQX - 1;
            qry[m] = 1 + r - 2 * MQX - MY;
        }
    }
    double a_err = 0.0, a_pc = 0.0;
    auto items = [&](auto vec_c) {
    constexpr bool VEC = decltype(vec_c)::value;
    (void)VEC;
    for (int it = lb; it < nitems; it += I.wblk) {
        const MarchItem m = march_item<MX, MY>(it, n);
        unsigned vo[NVL], qpos[NQL];
#pragma unroll
        for (int q = 0; q < NVL; ++q) {
            const int i = min(tid + q * CH_BLOCK, MVP - 1);
            const int ry = i / MVX, rx = i - ry * MVX;
            vo[q] = (unsigned)(wrapi(m.y0 - 2 + ry, n) * n + wrapi(m.x0 - 2 + rx, n)) * 8u;
        }
#pragma unroll
        for (int q = 0; q < NQL; ++q)
            qpos[q] = (unsigned)(wrapi(m.y0 - 1 + qry[q], n) * n + wrapi(m.x0 - 1 + qrx[q], n)) * 8u;
        const int gx = m.x0 + cx, gy = m.y0 + cy;
        bool din[NPT];
#pragma unroll
        for (int e = 0; e < NPT; ++e) din[e] = gx + e < n && gy < n;
        // s = y^n + y^{n+1} over the operand region of plane z
        auto load_s = [&](int z, double (&r)[NVL]) {
            const __amdgpu_buffer_rsrc_t ra = plane_rsrc(ya + (size_t)wrapi(z, n) * n2, pb);
            const __amdgpu_buffer_rsrc_t rb = plane_rsrc(yb + (size_t)wrapi(z, n) * n2, pb);
            double t[NVL];
#pragma unroll
            for (int q = 0; q < NVL; ++q) {
                r[q] = bload<double>(ra, vo[q]);
                t[q] = bload<double>(rb, vo[q]);
            }
#pragma unroll
            for (int q = 0; q < NVL; ++q) r[q] += t[q];
        };
        auto store_s = [&](int z, const double (&r)[NVL]) {
            double* d = sv[(z - m.z0 + 2) % 3];
#pragma unroll
            for (int q = 0; q < NVL; ++q) d[min(tid + q * CH_BLOCK, MVP - 1)] = r[q];
        };
        // both states at the q points of plane z
        auto load_ab = [&](int z, double (&a)[NQL], double (&b)[NQL]) {
            const __amdgpu_buffer_rsrc_t ra = plane_rsrc(ya + (size_t)wrapi(z, n) * n2, pb);
            const __amdgpu_buffer_rsrc_t rb = plane_rsrc(yb + (size_t)wrapi(z, n) * n2, pb);
#pragma unroll
            for (int q = 0; q < NQL; ++q) {
                a[q] = bload<double>(ra, qpos[q]);
                b[q] = bload<double>(rb, qpos[q]);
            }
        };
        const int z0 = m.z0;
        // carried: s of the plane below at the q points; F'(y^n) + F'(y^{n+1})
        // of the current plane at the q points; both states of the plane
        // below at the pair; q one and two planes below at the pair
        double sm[NQL], fr[NQL], am[NPT], bm[NPT], ap[NPT], bp[NPT], qm2[NPT], qm1[NPT];
        {
            double a[NVL], b[NVL], aa[NQL], bb[NQL];
            load_s(z0 - 1, a);
            load_s(z0, b);
            {
                double ta[NQL], tb[NQL];
                load_ab(z0 - 2, ta, tb);
#pragma unroll
                for (int q = 0; q < NQL; ++q) sm[q] = ta[q] + tb[q];
            }
            load_ab(z0 - 1, aa, bb);
            store_s(z0 - 1, a);
            store_s(z0, b);
#pragma unroll
            for (int q = 0; q < NQL; ++q) fr[q] = aa[q] * (aa[q] * aa[q] - 1.0) + bb[q] * (bb[q] * bb[q] - 1.0);
#pragma unroll
            for (int e = 0; e < NPT; ++e) {
                ap[e] = aa[e];
                bp[e] = bb[e];
                am[e] = bm[e] = qm2[e] = qm1[e] = 0.0;
            }
            __syncthreads();
        }
        for (int p = z0 - 1; p <= z0 + m.zl; ++p) {
            const bool more = p + 1 <= z0 + m.zl;
            double nv[NVL], na[NQL], nb2[NQL];
            if (more) {
                load_s(p + 2, nv);
                load_ab(p + 1, na, nb2);
            }
            double vc[NQL], qn[NQL];
            {
                const double* v0 = sv[(p - z0 + 2) % 3];
                const double* vp = sv[(p - z0 + 3) % 3];
                double* qd = sq[(p - z0 + 1) & 1];
                const int c = (qry[0] + 1) * MVX + (qrx[0] + 1);
                const LPair<double> lft = lds_pair(v0 + c - 2), mid = lds_pair(v0 + c), rgt = lds_pair(v0 + c + 2);
                const LPair<double> up = lds_pair(v0 + c - MVX), dn = lds_pair(v0 + c + MVX), ab = lds_pair(vp + c);
                vc[0] = mid.a;
                vc[1] = mid.b;
                double nb0 = (lft.b + mid.b) + (up.a + dn.a);
                double nb1 = (mid.a + rgt.a) + (up.b + dn.b);
                nb0 += sm[0] + ab.a;
                nb1 += sm[1] + ab.b;
                qn[0] = fr[0] + e2ih2 * (6.0 * vc[0] - nb0);
                qn[1] = fr[1] + e2ih2 * (6.0 * vc[1] - nb1);
                *reinterpret_cast<LPair<double>*>(qd + qry[0] * MQS + qrx[0] + 1) = LPair<double>{qn[0], qn[1]};
#pragma unroll
                for (int q = NPT; q < NQL; ++q) {
                    const int cc = (qry[q] + 1) * MVX + (qrx[q] + 1);
                    vc[q] = v0[cc];
                    double nb = (v0[cc - 1] + v0[cc + 1]) + (v0[cc - MVX] + v0[cc + MVX]);
                    nb += sm[q] + vp[cc];
                    qn[q] = fr[q] + e2ih2 * (6.0 * vc[q] - nb);
                    qd[qry[q] * MQS + qrx[q] + 1] = qn[q];
                }
            }
            if (p - 1 >= z0) {   // y_PC on plane p - 1 at the pair
                const double* qmid = sq[(p - z0) & 1];
                const int c = qry[0] * MQS + qrx[0] + 1;
                const LPair<double> lft = lds_pair(qmid + c - 2), rgt = lds_pair(qmid + c + 2);
                const LPair<double> up = lds_pair(qmid + c - MQS), dn = lds_pair(qmid + c + MQS);
                double nb[NPT] = {(lft.b + qm1[1]) + (up.a + dn.a), (qm1[0] + rgt.a) + (up.b + dn.b)};
#pragma unroll
                for (int e = 0; e < NPT; ++e) {
                    nb[e] += qm2[e] + qn[e];
                    const double ypc = am[e] - half_tau * (ih2 * (6.0 * qm1[e] - nb[e]));
                    const double er = bm[e] - ypc;
                    if (din[e]) {
                        a_err += er * er;
                        a_pc += ypc * ypc;
                    }
                }
            }
            if (more) store_s(p + 2, nv);
#pragma unroll
            for (int e = 0; e < NPT; ++e) {
                am[e] = ap[e];
                bm[e] = bp[e];
                qm2[e] = qm1[e];
                qm1[e] = qn[e];
            }
            if (more) {
#pragma unroll
                for (int q = 0; q < NQL; ++q) fr[q] = na[q] * (na[q] * na[q] - 1.0) + nb2[q] * (nb2[q] * nb2[q] - 1.0);
#pragma unroll
                for (int e = 0; e < NPT; ++e) {
                    ap[e] = na[e];
                    bp[e] = nb2[e];
                }
            }
#pragma unroll
            for (int q = 0; q < NQL; ++q) sm[q] = vc[q];
            __syncthreads();
        }
    }
    };
    if (DV == 1 || (DV == 2 && n % NPT == 0)) items(std::true_type{});
    else items(std::false_type{});
    double x[2] = {a_err, a_pc};
    write_partials<2, RED_SUM>(x, pout);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------
#define MARGS dim3(t.wgrid), dim3(CH_BLOCK), 0, s, b.ctl, t.inst, t.wb2i, t.hinst[0], t.ninst

template <typename TV, typename TY, bool NT, bool NTW>
static void launch_matvec_m(const Table& t, const DevBuffers& b, const TY* y, int k, int store_w, double* pout,
                            bool timing, hipStream_t s) {
    TV* V = static_cast<TV*>(b.V);
    const int zl = sizeof(TV) == 4 ? march_len_fp32(t.hinst[0].n) : CH_MARCH_L;   // single-grid launches
    const bool vec = t.hinst[0].n % MGeo<TV>::NPT == 0;   // the tile pair as one vector
    if (k > CH_MSMALL) {
        if (timing) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 1, 2, true, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
        else if (t.ninst == 1) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 0, 2, true, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
        else hipLaunchKernelGGL((k_matvec_m<TV, TY, false, 0, 2, true, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
    } else if (timing) {
        if (vec) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 1, 1, false, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
        else hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 1, 0, false, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
    } else if (t.ninst == 1) {
        if (vec) hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 0, 1, false, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
        else hipLaunchKernelGGL((k_matvec_m<TV, TY, true, 0, 0, false, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
    } else {
        hipLaunchKernelGGL((k_matvec_m<TV, TY, false, 0, 2, false, NT, NTW>), MARGS, V, b.ldv, k, store_w, y, pout, zl);
    }
}

template <typename TV, typename TY>
static void launch_matvec_m(const Table& t, const DevBuffers& b, const TY* y, int k, int store_w, double* pout,
                            bool timing, hipStream_t s) {
    const bool nt = stream_columns(b.ldv, sizeof(TV), k), ntw = stream_store(b.ldv, sizeof(TV), k);
    if (nt && ntw) launch_matvec_m<TV, TY, true, true>(t, b, y, k, store_w, pout, timing, s);
    else if (nt) launch_matvec_m<TV, TY, true, false>(t, b, y, k, store_w, pout, timing, s);
    else if (ntw) launch_matvec_m<TV, TY, false, true>(t, b, y, k, store_w, pout, timing, s);
    else launch_matvec_m<TV, TY, false, false>(t, b, y, k, store_w, pout, timing, s);
}

hipError_t launch_matvec_march(const Table& t, int prec, const DevBuffers& b, const double* y, int k, bool store_w,
                               double* pout, bool timing, hipStream_t s) {
    const int sw = store_w ? 1 : 0;
    if (prec == CH_FP64) launch_matvec_m<double, double>(t, b, y, k, sw, pout, timing, s);
    else launch_matvec_m<float, float>(t, b, b.y32, k, sw, pout, timing, s);
    return hipGetLastError();
}

template <typename TV>
static void launch_est_m(const Table& t, const DevBuffers& b, const double* y0, const double* y1, float* y32,
                         double* pout, hipStream_t s) {
    TV* V0 = static_cast<TV*>(b.V);
    const int zl = sizeof(TV) == 4 ? march_len_fp32(t.hinst[0].n) : CH_MARCH_L;   // single-grid launches
    if (t.ninst == 1) {
        if (t.hinst[0].n % MGeo<double>::NPT == 0)
            hipLaunchKernelGGL((k_est_m<TV, true, 1>), MARGS, y0, y1, b.fcur, V0, y32, pout, zl);
        else
            hipLaunchKernelGGL((k_est_m<TV, true, 0>), MARGS, y0, y1, b.fcur, V0, y32, pout, zl);
    } else {
        hipLaunchKernelGGL((k_est_m<TV, false, 2>), MARGS, y0, y1, b.fcur, V0, y32, pout, zl);
    }
}

hipError_t launch_est_march(const Table& t, int prec, const DevBuffers& b, const double* y0, const double* y1,
                            double* pout, hipStream_t s) {
    if (prec == CH_FP64) launch_est_m<double>(t, b, y0, y1, nullptr, pout, s);
    else launch_est_m<float>(t, b, y0, y1, b.y32, pout, s);
    return hipGetLastError();
}

hipError_t launch_lim_stage_march(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                                  bool timing, hipStream_t s) {
    const bool vec = t.hinst[0].n % MGeo<double>::NPT == 0;
    if (timing) {
        if (vec) hipLaunchKernelGGL((k_lim_stage_m<true, 1, 1>), MARGS, yin, yout, b.zbuf, b.lcoef, l);
        else hipLaunchKernelGGL((k_lim_stage_m<true, 1, 0>), MARGS, yin, yout, b.zbuf, b.lcoef, l);
    } else if (t.ninst == 1) {
        if (vec) hipLaunchKernelGGL((k_lim_stage_m<true, 0, 1>), MARGS, yin, yout, b.zbuf, b.lcoef, l);
        else hipLaunchKernelGGL((k_lim_stage_m<true, 0, 0>), MARGS, yin, yout, b.zbuf, b.lcoef, l);
    } else {
        hipLaunchKernelGGL((k_lim_stage_m<false, 0, 2>), MARGS, yin, yout, b.zbuf, b.lcoef, l);
    }
    return hipGetLastError();
}

hipError_t launch_est_lim_march(const Table& t, const DevBuffers& b, const double* y0, const double* y1, double* pout,
                                hipStream_t s) {
    if (t.ninst == 1) hipLaunchKernelGGL((k_est_lim_m<true, 1>), MARGS, y0, y1, pout);
    else hipLaunchKernelGGL((k_est_lim_m<false, 2>), MARGS, y0, y1, pout);
    return hipGetLastError();
}
