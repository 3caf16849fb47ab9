// 2-D stencil kernels on row strips: the Jacobian matvec (with its
// Gram-Schmidt dot products) and the LIM stage.
//
// Same operators as the tile kernels (Section 2, eq. IVP; Section 3.1,
// eqs. J, A_g; Section 3.3, eq. A_g_cs):
//     Ahat v        = A (d v + eps^2 A v),             d = 3 y^2 - 1 (+1 Eyre)
//     ghat - Ahat z = A (c - d z - eps^2 A z),         c = 2 y^3 (+ y Eyre)
//
// Layout.  Each wave owns a strip of CH_STRIP_ROWS grid rows.  Lane L holds
// VX consecutive columns of every row it touches, so one row of an operand is
// one buffer load per lane (16 bytes for 4 FP32 or 2 FP64 values) with a
// wave-uniform row offset: no per-element address arithmetic.  The x
// neighbours of a lane's first and last column come from the adjacent lanes
// by DPP whole-wave shifts; the y neighbours are the rows above and below,
// held in registers.  The first and last CH_STRIP_HALO lanes cover the halo
// columns only, so a wave needs nothing from other waves: there is no LDS
// staging and no barrier until the final dot-product reduction.
//
// Wave w of strip workgroup b (counted from the instance's first one, XCD
// banded) takes strips 4b' + w, 4b' + w + 4 wblk, ...; strip s covers columns
// [(s % nsx) OW, + OW) and rows [(s / nsx) SR, + SR).
#include "ch_common.h"

namespace {

constexpr int SR = CH_STRIP_ROWS;

// Raw buffer resource over one grid row (wave-uniform base; lanes address it
// by byte offset; an offset past the row reads zero and drops a store).  The
// last word is the gfx9 data-format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

using u32x2 = unsigned __attribute__((ext_vector_type(2)));
using u32x4 = unsigned __attribute__((ext_vector_type(4)));

// VX consecutive values of type T at byte offset `bo` of row resource r.
template <typename T, int VX>
__device__ __forceinline__ void load_row(__amdgpu_buffer_rsrc_t r, unsigned bo, T (&v)[VX]) {
    constexpr unsigned so = 0;
    constexpr int B = VX * (int)sizeof(T);
    if constexpr (B == 4) {
        v[0] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, bo, so, 0));
    } else if constexpr (B == 8) {
        const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, bo, so, 0);
        struct P { T e[VX]; };
        const P p = __builtin_bit_cast(P, x);
#pragma unroll
        for (int e = 0; e < VX; ++e) v[e] = p.e[e];
    } else if constexpr (B == 16) {
        const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, bo, so, 0);
        struct P { T e[VX]; };
        const P p = __builtin_bit_cast(P, x);
#pragma unroll
        for (int e = 0; e < VX; ++e) v[e] = p.e[e];
    } else {
        static_assert(B == 32, "row chunk of 4, 8, 16 or 32 bytes");
        constexpr int H = VX / 2;
        T a[H], c[H];
        load_row<T, H>(r, bo, a);
        load_row<T, H>(r, bo + 16u, c);
#pragma unroll
        for (int e = 0; e < H; ++e) {
            v[e] = a[e];
            v[H + e] = c[e];
        }
    }
}

template <typename T, int VX>
__device__ __forceinline__ void store_row(__amdgpu_buffer_rsrc_t r, unsigned bo, const T (&v)[VX]) {
    constexpr unsigned so = 0;
    constexpr int B = VX * (int)sizeof(T);
    struct P { T e[VX]; };
    P p;
#pragma unroll
    for (int e = 0; e < VX; ++e) p.e[e] = v[e];
    if constexpr (B == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, p), r, bo, so, 0);
    } else if constexpr (B == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, p), r, bo, so, 0);
    } else if constexpr (B == 16) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, p), r, bo, so, 0);
    } else {
        static_assert(B == 32, "row chunk of 4, 8, 16 or 32 bytes");
        constexpr int H = VX / 2;
        T a[H], c[H];
#pragma unroll
        for (int e = 0; e < H; ++e) {
            a[e] = v[e];
            c[e] = v[H + e];
        }
        store_row<T, H>(r, bo, a);
        store_row<T, H>(r, bo + 16u, c);
    }
}

// Whole-wave DPP shifts: lane L receives lane L - 1 (from_left) or L + 1
// (from_right); the wave's end lanes receive 0 (only halo lanes read them).
enum { DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138 };

template <int CTRL>
__device__ __forceinline__ float wave_shift(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double wave_shift(double x) {
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Unscaled -Laplacian (4 c - (l + r) - (u + d)) at element e of row `c`,
// with rows `up` and `dn` above and below.  The x neighbours across the
// lane boundary arrive by DPP (xl: the left lane's last element, xr: the
// right lane's first).
template <typename T, int VX>
__device__ __forceinline__ T lap5(const T (&up)[VX], const T (&c)[VX], const T (&dn)[VX], T xl, T xr, int e) {
    const T l = e > 0 ? c[e - 1] : xl;
    const T r = e < VX - 1 ? c[e + 1] : xr;
    const T nb = (l + r) + (up[e] + dn[e]);
    return T(4) * c[e] - nb;
}

// Flux form of the variable-mobility operator (Section 2, Remark 1),
// unscaled: sum over the four neighbours k of (m_c + m_k)/2 (q_c - q_k), the
// mobilities m laid out as the values q (mxl, mxr: the lane neighbours' m).
// With m = 1 it equals lap5.
template <typename T, int VX>
__device__ __forceinline__ T lap5m(const T (&up)[VX], const T (&c)[VX], const T (&dn)[VX], T xl, T xr,
                                   const T (&mup)[VX], const T (&mc)[VX], const T (&mdn)[VX], T mxl, T mxr, int e) {
    const T l = e > 0 ? c[e - 1] : xl, r = e < VX - 1 ? c[e + 1] : xr;
    const T ml = e > 0 ? mc[e - 1] : mxl, mr = e < VX - 1 ? mc[e + 1] : mxr;
    const T q = c[e], m = mc[e];
    const T fx = (m + ml) * (q - l) + (m + mr) * (q - r);
    const T fy = (m + mup[e]) * (q - up[e]) + (m + mdn[e]) * (q - dn[e]);
    return T(0.5) * (fx + fy);
}

// The outer operator at element e of row c: A (MOB false) or A_M (MOB true,
// mobility rows m), both unscaled.
template <bool MOB, typename T, int VX>
__device__ __forceinline__ T outer_op(const T (&up)[VX], const T (&c)[VX], const T (&dn)[VX], T xl, T xr,
                                      const T (&mup)[VX], const T (&mc)[VX], const T (&mdn)[VX], T mxl, T mxr, int e) {
    if constexpr (MOB) return lap5m<T, VX>(up, c, dn, xl, xr, mup, mc, mdn, mxl, mxr, e);
    else return lap5<T, VX>(up, c, dn, xl, xr, e);
}

// Mobility coefficients (from the control block) of a MOB launch.
struct Mob {
    double m0, m1;
};
__device__ __forceinline__ Mob mob_of(const Ctl* ctl, bool on) { return on ? Mob{ctl->mob0, ctl->mob1} : Mob{0.0, 0.0}; }

// Mobility rows of a block of state rows (MOB), or nothing.
template <bool MOB, typename T, int VX, int NR>
struct MobRows {
    T m[MOB ? NR : 1][VX];
    __device__ __forceinline__ void set(int j, const T (&y)[VX], T m0, T m1) {
        if constexpr (MOB) {
#pragma unroll
            for (int e = 0; e < VX; ++e) m[j][e] = mobility_of(y[e], m0, m1);
        }
    }
    __device__ __forceinline__ const T (&row(int j) const)[VX] { return m[MOB ? j : 0]; }
    __device__ __forceinline__ T left(int j) const {
        if constexpr (MOB) return wave_shift<DPP_WAVE_SHR1>(m[j][VX - 1]);
        else return T(0);
    }
    __device__ __forceinline__ T right(int j) const {
        if constexpr (MOB) return wave_shift<DPP_WAVE_SHL1>(m[j][0]);
        else return T(0);
    }
};

template <typename T>
__device__ __forceinline__ T dcoef(T y, int eyre) {
    return T(3) * y * y - T(1) + T(eyre);
}
template <typename T>
__device__ __forceinline__ T ccoef(T y, int eyre) {
    return T(2) * y * y * y + (eyre ? y : T(0));
}

// Strip geometry of one wave.
template <int VX>
struct StripPos {
    int r0;         // first row
    int xl;         // lane's first column, in [0, n)
    bool out;       // the lane's columns are outputs of this strip
    bool need;      // ... or the halo of one
    bool rev;       // the lane's values are those of its columns in reverse (Neumann mirror)
};

// Grid column of the first of the VX columns [c, c + VX) of a lane (c a
// multiple of VX, VX dividing n, -n < c < 2n): periodic wrap, or, past a
// Neumann boundary, the mirror chunk [-c - VX, -c) or [2n - c - VX, 2n - c),
// whose values the lane then takes in reverse order (rev).
template <int VX>
__device__ __forceinline__ int chunk_col(int c, int n, int bc, bool& rev) {
    rev = false;
    if (bc == CH_BC_NEUMANN && (c < 0 || c >= n)) {
        rev = VX > 1;
        const int x = c < 0 ? -c - VX : 2 * n - c - VX;
        return x < 0 ? 0 : x;   // lanes past the halo (never read) stay in bounds
    }
    const int x = c % n;
    return x < 0 ? x + n : x;
}

// Reverse the VX values of a lane when `rev`, without a branch.
template <typename T, int VX>
__device__ __forceinline__ void flip_if(bool rev, T (&v)[VX]) {
    if constexpr (VX > 1) {
        T t[VX];
#pragma unroll
        for (int e = 0; e < VX; ++e) t[e] = v[VX - 1 - e];
#pragma unroll
        for (int e = 0; e < VX; ++e) v[e] = rev ? t[e] : v[e];
    }
}

// A lane offset past every row: the load returns zeros without a memory
// access (lanes that neither own nor border an output column).
constexpr unsigned OFF_ROW = 0x80000000u;

template <int VX>
__device__ __forceinline__ StripPos<VX> strip_pos(int s, int nsx, int n, int lane, int bc) {
    constexpr int HL = CH_STRIP_HALO(VX), OW = strip_cols(VX);
    StripPos<VX> p;
    const int sx = s % nsx;
    p.r0 = (s / nsx) * SR;
    const int c = sx * OW + (lane - HL) * VX;     // first column, before the boundary fold
    p.xl = chunk_col<VX>(c, n, bc, p.rev);
    p.out = lane >= HL && lane < 64 - HL && c < n;
    p.need = c < n + HL * VX;
    return p;
}

// Row r (r in [-n, 2n): periodic wrap or Neumann mirror) of an instance's
// field of n x n values of type T.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t grid_row(const T* f, int r, int n, int bc) {
    return row_rsrc(f + (size_t)bc_index(r, n, bc) * n, (unsigned)n * (unsigned)sizeof(T));
}

// ---------------------------------------------------------------------------
// w = Ahat u, u = vscale[k] V_k (the matvec of Fig. 3), stored in column k + 1
// (unless store_w is 0), with the partials of its dot products:
//   DM_ONE  <w, V_0>                                   (the first MGS dot)
//   DM_DC   rows i < k: <u, V_i>; rows k + i: <w, V_i>;
//           row 2k: <u, u>; row 2k + 1: <u, w>          (DCGS2)
// Every instance uses its own strip width (VX = I.vx), so its arithmetic and
// its partials do not depend on the other members of a batch.
// ---------------------------------------------------------------------------
enum DotMode { DM_ONE = 0, DM_DC = 1 };

template <typename TV, int DM>
struct MatvecArgs {
    TV* V;
    size_t ldv;
    int k, store_w;
    const TV* y;
};

// The strips of this wave; dot-product totals go to red[.][wv] (DM_DC) or
// are returned per lane (DM_ONE).
template <typename TV, int DM, int VX, bool NEU, bool MOB>
__device__ __forceinline__ double matvec_strips(const Inst& I, const MatvecArgs<TV, DM>& A, TV sc, int wv,
                                                double (*red)[CH_STRIP_WAVES], Mob mob) {
    constexpr int NU = SR + 4, ND = SR + 2, W = CH_STRIP_WAVES;
    const int lane = threadIdx.x & 63;
    const int n = I.n, k = A.k;
    constexpr int bc = NEU ? CH_BC_NEUMANN : CH_BC_PERIODIC;
    const TV* U = A.V + (size_t)k * A.ldv + I.off;
    TV* Wc = A.V + (size_t)(k + 1) * A.ldv + I.off;
    const TV* Y = A.y + I.off;
    const TV ih2 = TV(I.inv_h2), e2ih2 = TV(I.eps2 * I.inv_h2);
    const int eyre = I.eyre;
    const int nsx = (n + strip_cols(VX) - 1) / strip_cols(VX);
    const int ns = nsx * ((n + SR - 1) / SR);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    const int hv = wave_sum8_holder(lane);
    double one = 0.0;
    for (int s = lb * W + wv; s < ns; s += I.wblk * W) {
        const StripPos<VX> P = strip_pos<VX>(s, nsx, n, lane, bc);
        const unsigned bo = (unsigned)P.xl * (unsigned)sizeof(TV);
        const unsigned bs = P.need ? bo : OFF_ROW;   // stencil operands
        const unsigned bd = P.out ? bo : OFF_ROW;    // basis columns of the dot products
        TV u[NU][VX], d[ND][VX];
#pragma unroll
        for (int j = 0; j < NU; ++j) load_row<TV, VX>(grid_row(U, P.r0 - 2 + j, n, bc), bs, u[j]);
#pragma unroll
        for (int j = 0; j < ND; ++j) load_row<TV, VX>(grid_row(Y, P.r0 - 1 + j, n, bc), bs, d[j]);
#pragma unroll
        for (int j = 0; j < NU; ++j) flip_if<TV, VX>(P.rev, u[j]);
#pragma unroll
        for (int j = 0; j < ND; ++j) flip_if<TV, VX>(P.rev, d[j]);
#pragma unroll
        for (int j = 0; j < NU; ++j)
#pragma unroll
            for (int e = 0; e < VX; ++e) u[j][e] *= sc;
        MobRows<MOB, TV, VX, ND> mb;
#pragma unroll
        for (int j = 0; j < ND; ++j) mb.set(j, d[j], TV(mob.m0), TV(mob.m1));
#pragma unroll
        for (int j = 0; j < ND; ++j)
#pragma unroll
            for (int e = 0; e < VX; ++e) d[j][e] = dcoef(d[j][e], eyre);
        // inner expression d u + eps^2 A u on rows r0 - 1 .. r0 + SR
        TV q[ND][VX];
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const TV xl = wave_shift<DPP_WAVE_SHR1>(u[j + 1][VX - 1]), xr = wave_shift<DPP_WAVE_SHL1>(u[j + 1][0]);
#pragma unroll
            for (int e = 0; e < VX; ++e)
                q[j][e] = d[j][e] * u[j + 1][e] + e2ih2 * lap5<TV, VX>(u[j], u[j + 1], u[j + 2], xl, xr, e);
        }
        // w = A q (A_M q with mobility) on rows r0 .. r0 + SR - 1
        TV w[SR][VX];
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            const TV xl = wave_shift<DPP_WAVE_SHR1>(q[i + 1][VX - 1]), xr = wave_shift<DPP_WAVE_SHL1>(q[i + 1][0]);
            const TV ml = mb.left(i + 1), mr = mb.right(i + 1);
#pragma unroll
            for (int e = 0; e < VX; ++e)
                w[i][e] = ih2 * outer_op<MOB, TV, VX>(q[i], q[i + 1], q[i + 2], xl, xr, mb.row(i), mb.row(i + 1),
                                                      mb.row(i + 2), ml, mr, e);
        }
        bool rowin[SR];
#pragma unroll
        for (int i = 0; i < SR; ++i) rowin[i] = P.r0 + i < n;
        // stores outside the grid or of no use go past the row (dropped)
#pragma unroll
        for (int i = 0; i < SR; ++i)
            store_row<TV, VX>(grid_row(Wc, P.r0 + i, n, bc), A.store_w && P.out && rowin[i] ? bo : OFF_ROW, w[i]);
        // the strip's points (zero outside the grid), in FP64
        double ud[SR][VX], wd[SR][VX];
#pragma unroll
        for (int i = 0; i < SR; ++i)
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const bool in = P.out && rowin[i];
                ud[i][e] = in ? double(u[i + 2][e]) : 0.0;
                wd[i][e] = in ? double(w[i][e]) : 0.0;
            }
        if (DM == DM_ONE) {
            const TV* V0 = A.V + I.off;
#pragma unroll
            for (int i = 0; i < SR; ++i) {
                TV v0[VX];
                load_row<TV, VX>(grid_row(V0, P.r0 + i, n, bc), bd, v0);
#pragma unroll
                for (int e = 0; e < VX; ++e) one += wd[i][e] * double(v0[e]);
            }
        } else {
            // Columns in blocks of two through two buffers that alternate:
            // the loads of one block are in flight while the other is summed,
            // and no loaded value is copied between registers.  A column past
            // k reads zeros (an offset past the row), so the loads sit in no
            // branch; a branch around them would make the compiler wait for
            // every outstanding load where it joins.
            constexpr int RB = 2;
            auto fetch = [&](int c0, TV (&bl)[RB][SR][VX]) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int c = c0 + r;
                    const TV* Q = A.V + (size_t)(c < k ? c : 0) * A.ldv + I.off;
                    const unsigned o = c < k ? bd : OFF_ROW;
#pragma unroll
                    for (int i = 0; i < SR; ++i) load_row<TV, VX>(grid_row(Q, P.r0 + i, n, bc), o, bl[r][i]);
                }
            };
            auto sums = [&](const TV (&bl)[RB][SR][VX], double* a) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    double su = 0.0, sw = 0.0;
#pragma unroll
                    for (int i = 0; i < SR; ++i)
#pragma unroll
                        for (int e = 0; e < VX; ++e) {
                            const double qv = double(bl[r][i][e]);
                            su += ud[i][e] * qv;
                            sw += wd[i][e] * qv;
                        }
                    a[2 * r] = su;
                    a[2 * r + 1] = sw;
                }
            };
            TV ba[RB][SR][VX], bb[RB][SR][VX];
            fetch(0, ba);
            for (int c0 = 0; c0 < k; c0 += 2 * RB) {   // four columns per wave_sum8
                double a[8];
                fetch(c0 + RB, bb);
                sums(ba, a);
                fetch(c0 + 2 * RB, ba);
                sums(bb, a + 2 * RB);
                const double tot = wave_sum8(a);
                const int c = c0 + (hv >> 1);   // column of the value this lane holds
                if (hv >= 0 && c < k) red[(hv & 1) ? k + c : c][wv] += tot;
            }
            double b8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < SR; ++i)
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    b8[0] += ud[i][e] * ud[i][e];
                    b8[1] += ud[i][e] * wd[i][e];
                }
            const double tot = wave_sum8(b8);
            if (hv == 0 || hv == 1) red[2 * k + hv][wv] += tot;
        }
    }
    return one;
}

// VX: the strip width of a single-instance launch; 0: per instance (batches).
// TAG distinguishes the launches of the timing aid (same code, another symbol).
// NEU: the single grid has Neumann boundaries (batches are periodic).
template <typename TV, bool SINGLE, int DM, int TAG, int VX, bool NEU = false, bool MOB = false>
__global__ __launch_bounds__(CH_STRIP_BLOCK) void k_matvec_s(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                       const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                       TV* __restrict__ V, size_t ldv, int k, int store_w,
                                                       const TV* __restrict__ ybase, double* __restrict__ pout) {
    constexpr int W = CH_STRIP_WAVES;
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->done | ctl->halted) return;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    // DCGS2 keeps its columns normalised, except the start vector
    const TV sc = TV(DM == DM_DC && k > 0 ? 1.0 : ctl->vscale[k]);
    const int nrows = DM == DM_DC ? 2 * k + 2 : 1;
    __shared__ double red[DM == DM_DC ? CH_DROWS : 1][W];
    for (int i = lane; i < nrows; i += 64) red[i][wv] = 0.0;   // each wave clears its own column
    const MatvecArgs<TV, DM> A{V, ldv, k, store_w, ybase};
    double one;
    if constexpr (VX > 0) {
        one = matvec_strips<TV, DM, VX, NEU, MOB>(I, A, sc, wv, red, mob_of(ctl, MOB));
    } else {
        if (I.vx == 1) {
            one = matvec_strips<TV, DM, 1, false, false>(I, A, sc, wv, red, Mob{});
        } else if (sizeof(TV) == 8 || I.vx == 2) {
            one = matvec_strips<TV, DM, 2, false, false>(I, A, sc, wv, red, Mob{});
        } else {
            one = matvec_strips<TV, DM, (sizeof(TV) == 4 ? 4 : 2), false, false>(I, A, sc, wv, red, Mob{});
        }
    }
    if (DM == DM_DC) {
        __syncthreads();
        for (int i = threadIdx.x; i < nrows; i += CH_STRIP_BLOCK) {
            double t = red[i][0];
#pragma unroll
            for (int x = 1; x < W; ++x) t += red[i][x];
            pout[(size_t)i * CH_MAXB + blockIdx.x] = t;
        }
    } else {
        double x[1] = {one};
        write_partials<1, RED_SUM>(x, pout);
    }
}

// ---------------------------------------------------------------------------
// LIM stage (one iteration of Fig. 1):
//   y_next = (y^n + tau a_m z + tau (ghat - Ahat z)) / (1 + tau a_m)
// The coefficients (tau a_m, 1 / (1 + tau a_m)) of stage position `pos` come
// from the plan launch.
// ---------------------------------------------------------------------------
template <int VX, bool NEU, bool MOB>
__device__ __forceinline__ void lim_strips(const Inst& I, const double* __restrict__ ybase,
                                           const double* __restrict__ zbase, double* __restrict__ obase, double ta,
                                           double inv, double tau, int wv, Mob mob) {
    constexpr int NU = SR + 4, ND = SR + 2, W = CH_STRIP_WAVES;
    const int lane = threadIdx.x & 63;
    const int n = I.n;
    constexpr int bc = NEU ? CH_BC_NEUMANN : CH_BC_PERIODIC;
    const double* Z = zbase + I.off;
    const double* Y = ybase + I.off;
    double* O = obase + I.off;
    const double inv_h2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    const int eyre = I.eyre;
    const int nsx = (n + strip_cols(VX) - 1) / strip_cols(VX);
    const int ns = nsx * ((n + SR - 1) / SR);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    for (int s = lb * W + wv; s < ns; s += I.wblk * W) {
        const StripPos<VX> P = strip_pos<VX>(s, nsx, n, lane, bc);
        const unsigned bo = (unsigned)P.xl * 8u;
        const unsigned bs = P.need ? bo : OFF_ROW;
        double z[NU][VX], y[ND][VX];
#pragma unroll
        for (int j = 0; j < NU; ++j) load_row<double, VX>(grid_row(Z, P.r0 - 2 + j, n, bc), bs, z[j]);
#pragma unroll
        for (int j = 0; j < ND; ++j) load_row<double, VX>(grid_row(Y, P.r0 - 1 + j, n, bc), bs, y[j]);
#pragma unroll
        for (int j = 0; j < NU; ++j) flip_if<double, VX>(P.rev, z[j]);
#pragma unroll
        for (int j = 0; j < ND; ++j) flip_if<double, VX>(P.rev, y[j]);
        MobRows<MOB, double, VX, ND> mb;
#pragma unroll
        for (int j = 0; j < ND; ++j) mb.set(j, y[j], mob.m0, mob.m1);
        // inner expression d z + eps^2 A z - c on rows r0 - 1 .. r0 + SR
        double q[ND][VX];
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const double xl = wave_shift<DPP_WAVE_SHR1>(z[j + 1][VX - 1]), xr = wave_shift<DPP_WAVE_SHL1>(z[j + 1][0]);
#pragma unroll
            for (int e = 0; e < VX; ++e)
                q[j][e] = dcoef(y[j][e], eyre) * z[j + 1][e] + e2ih2 * lap5<double, VX>(z[j], z[j + 1], z[j + 2], xl, xr, e) -
                          ccoef(y[j][e], eyre);
        }
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            const double xl = wave_shift<DPP_WAVE_SHR1>(q[i + 1][VX - 1]), xr = wave_shift<DPP_WAVE_SHL1>(q[i + 1][0]);
            const double ml = mb.left(i + 1), mr = mb.right(i + 1);
            double o[VX];
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const double r = -inv_h2 * outer_op<MOB, double, VX>(q[i], q[i + 1], q[i + 2], xl, xr, mb.row(i),
                                                                    mb.row(i + 1), mb.row(i + 2), ml, mr, e);
                o[e] = (y[i + 1][e] + ta * z[i + 2][e] + tau * r) * inv;
            }
            if (P.out && P.r0 + i < n) store_row<double, VX>(grid_row(O, P.r0 + i, n, bc), bo, o);
        }
    }
}

// Stage launch l (lim_launch) of each instance: its source and destination
// follow from its own Chebyshev order.
template <bool SINGLE, int TAG, int VX, bool NEU = false, bool MOB = false>
__global__ __launch_bounds__(CH_STRIP_BLOCK) void k_lim_stage_s(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                          const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                          const double* __restrict__ ybase, double* youtbase,
                                                          double* zbufbase, const double* __restrict__ coefs, int l,
                                                          int pairs) {
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    const LimLaunch L = lim_launch(ctl->p, l, pairs != 0, ybase, youtbase, zbufbase);
    if (!L.live) return;
    const double* zbase = L.src;
    double* obase = L.dst;
    const int pos = L.pos;
    const double* cf = coefs + ((size_t)I.slot * 2 * CH_PMAX + pos) * 2;
    const double ta = cf[0], inv = cf[1], tau = ctl->tau0;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if constexpr (VX > 0) {
        lim_strips<VX, NEU, MOB>(I, ybase, zbase, obase, ta, inv, tau, wv, mob_of(ctl, MOB));
    } else {
        if (I.vx == 1) lim_strips<1, false, false>(I, ybase, zbase, obase, ta, inv, tau, wv, Mob{});
        else lim_strips<2, false, false>(I, ybase, zbase, obase, ta, inv, tau, wv, Mob{});
    }
}

// ---------------------------------------------------------------------------
// Two consecutive LIM stages (positions pos and pos + 1) in one pass: the
// first stage's result stays in registers.  A strip of LIM2_ROWS output rows
// reads z with a halo of 4 rows and 4 columns (two stencil radii) and y^n with
// a halo of 3 rows; the HBM traffic of the pair is that of one stage (read
// y^n and z, write the result).  Each point is computed with the same
// expressions as two launches of the single stage.  Two rows per strip: with
// four, the registers (192) leave two waves per SIMD and the pair is slower;
// sharing the block's rows through LDS exposes their load latency at the
// barrier and is slower too.
// ---------------------------------------------------------------------------
#ifndef CH_LIM2_ROWS
#define CH_LIM2_ROWS 2
#endif
constexpr int LIM2_ROWS = CH_LIM2_ROWS;
template <int VX>
constexpr int lim2_halo_lanes() { return VX >= 2 ? 2 : 4; }   // 4 columns
template <int VX>
constexpr int lim2_cols() { return (64 - 2 * lim2_halo_lanes<VX>()) * VX; }

// Periodic row index for any r.
__device__ __forceinline__ int wrap_row_any(int r, int n) {
    r %= n;
    return r < 0 ? r + n : r;
}

template <int VX, bool NEU, bool MOB>
__device__ __forceinline__ void lim2_strips(const Inst& I, const double* __restrict__ ybase,
                                            const double* __restrict__ zbase, double* __restrict__ obase,
                                            double ta1, double inv1, double ta2, double inv2, double tau, int wv,
                                            Mob mob) {
    constexpr int R = LIM2_ROWS, HL = lim2_halo_lanes<VX>(), OW = lim2_cols<VX>(), W = CH_STRIP_WAVES;
    constexpr int NZ = R + 8, NY = R + 6, NQ1 = R + 6, NO1 = R + 4, NQ2 = R + 2;
    const int lane = threadIdx.x & 63;
    const int n = I.n;
    const double* Z = zbase + I.off;
    const double* Y = ybase + I.off;
    double* O = obase + I.off;
    const double inv_h2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    const int eyre = I.eyre;
    const unsigned rb = (unsigned)n * 8u;
    const int nsx = (n + OW - 1) / OW;
    const int ns = nsx * ((n + R - 1) / R);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    constexpr int bc = NEU ? CH_BC_NEUMANN : CH_BC_PERIODIC;
    // rows r0 - 4 .. r0 + R + 3: periodic, or mirrored (within n of the grid for n >= 5)
    auto row = [&](int r) { return bc == CH_BC_NEUMANN ? bc_index(r, n, bc) : wrap_row_any(r, n); };
    for (int s = lb * W + wv; s < ns; s += I.wblk * W) {
        const int sx = s % nsx, r0 = (s / nsx) * R;
        const int c = sx * OW + (lane - HL) * VX;
        bool rev;
        const int xl = chunk_col<VX>(c, n, bc, rev);
        const bool out = lane >= HL && lane < 64 - HL && c < n;
        const unsigned bo = (unsigned)xl * 8u;
        const unsigned bs = c < n + HL * VX ? bo : OFF_ROW;
        // z rows r0 - 4 + j, y rows r0 - 3 + j
        double z[NZ][VX], y[NY][VX];
#pragma unroll
        for (int j = 0; j < NZ; ++j)
            load_row<double, VX>(row_rsrc(Z + (size_t)row(r0 - 4 + j) * n, rb), bs, z[j]);
#pragma unroll
        for (int j = 0; j < NY; ++j)
            load_row<double, VX>(row_rsrc(Y + (size_t)row(r0 - 3 + j) * n, rb), bs, y[j]);
#pragma unroll
        for (int j = 0; j < NZ; ++j) flip_if<double, VX>(rev, z[j]);
#pragma unroll
        for (int j = 0; j < NY; ++j) flip_if<double, VX>(rev, y[j]);
        MobRows<MOB, double, VX, NY> mb;   // mobility rows r0 - 3 + j
#pragma unroll
        for (int j = 0; j < NY; ++j) mb.set(j, y[j], mob.m0, mob.m1);
        // first stage: q1 on rows r0 - 3 + j, its result o1 on rows r0 - 2 + j
        double q1[NQ1][VX];
#pragma unroll
        for (int j = 0; j < NQ1; ++j) {
            const double xl1 = wave_shift<DPP_WAVE_SHR1>(z[j + 1][VX - 1]), xr1 = wave_shift<DPP_WAVE_SHL1>(z[j + 1][0]);
#pragma unroll
            for (int e = 0; e < VX; ++e)
                q1[j][e] = dcoef(y[j][e], eyre) * z[j + 1][e] + e2ih2 * lap5<double, VX>(z[j], z[j + 1], z[j + 2], xl1, xr1, e) -
                           ccoef(y[j][e], eyre);
        }
        double o1[NO1][VX];
#pragma unroll
        for (int j = 0; j < NO1; ++j) {
            const double xl1 = wave_shift<DPP_WAVE_SHR1>(q1[j + 1][VX - 1]), xr1 = wave_shift<DPP_WAVE_SHL1>(q1[j + 1][0]);
            const double ml = mb.left(j + 1), mr = mb.right(j + 1);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const double r = -inv_h2 * outer_op<MOB, double, VX>(q1[j], q1[j + 1], q1[j + 2], xl1, xr1, mb.row(j),
                                                                    mb.row(j + 1), mb.row(j + 2), ml, mr, e);
                o1[j][e] = (y[j + 1][e] + ta1 * z[j + 2][e] + tau * r) * inv1;
            }
        }
        // second stage: q2 on rows r0 - 1 + j, the output on rows r0 + i
        double q2[NQ2][VX];
#pragma unroll
        for (int j = 0; j < NQ2; ++j) {
            const double xl1 = wave_shift<DPP_WAVE_SHR1>(o1[j + 1][VX - 1]), xr1 = wave_shift<DPP_WAVE_SHL1>(o1[j + 1][0]);
#pragma unroll
            for (int e = 0; e < VX; ++e)
                q2[j][e] = dcoef(y[j + 2][e], eyre) * o1[j + 1][e] +
                           e2ih2 * lap5<double, VX>(o1[j], o1[j + 1], o1[j + 2], xl1, xr1, e) - ccoef(y[j + 2][e], eyre);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const double xl1 = wave_shift<DPP_WAVE_SHR1>(q2[i + 1][VX - 1]), xr1 = wave_shift<DPP_WAVE_SHL1>(q2[i + 1][0]);
            const double ml = mb.left(i + 3), mr = mb.right(i + 3);
            double o[VX];
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const double r = -inv_h2 * outer_op<MOB, double, VX>(q2[i], q2[i + 1], q2[i + 2], xl1, xr1, mb.row(i + 2),
                                                                    mb.row(i + 3), mb.row(i + 4), ml, mr, e);
                o[e] = (y[i + 3][e] + ta2 * o1[i + 2][e] + tau * r) * inv2;
            }
            if (out && r0 + i < n) store_row<double, VX>(row_rsrc(O + (size_t)(r0 + i) * n, rb), bo, o);
        }
    }
}

template <bool SINGLE, int TAG, int VX, bool NEU = false, bool MOB = false>
__global__ __launch_bounds__(CH_STRIP_BLOCK) void k_lim_stage2_s(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                           const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                           const double* __restrict__ ybase, double* youtbase,
                                                           double* zbufbase, const double* __restrict__ coefs, int l) {
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    const LimLaunch L = lim_launch(ctl->p, l, true, ybase, youtbase, zbufbase);
    if (!L.live) return;
    const double* zbase = L.src;
    double* obase = L.dst;
    const int pos = L.pos;
    const double* cf = coefs + ((size_t)I.slot * 2 * CH_PMAX + pos) * 2;
    const double ta1 = cf[0], inv1 = cf[1], ta2 = cf[2], inv2 = cf[3], tau = ctl->tau0;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if constexpr (VX > 0) {
        lim2_strips<VX, NEU, MOB>(I, ybase, zbase, obase, ta1, inv1, ta2, inv2, tau, wv, mob_of(ctl, MOB));
    } else {
        if (I.vx == 1) lim2_strips<1, false, false>(I, ybase, zbase, obase, ta1, inv1, ta2, inv2, tau, wv, Mob{});
        else lim2_strips<2, false, false>(I, ybase, zbase, obase, ta1, inv1, ta2, inv2, tau, wv, Mob{});
    }
}

// ---------------------------------------------------------------------------
// EE2 estimate and next start vector (Fig. 4; eq. LIMest):
//   f1 = f(y^{n+1});  y_PC = y^n + tau/2 (f(y^n) + f1)  (eq. LIMest, since
//   f(y) = -A (F'(y) + eps^2 A y));  est = ||y^{n+1} - y_PC|| / ||y_PC||.
// f1 becomes the next step's f(y^n) and start vector; ||A c(y^{n+1})|| the next
// ||ghat||.  Lane partials of the four sums are returned in acc.
// ---------------------------------------------------------------------------
template <typename TV, int VX, bool NEU, bool MOB>
__device__ __forceinline__ void est_strips(const Inst& I, const double* __restrict__ y0base,
                                           const double* __restrict__ y1base, double* __restrict__ fbase,
                                           TV* __restrict__ V0base, float* __restrict__ y32base, double half_tau,
                                           int wv, double (&acc)[4], Mob mob) {
    constexpr int NU = SR + 4, ND = SR + 2, W = CH_STRIP_WAVES;
    const int lane = threadIdx.x & 63;
    const int n = I.n;
    constexpr int bc = NEU ? CH_BC_NEUMANN : CH_BC_PERIODIC;
    const double* Y0 = y0base + I.off;
    const double* Y1 = y1base + I.off;
    double* F = fbase + I.off;
    TV* V0 = V0base + I.off;
    float* Y32 = y32base ? y32base + I.off : nullptr;
    const double inv_h2 = I.inv_h2, e2ih2 = I.eps2 * I.inv_h2;
    const int eyre = I.eyre;
    const int nsx = (n + strip_cols(VX) - 1) / strip_cols(VX);
    const int ns = nsx * ((n + SR - 1) / SR);
    const int lb = xcd_remap(blockIdx.x - I.wblk0, I.wblk);
    for (int s = lb * W + wv; s < ns; s += I.wblk * W) {
        const StripPos<VX> P = strip_pos<VX>(s, nsx, n, lane, bc);
        const unsigned bo = (unsigned)P.xl * 8u;
        const unsigned bs = P.need ? bo : OFF_ROW, bd = P.out ? bo : OFF_ROW;
        double y1[NU][VX], y0[SR][VX], f0[SR][VX];
#pragma unroll
        for (int j = 0; j < NU; ++j) load_row<double, VX>(grid_row(Y1, P.r0 - 2 + j, n, bc), bs, y1[j]);
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            load_row<double, VX>(grid_row(Y0, P.r0 + i, n, bc), bd, y0[i]);
            load_row<double, VX>(grid_row(F, P.r0 + i, n, bc), bd, f0[i]);
        }
#pragma unroll
        for (int j = 0; j < NU; ++j) flip_if<double, VX>(P.rev, y1[j]);
        MobRows<MOB, double, VX, ND> mb;   // M(y^{n+1}) on rows r0 - 1 .. r0 + SR
#pragma unroll
        for (int j = 0; j < ND; ++j) mb.set(j, y1[j + 1], mob.m0, mob.m1);
        // inner expressions on rows r0 - 1 .. r0 + SR: F'(y) + eps^2 A y and c(y)
        double q[ND][VX], c[ND][VX];
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const double xl = wave_shift<DPP_WAVE_SHR1>(y1[j + 1][VX - 1]), xr = wave_shift<DPP_WAVE_SHL1>(y1[j + 1][0]);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const double v = y1[j + 1][e];
                q[j][e] = v * (v * v - 1.0) + e2ih2 * lap5<double, VX>(y1[j], y1[j + 1], y1[j + 2], xl, xr, e);
                c[j][e] = ccoef(v, eyre);
            }
        }
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            const double ql = wave_shift<DPP_WAVE_SHR1>(q[i + 1][VX - 1]), qr = wave_shift<DPP_WAVE_SHL1>(q[i + 1][0]);
            const double cl = wave_shift<DPP_WAVE_SHR1>(c[i + 1][VX - 1]), cr = wave_shift<DPP_WAVE_SHL1>(c[i + 1][0]);
            const double ml = mb.left(i + 1), mr = mb.right(i + 1);
            const bool in = P.out && P.r0 + i < n;
            double f1[VX];
            TV fv[VX];
            float yf[VX];
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                f1[e] = -inv_h2 * outer_op<MOB, double, VX>(q[i], q[i + 1], q[i + 2], ql, qr, mb.row(i), mb.row(i + 1),
                                                            mb.row(i + 2), ml, mr, e);
                const double g1 = inv_h2 * outer_op<MOB, double, VX>(c[i], c[i + 1], c[i + 2], cl, cr, mb.row(i),
                                                                     mb.row(i + 1), mb.row(i + 2), ml, mr, e);
                const double ypc = y0[i][e] + half_tau * (f0[i][e] + f1[e]);
                const double yv = y1[i + 2][e];
                const double er = yv - ypc;
                if (in) {
                    acc[0] += er * er;
                    acc[1] += ypc * ypc;
                    acc[2] += f1[e] * f1[e];
                    acc[3] += g1 * g1;
                }
                fv[e] = TV(f1[e]);
                yf[e] = float(yv);
            }
            if (in) {
                store_row<double, VX>(grid_row(F, P.r0 + i, n, bc), bo, f1);
                store_row<TV, VX>(grid_row(V0, P.r0 + i, n, bc), (unsigned)P.xl * (unsigned)sizeof(TV), fv);
                if (Y32) store_row<float, VX>(grid_row(Y32, P.r0 + i, n, bc), (unsigned)P.xl * 4u, yf);
            }
        }
    }
}

template <typename TV, bool SINGLE, int VX, bool NEU = false, bool MOB = false>
__global__ __launch_bounds__(CH_STRIP_BLOCK) void k_est_ee_s(Ctl* __restrict__ ctls, const Inst* __restrict__ insts,
                                                       const int* __restrict__ wb2i, const Inst inst0, int ninst,
                                                       const double* __restrict__ y0base,
                                                       const double* __restrict__ y1base, double* __restrict__ fbase,
                                                       TV* __restrict__ V0base, float* __restrict__ y32base,
                                                       double* __restrict__ pout) {
    const Inst I = SINGLE ? inst0 : insts[wb2i[blockIdx.x]];
    Ctl* ctl = ctls + I.slot;
    if (ctl->halted) return;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const double half_tau = 0.5 * (ctl->mode == MODE_EE ? ctl->tau_acc : ctl->tau_step);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (VX > 0) {
        est_strips<TV, VX, NEU, MOB>(I, y0base, y1base, fbase, V0base, y32base, half_tau, wv, acc, mob_of(ctl, MOB));
    } else {
        if (I.vx == 1) est_strips<TV, 1, false, false>(I, y0base, y1base, fbase, V0base, y32base, half_tau, wv, acc, Mob{});
        else if (sizeof(TV) == 8 || I.vx == 2) est_strips<TV, 2, false, false>(I, y0base, y1base, fbase, V0base, y32base, half_tau, wv, acc, Mob{});
        else est_strips<TV, (sizeof(TV) == 4 ? 4 : 2), false, false>(I, y0base, y1base, fbase, V0base, y32base, half_tau, wv, acc, Mob{});
    }
    write_partials<4, RED_SUM>(acc, pout);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define WARGS dim3(t.wgrid), dim3(CH_STRIP_BLOCK), 0, s, b.ctl, t.inst, t.wb2i, t.hinst[0], t.ninst

// A single grid with Neumann boundaries (batches are periodic).
static bool neumann(const Table& t) { return t.ninst == 1 && t.hinst[0].bc == CH_BC_NEUMANN; }

template <typename TV, int DM, bool TIMING, int VX>
static void launch_matvec_one(const Table& t, const DevBuffers& b, const TV* y, int k, int store_w, double* pout,
                              hipStream_t s) {
    if (mobility(t))
        hipLaunchKernelGGL((k_matvec_s<TV, true, DM, TIMING ? 1 : 0, VX, false, true>), WARGS, static_cast<TV*>(b.V),
                           b.ldv, k, store_w, y, pout);
    else if (neumann(t))
        hipLaunchKernelGGL((k_matvec_s<TV, true, DM, TIMING ? 1 : 0, VX, true>), WARGS, static_cast<TV*>(b.V), b.ldv,
                           k, store_w, y, pout);
    else
        hipLaunchKernelGGL((k_matvec_s<TV, true, DM, TIMING ? 1 : 0, VX>), WARGS, static_cast<TV*>(b.V), b.ldv, k,
                           store_w, y, pout);
}

template <typename TV, int DM, bool TIMING>
static void launch_matvec_single(const Table& t, const DevBuffers& b, const TV* y, int k, int store_w, double* pout,
                                 hipStream_t s) {
    const int vx = t.hinst[0].vx;
    if constexpr (sizeof(TV) == 4) {
        if (vx >= 4) return launch_matvec_one<TV, DM, TIMING, 4>(t, b, y, k, store_w, pout, s);
    }
    if (vx >= 2) launch_matvec_one<TV, DM, TIMING, 2>(t, b, y, k, store_w, pout, s);
    else launch_matvec_one<TV, DM, TIMING, 1>(t, b, y, k, store_w, pout, s);
}

template <typename TV, int DM>
static void launch_matvec_s(const Table& t, const DevBuffers& b, const TV* y, int k, int store_w, double* pout,
                            bool timing, hipStream_t s) {
    if (timing)
        launch_matvec_single<TV, DM, true>(t, b, y, k, store_w, pout, s);
    else if (t.ninst == 1)
        launch_matvec_single<TV, DM, false>(t, b, y, k, store_w, pout, s);
    else
        hipLaunchKernelGGL((k_matvec_s<TV, false, DM, 0, 0>), WARGS, static_cast<TV*>(b.V), b.ldv, k, store_w, y,
                           pout);
}

hipError_t launch_matvec_strip(const Table& t, int prec, const DevBuffers& b, const double* y, int k, int dots,
                               bool store_w, double* pout, bool timing, hipStream_t s) {
    const int sw = store_w ? 1 : 0;
    if (prec == CH_FP64) {
        if (dots == MV_DOTS_DC) launch_matvec_s<double, DM_DC>(t, b, y, k, sw, pout, timing, s);
        else launch_matvec_s<double, DM_ONE>(t, b, y, k, sw, pout, timing, s);
    } else {
        if (dots == MV_DOTS_DC) launch_matvec_s<float, DM_DC>(t, b, b.y32, k, sw, pout, timing, s);
        else launch_matvec_s<float, DM_ONE>(t, b, b.y32, k, sw, pout, timing, s);
    }
    return hipGetLastError();
}

hipError_t launch_lim_stage_strip(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                                  bool pairs, bool timing, hipStream_t s) {
    const bool two = t.hinst[0].vx >= 2;
    const int pr = pairs ? 1 : 0;
    if (mobility(t)) {
        if (two) hipLaunchKernelGGL((k_lim_stage_s<true, 0, 2, false, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
        else hipLaunchKernelGGL((k_lim_stage_s<true, 0, 1, false, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
    } else if (neumann(t)) {
        if (two) hipLaunchKernelGGL((k_lim_stage_s<true, 0, 2, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
        else hipLaunchKernelGGL((k_lim_stage_s<true, 0, 1, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
    } else if (timing) {
        if (two) hipLaunchKernelGGL((k_lim_stage_s<true, 1, 2>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
        else hipLaunchKernelGGL((k_lim_stage_s<true, 1, 1>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
    } else if (t.ninst == 1) {
        if (two) hipLaunchKernelGGL((k_lim_stage_s<true, 0, 2>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
        else hipLaunchKernelGGL((k_lim_stage_s<true, 0, 1>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
    } else {
        hipLaunchKernelGGL((k_lim_stage_s<false, 0, 0>), WARGS, yin, yout, b.zbuf, b.lcoef, l, pr);
    }
    return hipGetLastError();
}

hipError_t launch_lim_stage2_strip(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                                   bool timing, hipStream_t s) {
    const bool two = t.hinst[0].vx >= 2;
    if (mobility(t)) {
        if (two) hipLaunchKernelGGL((k_lim_stage2_s<true, 0, 2, false, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
        else hipLaunchKernelGGL((k_lim_stage2_s<true, 0, 1, false, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
    } else if (neumann(t)) {
        if (two) hipLaunchKernelGGL((k_lim_stage2_s<true, 0, 2, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
        else hipLaunchKernelGGL((k_lim_stage2_s<true, 0, 1, true>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
    } else if (timing) {
        if (two) hipLaunchKernelGGL((k_lim_stage2_s<true, 1, 2>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
        else hipLaunchKernelGGL((k_lim_stage2_s<true, 1, 1>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
    } else if (t.ninst == 1) {
        if (two) hipLaunchKernelGGL((k_lim_stage2_s<true, 0, 2>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
        else hipLaunchKernelGGL((k_lim_stage2_s<true, 0, 1>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
    } else {
        hipLaunchKernelGGL((k_lim_stage2_s<false, 0, 0>), WARGS, yin, yout, b.zbuf, b.lcoef, l);
    }
    return hipGetLastError();
}

template <typename TV>
static void launch_est_ee_s(const Table& t, const DevBuffers& b, const double* y0, const double* y1, float* y32,
                            double* pout, hipStream_t s) {
    TV* V0 = static_cast<TV*>(b.V);
    if (t.ninst > 1) {
        hipLaunchKernelGGL((k_est_ee_s<TV, false, 0>), WARGS, y0, y1, b.fcur, V0, y32, pout);
        return;
    }
    const int vx = t.hinst[0].vx;
    if (mobility(t)) {
        if (sizeof(TV) == 4 && vx >= 4)
            hipLaunchKernelGGL((k_est_ee_s<TV, true, (sizeof(TV) == 4 ? 4 : 2), false, true>), WARGS, y0, y1, b.fcur,
                               V0, y32, pout);
        else if (vx >= 2) hipLaunchKernelGGL((k_est_ee_s<TV, true, 2, false, true>), WARGS, y0, y1, b.fcur, V0, y32, pout);
        else hipLaunchKernelGGL((k_est_ee_s<TV, true, 1, false, true>), WARGS, y0, y1, b.fcur, V0, y32, pout);
        return;
    }
    if (neumann(t)) {
        if (sizeof(TV) == 4 && vx >= 4)
            hipLaunchKernelGGL((k_est_ee_s<TV, true, (sizeof(TV) == 4 ? 4 : 2), true>), WARGS, y0, y1, b.fcur, V0, y32,
                               pout);
        else if (vx >= 2) hipLaunchKernelGGL((k_est_ee_s<TV, true, 2, true>), WARGS, y0, y1, b.fcur, V0, y32, pout);
        else hipLaunchKernelGGL((k_est_ee_s<TV, true, 1, true>), WARGS, y0, y1, b.fcur, V0, y32, pout);
        return;
    }
    if constexpr (sizeof(TV) == 4) {
        if (vx >= 4) {
            hipLaunchKernelGGL((k_est_ee_s<TV, true, 4>), WARGS, y0, y1, b.fcur, V0, y32, pout);
            return;
        }
    }
    if (vx >= 2) hipLaunchKernelGGL((k_est_ee_s<TV, true, 2>), WARGS, y0, y1, b.fcur, V0, y32, pout);
    else hipLaunchKernelGGL((k_est_ee_s<TV, true, 1>), WARGS, y0, y1, b.fcur, V0, y32, pout);
}

hipError_t launch_est_ee_strip(const Table& t, int prec, const DevBuffers& b, const double* y0, const double* y1,
                               double* pout, hipStream_t s) {
    if (prec == CH_FP64) launch_est_ee_s<double>(t, b, y0, y1, nullptr, pout, s);
    else launch_est_ee_s<float>(t, b, y0, y1, b.y32, pout, s);
    return hipGetLastError();
}
