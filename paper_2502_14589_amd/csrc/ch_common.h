// Device helpers shared by the libch kernels: deterministic two-stage
// reductions, 16-byte vector access and the stencil tile geometry.
#pragma once

#include "ch_internal.h"

// ---------------------------------------------------------------------------
// Reductions.  Wave64 butterfly, then the waves of a workgroup through LDS,
// then one partial per workgroup in global memory, added up in a fixed order
// by the consuming launch (below), so results do not depend on scheduling.
// ---------------------------------------------------------------------------

// Lane exchanges.  Within a row of 16 lanes the data-parallel-primitive
// (DPP) forms move data in the vector ALU; across rows a permute through the
// LDS crossbar is needed.  Pairings used (each an involution):
//   DPP_XOR1  quad_perm [1,0,3,2]     lane ^ 1
//   DPP_XOR2  quad_perm [2,3,0,1]     lane ^ 2
//   DPP_HMIR  row_half_mirror         lane <-> 7 - lane within 8 lanes
//   DPP_MIR   row_mirror              lane <-> 15 - lane within 16 lanes
enum DppCtrl { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HMIR = 0x141, DPP_MIR = 0x140 };

template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Butterfly over the 64 lanes: DPP within rows, two permutes across them.
template <typename Op>
__device__ __forceinline__ double wave_reduce(double x, Op op) {
    x = op(x, dpp_move<DPP_XOR1>(x));
    x = op(x, dpp_move<DPP_XOR2>(x));
    x = op(x, dpp_move<DPP_HMIR>(x));
    x = op(x, dpp_move<DPP_MIR>(x));
    x = op(x, __shfl_xor(x, 16, 64));
    x = op(x, __shfl_xor(x, 32, 64));
    return x;
}

__device__ __forceinline__ double wave_sum(double x) {
    return wave_reduce(x, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ double wave_max(double x) {
    return wave_reduce(x, [](double a, double b) { return fmax(a, b); });
}

__device__ __forceinline__ double wave_min(double x) {
    return wave_reduce(x, [](double a, double b) { return fmin(a, b); });
}

// Eight wave-wide sums at once.  In each of three exchanges (row mirror, half
// mirror, lane ^ 2) a lane keeps half of its values, sends the other half to
// its partner and adds the partner's copy of the half it kept; then plain
// butterfly steps over the lanes that hold the same value (lane ^ 1, ^ 16,
// ^ 32).  Seven DPP moves and two cross-row permutes per double instead of
// the 48 permutes of eight wave_sum calls.  Lane L ends with the total of
// value ((L >> 3) & 1) * 4 + ((L >> 2) & 1) * 2 + ((L >> 1) & 1); lanes 2v
// (v = 0..7) hold value v (see wave_sum8_holder).
template <int CTRL>
__device__ __forceinline__ void keep_half(double* a, int h, bool hi) {
#pragma unroll
    for (int i = 0; i < h; ++i) {
        const double send = hi ? a[i] : a[i + h];
        const double keep = hi ? a[i + h] : a[i];
        a[i] = keep + dpp_move<CTRL>(send);
    }
}

__device__ __forceinline__ double wave_sum8(double (&a)[8]) {
    const int lane = threadIdx.x & 63;
    keep_half<DPP_MIR>(a, 4, (lane & 8) != 0);
    keep_half<DPP_HMIR>(a, 2, (lane & 4) != 0);
    keep_half<DPP_XOR2>(a, 1, (lane & 2) != 0);
    double x = a[0];
    x += dpp_move<DPP_XOR1>(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

// Index of the value whose total lane `lane` is to store after wave_sum8,
// or -1 (each value is stored by one lane).
__device__ __forceinline__ int wave_sum8_holder(int lane) { return (lane & 0x31) == 0 ? (lane >> 1) & 7 : -1; }

enum RedOp { RED_SUM = 0, RED_MIN = 1, RED_MAX = 2 };

template <int OP>
__device__ __forceinline__ double red_wave(double x) {
    if (OP == RED_SUM) return wave_sum(x);
    if (OP == RED_MIN) return wave_min(x);
    return wave_max(x);
}

template <int OP>
__device__ __forceinline__ double red_combine(double a, double b) {
    if (OP == RED_SUM) return a + b;
    if (OP == RED_MIN) return fmin(a, b);
    return fmax(a, b);
}

template <int OP>
__device__ __forceinline__ double red_identity() {
    if (OP == RED_SUM) return 0.0;
    if (OP == RED_MIN) return __builtin_inf();
    return -__builtin_inf();
}

// Workgroup reduction of NR values (up to 16 waves); the result is valid in
// thread 0.
template <int NR, int OP>
__device__ __forceinline__ void block_reduce(double (&x)[NR], double (*lds)[NR]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (int)(blockDim.x >> 6);
#pragma unroll
    for (int r = 0; r < NR; ++r) x[r] = red_wave<OP>(x[r]);
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) lds[wid][r] = x[r];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double s = lds[0][r];
            for (int w = 1; w < nw; ++w) s = red_combine<OP>(s, lds[w][r]);
            x[r] = s;
        }
    }
    __syncthreads();
}

// Grid-wide reductions without atomics or fences.  A producing launch writes
// one partial per workgroup (and per sum) into a partials slot; the launch
// that consumes them -- the next one on the stream, so the kernel boundary
// orders and publishes the writes -- sums the partials in a fixed order in
// every workgroup.  Deterministic: each consumer workgroup sees the same total.
// Slots alternate between consecutive producers (ping-pong), so a consumer
// never overwrites the partials it is still reading.
template <int NR, int OP>
__device__ __forceinline__ void write_partials(double (&x)[NR], double* __restrict__ pout) {
    __shared__ double lds[16][NR];
    block_reduce<NR, OP>(x, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) pout[r * CH_MAXB + blockIdx.x] = x[r];
    }
}

// Total of the partials [p0, p0 + np) of each of the NR sums, returned in every
// thread.  np <= CH_PART_PER_THREAD * CH_BLOCK; every thread issues its loads
// at once (one memory latency), then adds them in a fixed order.
#define CH_PART_PER_THREAD 8
template <int NR, int OP>
__device__ __forceinline__ void sum_partials(const double* __restrict__ pin, int p0, int np, double (&tot)[NR]) {
    __shared__ double lds[16][NR];
    __shared__ double res[NR];
    double v[NR][CH_PART_PER_THREAD];
#pragma unroll
    for (int u = 0; u < CH_PART_PER_THREAD; ++u) {
        const int b = threadIdx.x + u * CH_BLOCK;
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r][u] = b < np ? pin[r * CH_MAXB + p0 + b] : red_identity<OP>();
    }
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        s[r] = v[r][0];
#pragma unroll
        for (int u = 1; u < CH_PART_PER_THREAD; ++u) s[r] = red_combine<OP>(s[r], v[r][u]);
    }
    block_reduce<NR, OP>(s, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) res[r] = s[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) tot[r] = res[r];
}

// The partials an instance's consumer adds up: those of its tile, strip or
// streaming workgroups, whichever kind (PartKind) produced them.
template <int NR, int OP>
__device__ __forceinline__ void sum_inst_partials(const double* __restrict__ pin, const Inst& I, int kind,
                                                  double (&tot)[NR]) {
    if (kind == PK_TILE)
        sum_partials<NR, OP>(pin, I.sblk0, I.sblk, tot);
    else if (kind == PK_STRIP)
        sum_partials<NR, OP>(pin, I.wblk0, I.wblk, tot);
    else
        sum_partials<NR, OP>(pin, I.cblk0, I.cblk, tot);
}

// ---------------------------------------------------------------------------
// 16-byte vectors
// ---------------------------------------------------------------------------
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double2; static constexpr int W = 2; };
template <> struct Vec16<float> { using type = float4; static constexpr int W = 4; };

// ---------------------------------------------------------------------------
// Stencil tiles.  A workgroup owns a TX x TY (x TZ) block of outputs; the
// operand is staged in LDS with a halo of 2 (A applied twice) and the frozen
// state with a halo of 1.  Periodic wrap by index arithmetic.
// ---------------------------------------------------------------------------
template <int DIM> struct Geo;
template <> struct Geo<2> {
    static constexpr int TX = 64, TY = 8, TZ = 1;
};
template <> struct Geo<3> {
    static constexpr int TX = 32, TY = 4, TZ = 4;
};

template <int DIM, int H> struct Region {
    static constexpr int X = Geo<DIM>::TX + 2 * H;
    static constexpr int Y = Geo<DIM>::TY + 2 * H;
    static constexpr int Z = DIM == 3 ? Geo<DIM>::TZ + 2 * H : 1;
    static constexpr int SIZE = X * Y * Z;
};

__device__ __forceinline__ int wrapi(int g, int n) {
    int w = g % n;
    return w < 0 ? w + n : w;
}

struct TileOrigin {
    int x0, y0, z0;
};

template <int DIM>
__device__ __forceinline__ int num_tiles(int n, int& ntx, int& nty) {
    ntx = (n + Geo<DIM>::TX - 1) / Geo<DIM>::TX;
    nty = (n + Geo<DIM>::TY - 1) / Geo<DIM>::TY;
    const int ntz = DIM == 3 ? (n + Geo<DIM>::TZ - 1) / Geo<DIM>::TZ : 1;
    return ntx * nty * ntz;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous band of tiles so that halo rows shared by neighbouring tiles
// are re-read from the same L2.  Bijective on [0, G).
__device__ __forceinline__ int xcd_remap(int bid, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = bid & 7, local = bid >> 3;
    return x * q + min(x, r) + local;
}

template <int DIM>
__device__ __forceinline__ TileOrigin tile_origin(int t, int ntx, int nty) {
    TileOrigin o;
    o.x0 = (t % ntx) * Geo<DIM>::TX;
    const int r = t / ntx;
    o.y0 = (r % nty) * Geo<DIM>::TY;
    o.z0 = DIM == 3 ? (r / nty) * Geo<DIM>::TZ : 0;
    return o;
}

// Global index of point i of the halo-H region around the tile (periodic wrap
// or Neumann mirror, bc_index, unless the whole region is inside the grid).
// Tile regions reach at most TX + H past the grid (< n for n >= 5 whenever a
// tile starts inside it), so one fold suffices except in the periodic wrap.
template <int DIM, int H>
__device__ __forceinline__ size_t region_index(const TileOrigin& o, int n, int i, bool interior, int bc) {
    using R = Region<DIM, H>;
    const int cx = i % R::X;
    const int rr = i / R::X;
    const int cy = rr % R::Y;
    const int cz = rr / R::Y;
    int gx = o.x0 + cx - H, gy = o.y0 + cy - H, gz = DIM == 3 ? o.z0 + cz - H : 0;
    if (!interior) {
        if (bc == CH_BC_NEUMANN) {
            gx = bc_index(min(gx, 2 * n - 1), n, bc);
            gy = bc_index(min(gy, 2 * n - 1), n, bc);
            if (DIM == 3) gz = bc_index(min(gz, 2 * n - 1), n, bc);
        } else {
            gx = wrapi(gx, n);
            gy = wrapi(gy, n);
            if (DIM == 3) gz = wrapi(gz, n);
        }
    }
    return ((size_t)gz * n + gy) * n + gx;
}

template <int DIM, int H>
__device__ __forceinline__ bool region_inside(const TileOrigin& o, int n) {
    return o.x0 >= H && o.x0 + Geo<DIM>::TX + H <= n && o.y0 >= H && o.y0 + Geo<DIM>::TY + H <= n &&
           (DIM == 2 || (o.z0 >= H && o.z0 + Geo<DIM>::TZ + H <= n));
}

// Load the regions of halo HA around the tile from `a` and of halo HB from
// `b`, calling putA(i, value) / putB(i, value) with the region's linear
// index.  Every load of both regions is issued before the first value is
// used, so a workgroup waits for memory once per tile.
template <int DIM, int HA, int HB, typename TA, typename TB, typename PA, typename PB>
__device__ __forceinline__ void load_regions(const TileOrigin& o, int n, int bc, const TA* __restrict__ a, PA&& putA,
                                             const TB* __restrict__ b, PB&& putB) {
    using RA = Region<DIM, HA>;
    using RB = Region<DIM, HB>;
    constexpr int NA = (RA::SIZE + CH_BLOCK - 1) / CH_BLOCK;
    constexpr int NB = (RB::SIZE + CH_BLOCK - 1) / CH_BLOCK;
    const bool ina = region_inside<DIM, HA>(o, n), inb = region_inside<DIM, HB>(o, n);
    TA va[NA];
    TB vb[NB];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        const int i = threadIdx.x + u * CH_BLOCK;
        if (i < RA::SIZE) va[u] = a[region_index<DIM, HA>(o, n, i, ina, bc)];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int i = threadIdx.x + u * CH_BLOCK;
        if (i < RB::SIZE) vb[u] = b[region_index<DIM, HB>(o, n, i, inb, bc)];
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        const int i = threadIdx.x + u * CH_BLOCK;
        if (i < RA::SIZE) putA(i, va[u]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int i = threadIdx.x + u * CH_BLOCK;
        if (i < RB::SIZE) putB(i, vb[u]);
    }
}

// One region of halo H, its loads issued together (see load_regions).
template <int DIM, int H, typename TS, typename Put>
__device__ __forceinline__ void load_region(const TileOrigin& o, int n, int bc, const TS* __restrict__ src, Put&& put) {
    using R = Region<DIM, H>;
    constexpr int NL = (R::SIZE + CH_BLOCK - 1) / CH_BLOCK;
    const bool in = region_inside<DIM, H>(o, n);
    TS v[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int i = threadIdx.x + u * CH_BLOCK;
        if (i < R::SIZE) v[u] = src[region_index<DIM, H>(o, n, i, in, bc)];
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int i = threadIdx.x + u * CH_BLOCK;
        if (i < R::SIZE) put(i, v[u]);
    }
}

// Index in the halo-2 region of the centre of halo-1 point i1.
template <int DIM>
__device__ __forceinline__ int r1_to_r2(int i1) {
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    const int cx = i1 % R1::X;
    const int rr = i1 / R1::X;
    const int cy = rr % R1::Y;
    const int cz = rr / R1::Y;
    return ((cz + (DIM == 3 ? 1 : 0)) * R2::Y + (cy + 1)) * R2::X + (cx + 1);
}

// Unscaled -Laplacian (2 dim c - neighbours) at index c of a region with row
// length RX and plane size RXY.
template <int DIM, int RX, int RXY, typename T>
__device__ __forceinline__ T lap_at(const T* s, int c) {
    T nb = (s[c - 1] + s[c + 1]) + (s[c - RX] + s[c + RX]);
    if (DIM == 3) nb += s[c - RXY] + s[c + RXY];
    return T(2 * DIM) * s[c] - nb;
}

template <int DIM, typename T>
__device__ __forceinline__ T lap2_at_r1(const T* s2, int i1) {
    using R2 = Region<DIM, 2>;
    return lap_at<DIM, R2::X, R2::X * R2::Y>(s2, r1_to_r2<DIM>(i1));
}

// Output point i0 of the tile: its halo-1 index and global coordinates.
template <int DIM>
__device__ __forceinline__ bool out_point(int i0, const TileOrigin& o, int n, int& i1, size_t& gi) {
    constexpr int TX = Geo<DIM>::TX, TY = Geo<DIM>::TY;
    using R1 = Region<DIM, 1>;
    const int cx = i0 % TX;
    const int rr = i0 / TX;
    const int cy = rr % TY;
    const int cz = rr / TY;
    i1 = ((cz + (DIM == 3 ? 1 : 0)) * R1::Y + (cy + 1)) * R1::X + (cx + 1);
    const int gx = o.x0 + cx, gy = o.y0 + cy, gz = o.z0 + cz;
    gi = ((size_t)gz * n + gy) * n + gx;
    return gx < n && gy < n && (DIM == 2 || gz < n);
}

template <int DIM, typename T>
__device__ __forceinline__ T lap1_at(const T* s1, int i1) {
    using R1 = Region<DIM, 1>;
    return lap_at<DIM, R1::X, R1::X * R1::Y>(s1, i1);
}

// Flux form of the variable-mobility operator (Section 2, Remark 1), unscaled:
// sum over the neighbours k of c of (m_c + m_k)/2 (s_c - s_k), for values s
// and mobilities m in two halo-1 regions (2-D).  With m = 1 it is lap1_at.
template <typename T>
__device__ __forceinline__ T lap1m_at(const T* s1, const T* m1, int i1) {
    using R1 = Region<2, 1>;
    constexpr int RX = R1::X;
    const T sc = s1[i1], mc = m1[i1];
    auto flux = [&](int k) { return (mc + m1[k]) * (sc - s1[k]); };
    return T(0.5) * ((flux(i1 - 1) + flux(i1 + 1)) + (flux(i1 - RX) + flux(i1 + RX)));
}

template <int DIM>
constexpr int tile_points() {
    return Geo<DIM>::TX * Geo<DIM>::TY * Geo<DIM>::TZ;
}
