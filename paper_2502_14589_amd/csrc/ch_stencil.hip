// Fused stencil kernels: Jacobian matvec with the first Gram-Schmidt dot,
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
#include "ch_common.h"

namespace {

__device__ __forceinline__ double cheb_node(int i, int p) {
    return cos(3.141592653589793 * double(2 * i - 1) / double(2 * p));
}

template <typename T>
__device__ __forceinline__ T dcoef(T y, int eyre) {
    return T(3) * y * y - T(1) + T(eyre);
}
template <typename T>
__device__ __forceinline__ T ccoef(T y, int eyre) {
    return T(2) * y * y * y + (eyre ? y : T(0));
}

// ---------------------------------------------------------------------------
// w = Ahat (vscale[k] V_k) and the partials of <w, V_0> (Fig. 3, lines 4-6, i = 1)
// ---------------------------------------------------------------------------
template <int DIM, typename TV, typename TY>
__global__ __launch_bounds__(CH_BLOCK) void k_matvec(Ctl* __restrict__ ctl, const TV* __restrict__ Vk,
                                                     const TY* __restrict__ y, TV* __restrict__ W,
                                                     const TV* __restrict__ V0, int k, double* __restrict__ pout,
                                                     int n, double eps2_, double inv_h2_, int eyre) {
    if (ctl->done | ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    __shared__ TV sv[R2::SIZE];
    __shared__ TV sd[R1::SIZE];
    __shared__ TV sq[R1::SIZE];
    const TV sc = TV(ctl->vscale[k]);
    const TV ih2 = TV(inv_h2_), e2ih2 = TV(eps2_ * inv_h2_);
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    double dot = 0.0;
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_region<DIM, 2>(o, n, Vk, [&](int i, TV v) { sv[i] = sc * v; });
        load_region<DIM, 1>(o, n, y, [&](int i, TY v) { sd[i] = dcoef(TV(v), eyre); });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += blockDim.x)
            sq[i] = sd[i] * sv[r1_to_r2<DIM>(i)] + e2ih2 * lap2_at_r1<DIM>(sv, i);
        __syncthreads();
        for (int i = threadIdx.x; i < tile_points<DIM>(); i += blockDim.x) {
            int i1;
            size_t gi;
            if (out_point<DIM>(i, o, n, i1, gi)) {
                const TV w = ih2 * lap1_at<DIM>(sq, i1);
                W[gi] = w;
                dot += double(w) * double(V0[gi]);
            }
        }
        __syncthreads();
    }
    double x[1] = {dot};
    write_partials<1, RED_SUM>(x, pout);
}

// ---------------------------------------------------------------------------
// Residual of the frozen linear problem at state z:
//     r = ghat - Ahat z = A (c(y) - d(y) z - eps^2 A z)
// With z = y this is f(y) (eq. IVP), the EE2 start vector (Fig. 3, line 2).
// Writes r to V_0 (and FP64 to fcur when write_f), optionally the FP32 copy
// of y; partials of ||r||^2 and ||A c(y)||^2 = ||ghat||^2 (eq. tol_phi).
// ---------------------------------------------------------------------------
template <int DIM, typename TV>
__global__ __launch_bounds__(CH_BLOCK) void k_resid(Ctl* __restrict__ ctl, const double* __restrict__ y,
                                                    const double* __restrict__ z, double* __restrict__ fout,
                                                    TV* __restrict__ V0, float* __restrict__ y32,
                                                    double* __restrict__ pout, int n, double eps2, double inv_h2,
                                                    int eyre) {
    if (ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    __shared__ double sz[R2::SIZE];
    __shared__ double sdq[R1::SIZE];   // d(y), then the inner expression
    __shared__ double sc[R1::SIZE];
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    double acc_r = 0.0, acc_g = 0.0;
    const double e2ih2 = eps2 * inv_h2;
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_region<DIM, 2>(o, n, z, [&](int i, double v) { sz[i] = v; });
        load_region<DIM, 1>(o, n, y, [&](int i, double v) {
            sdq[i] = dcoef(v, eyre);
            sc[i] = ccoef(v, eyre);
        });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += blockDim.x)
            sdq[i] = sdq[i] * sz[r1_to_r2<DIM>(i)] + e2ih2 * lap2_at_r1<DIM>(sz, i) - sc[i];
        __syncthreads();
        for (int i = threadIdx.x; i < tile_points<DIM>(); i += blockDim.x) {
            int i1;
            size_t gi;
            if (out_point<DIM>(i, o, n, i1, gi)) {
                const double r = -inv_h2 * lap1_at<DIM>(sdq, i1);
                const double g = inv_h2 * lap1_at<DIM>(sc, i1);
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
// EE2 estimate and next start vector (Fig. 4, line 8; eq. LIMest):
//   f1 = f(y^{n+1});  y_PC = y^n + tau/2 (f(y^n) + f1)  (eq. LIMest, since
//   f(y) = -A (F'(y) + eps^2 A y));  est = ||y^{n+1} - y_PC|| / ||y_PC||.
// f1 becomes the next step's f(y^n) and start vector; ||A c(y^{n+1})|| the next
// ||ghat||.  Partials of the four sums go to the step controller.
// ---------------------------------------------------------------------------
template <int DIM, typename TV>
__global__ __launch_bounds__(CH_BLOCK) void k_est_ee(Ctl* __restrict__ ctl, const double* __restrict__ y0,
                                                     const double* __restrict__ y1, double* __restrict__ fcur,
                                                     TV* __restrict__ V0, float* __restrict__ y32,
                                                     double* __restrict__ pout, int n, double eps2, double inv_h2,
                                                     int eyre) {
    if (ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    __shared__ double s1[R2::SIZE];
    __shared__ double sq[R1::SIZE];
    __shared__ double sc[R1::SIZE];
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    const double half_tau = 0.5 * (ctl->mode == MODE_EE ? ctl->tau_acc : ctl->tau_step);
    const double e2ih2 = eps2 * inv_h2;
    double a_err = 0.0, a_pc = 0.0, a_f = 0.0, a_g = 0.0;
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_region<DIM, 2>(o, n, y1, [&](int i, double v) { s1[i] = v; });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += blockDim.x) {
            const double v = s1[r1_to_r2<DIM>(i)];
            sq[i] = v * (v * v - 1.0) + e2ih2 * lap2_at_r1<DIM>(s1, i);
            sc[i] = ccoef(v, eyre);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < tile_points<DIM>(); i += blockDim.x) {
            int i1;
            size_t gi;
            if (out_point<DIM>(i, o, n, i1, gi)) {
                const double f1 = -inv_h2 * lap1_at<DIM>(sq, i1);
                const double g1 = inv_h2 * lap1_at<DIM>(sc, i1);
                const double ypc = y0[gi] + half_tau * (fcur[gi] + f1);
                const double yv = y1[gi];
                const double e = yv - ypc;
                a_err += e * e;
                a_pc += ypc * ypc;
                a_f += f1 * f1;
                a_g += g1 * g1;
                fcur[gi] = f1;
                V0[gi] = TV(f1);
                if (y32) y32[gi] = float(yv);
            }
        }
        __syncthreads();
    }
    double x[4] = {a_err, a_pc, a_f, a_g};
    write_partials<4, RED_SUM>(x, pout);
}

// ---------------------------------------------------------------------------
// LIM stage (Fig. 1, steps 6 and 10):
//   y_next = (y^n + tau a_m z + tau (ghat - Ahat z)) / (1 + tau a_m)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(CH_BLOCK) void k_lim_stage(Ctl* __restrict__ ctl, const double* __restrict__ y,
                                                        const double* __restrict__ z, double* __restrict__ out,
                                                        int m, int n, double eps2, double inv_h2, int eyre) {
    if (ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    __shared__ double sz[R2::SIZE];
    __shared__ double sdq[R1::SIZE];
    __shared__ double sc[R1::SIZE];
    const double tau = ctl->tau0;
    // Fig. 1, steps 2-5: beta_i = cos(pi (2i - 1) / (2p)), z_1 = beta_1,
    // a_m = lambda_max (z_1 - beta_m) / (1 + z_1)
    const int p = ctl->p;
    const double z1 = cheb_node(1, p);
    const double am = ctl->lam / (1.0 + z1) * (z1 - cheb_node(m, p));
    const double ta = tau * am;
    const double inv = 1.0 / (1.0 + ta);
    const double e2ih2 = eps2 * inv_h2;
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_region<DIM, 2>(o, n, z, [&](int i, double v) { sz[i] = v; });
        load_region<DIM, 1>(o, n, y, [&](int i, double v) {
            sdq[i] = dcoef(v, eyre);
            sc[i] = ccoef(v, eyre);
        });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += blockDim.x)
            sdq[i] = sdq[i] * sz[r1_to_r2<DIM>(i)] + e2ih2 * lap2_at_r1<DIM>(sz, i) - sc[i];
        __syncthreads();
        for (int i = threadIdx.x; i < tile_points<DIM>(); i += blockDim.x) {
            int i1;
            size_t gi;
            if (out_point<DIM>(i, o, n, i1, gi)) {
                const double r = -inv_h2 * lap1_at<DIM>(sdq, i1);
                const double zc = sz[r1_to_r2<DIM>(i1)];
                out[gi] = (y[gi] + ta * zc + tau * r) * inv;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// LIM estimate (Fig. 2, line 8; eq. LIMest):
//   y_PC = y^n - tau/2 A (F'(y^n) + F'(y^{n+1}) + eps^2 A (y^n + y^{n+1}));
// partials of ||y^{n+1} - y_PC||^2 and ||y_PC||^2 go to the controller.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(CH_BLOCK) void k_est_lim(Ctl* __restrict__ ctl, const double* __restrict__ y0,
                                                      const double* __restrict__ y1, double* __restrict__ pout,
                                                      int n, double eps2, double inv_h2) {
    if (ctl->halted) return;
    using R1 = Region<DIM, 1>;
    using R2 = Region<DIM, 2>;
    __shared__ double s0[R2::SIZE];
    __shared__ double s1[R2::SIZE];
    __shared__ double sq[R1::SIZE];
    const double tau = ctl->tau0;
    const double e2ih2 = eps2 * inv_h2;
    int ntx, nty;
    const int nt = num_tiles<DIM>(n, ntx, nty);
    double a_err = 0.0, a_pc = 0.0;
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
        const TileOrigin o = tile_origin<DIM>(t, ntx, nty);
        load_region<DIM, 2>(o, n, y0, [&](int i, double v) { s0[i] = v; });
        load_region<DIM, 2>(o, n, y1, [&](int i, double v) { s1[i] = v; });
        __syncthreads();
        for (int i = threadIdx.x; i < R1::SIZE; i += blockDim.x) {
            const int c = r1_to_r2<DIM>(i);
            const double a = s0[c], b = s1[c];
            sq[i] = a * (a * a - 1.0) + b * (b * b - 1.0) +
                    e2ih2 * (lap2_at_r1<DIM>(s0, i) + lap2_at_r1<DIM>(s1, i));
        }
        __syncthreads();
        for (int i = threadIdx.x; i < tile_points<DIM>(); i += blockDim.x) {
            int i1;
            size_t gi;
            if (out_point<DIM>(i, o, n, i1, gi)) {
                const int c = r1_to_r2<DIM>(i1);
                const double ypc = s0[c] - 0.5 * tau * inv_h2 * lap1_at<DIM>(sq, i1);
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

template <int DIM>
int stencil_grid(int n) {
    const int ntx = (n + Geo<DIM>::TX - 1) / Geo<DIM>::TX;
    const int nty = (n + Geo<DIM>::TY - 1) / Geo<DIM>::TY;
    const int ntz = DIM == 3 ? (n + Geo<DIM>::TZ - 1) / Geo<DIM>::TZ : 1;
    const long long nt = (long long)ntx * nty * ntz;
    return (int)(nt < 2048 ? nt : 2048);   // larger grids loop over tiles
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int DIM, typename TV>
static hipError_t launch_matvec_t(const Grid& g, const DevBuffers& b, PartSeq& ps, const void* y, int k,
                                  hipStream_t s) {
    TV* V = static_cast<TV*>(b.V);
    const TV* Vk = V + (size_t)k * b.ldv;
    TV* W = V + (size_t)(k + 1) * b.ldv;
    const int G = stencil_grid<DIM>(g.n);
    if (sizeof(TV) == sizeof(double)) {
        hipLaunchKernelGGL((k_matvec<DIM, TV, double>), dim3(G), dim3(CH_BLOCK), 0, s, b.ctl, Vk,
                           static_cast<const double*>(y), W, V, k, ps.out(), g.n, g.eps2, g.inv_h2, g.eyre);
    } else {
        hipLaunchKernelGGL((k_matvec<DIM, TV, float>), dim3(G), dim3(CH_BLOCK), 0, s, b.ctl, Vk,
                           static_cast<const float*>(y), W, V, k, ps.out(), g.n, g.eps2, g.inv_h2, g.eyre);
    }
    ps.produced(G);
    return hipGetLastError();
}

hipError_t launch_matvec(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, const double* y, int k,
                         hipStream_t s) {
    if (prec == CH_FP64)
        return g.dim == 2 ? launch_matvec_t<2, double>(g, b, ps, y, k, s)
                          : launch_matvec_t<3, double>(g, b, ps, y, k, s);
    return g.dim == 2 ? launch_matvec_t<2, float>(g, b, ps, b.y32, k, s)
                      : launch_matvec_t<3, float>(g, b, ps, b.y32, k, s);
}

template <int DIM, typename TV>
static hipError_t launch_resid_t(const Grid& g, const DevBuffers& b, PartSeq& ps, const double* y, const double* z,
                                 bool write_f, bool write_y32, hipStream_t s) {
    const int G = stencil_grid<DIM>(g.n);
    hipLaunchKernelGGL((k_resid<DIM, TV>), dim3(G), dim3(CH_BLOCK), 0, s, b.ctl, y, z, write_f ? b.fcur : nullptr,
                       static_cast<TV*>(b.V), write_y32 ? b.y32 : nullptr, ps.out(), g.n, g.eps2, g.inv_h2, g.eyre);
    ps.produced(G);
    return hipGetLastError();
}

hipError_t launch_resid(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, const double* y, const double* z,
                        bool write_f, bool write_y32, hipStream_t s) {
    if (prec == CH_FP64)
        return g.dim == 2 ? launch_resid_t<2, double>(g, b, ps, y, z, write_f, false, s)
                          : launch_resid_t<3, double>(g, b, ps, y, z, write_f, false, s);
    return g.dim == 2 ? launch_resid_t<2, float>(g, b, ps, y, z, write_f, write_y32, s)
                      : launch_resid_t<3, float>(g, b, ps, y, z, write_f, write_y32, s);
}

template <int DIM, typename TV>
static hipError_t launch_est_ee_t(const Grid& g, const DevBuffers& b, PartSeq& ps, const double* y0,
                                  const double* y1, float* y32, hipStream_t s) {
    const int G = stencil_grid<DIM>(g.n);
    hipLaunchKernelGGL((k_est_ee<DIM, TV>), dim3(G), dim3(CH_BLOCK), 0, s, b.ctl, y0, y1, b.fcur,
                       static_cast<TV*>(b.V), y32, ps.out(), g.n, g.eps2, g.inv_h2, g.eyre);
    ps.produced(G);
    return hipGetLastError();
}

hipError_t launch_est_ee(const Grid& g, int prec, const DevBuffers& b, PartSeq& ps, const double* y0,
                         const double* y1, hipStream_t s) {
    if (prec == CH_FP64)
        return g.dim == 2 ? launch_est_ee_t<2, double>(g, b, ps, y0, y1, nullptr, s)
                          : launch_est_ee_t<3, double>(g, b, ps, y0, y1, nullptr, s);
    return g.dim == 2 ? launch_est_ee_t<2, float>(g, b, ps, y0, y1, b.y32, s)
                      : launch_est_ee_t<3, float>(g, b, ps, y0, y1, b.y32, s);
}

hipError_t launch_lim_stage(const Grid& g, const DevBuffers& b, const double* y, const double* z, double* out,
                            int m, hipStream_t s) {
    if (g.dim == 2)
        hipLaunchKernelGGL((k_lim_stage<2>), dim3(stencil_grid<2>(g.n)), dim3(CH_BLOCK), 0, s, b.ctl, y, z, out, m,
                           g.n, g.eps2, g.inv_h2, g.eyre);
    else
        hipLaunchKernelGGL((k_lim_stage<3>), dim3(stencil_grid<3>(g.n)), dim3(CH_BLOCK), 0, s, b.ctl, y, z, out, m,
                           g.n, g.eps2, g.inv_h2, g.eyre);
    return hipGetLastError();
}

hipError_t launch_est_lim(const Grid& g, const DevBuffers& b, PartSeq& ps, const double* y0, const double* y1,
                          hipStream_t s) {
    int G;
    if (g.dim == 2) {
        G = stencil_grid<2>(g.n);
        hipLaunchKernelGGL((k_est_lim<2>), dim3(G), dim3(CH_BLOCK), 0, s, b.ctl, y0, y1, ps.out(), g.n, g.eps2,
                           g.inv_h2);
    } else {
        G = stencil_grid<3>(g.n);
        hipLaunchKernelGGL((k_est_lim<3>), dim3(G), dim3(CH_BLOCK), 0, s, b.ctl, y0, y1, ps.out(), g.n, g.eps2,
                           g.inv_h2);
    }
    ps.produced(G);
    return hipGetLastError();
}
