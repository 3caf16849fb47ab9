// Launchers of the 3-D marching kernels declared outside ch_internal.h.
#pragma once

#include "ch_internal.h"

// Rows (y) of the x-y block of a marching workgroup: 8 in FP64 (two x per
// thread), 16 in FP32 (four x per thread); the block is 64 wide.
constexpr int march_rows(int prec) { return prec == CH_FP64 ? 8 : 16; }

// Planes per z-run of the FP32 DCGS2 matvec: of the lengths CH_MARCH_L ..
// 2 CH_MARCH_L, the one whose work items (64 x 16 blocks times runs) fill the
// largest share of whole rounds of co-resident workgroups, the shorter on
// ties.  The kernel holds three workgroups per CU at its register count, so
// 256 CUs hold 768: at 256^3 runs of 16 give 1024 items (a second round a
// third full), runs of 22 give 768.  Only while every item has a workgroup
// of its own at CH_MARCH_L (at most CH_WBLK_MAX items): beyond that the
// workgroups loop over items, rounds no longer follow the item count, and
// longer runs were slower (384^3, 512^3).  FP64 (four workgroups per CU;
// 2048 items at 256^3) and the LIM kernels take CH_MARCH_L.
constexpr unsigned MARCH_SLOTS_FP32 = 256u * 3u;

__host__ __device__ inline int march_len_fp32(int n) {
    const unsigned nxy = (unsigned)((n + 63) / 64) * (unsigned)((n + 15) / 16);
    if ((unsigned long long)nxy * (unsigned)((n + CH_MARCH_L - 1) / CH_MARCH_L) > CH_WBLK_MAX) return CH_MARCH_L;
    int best = CH_MARCH_L;
    unsigned long long bi = 0, br = 1;   // items and rounds of the best length so far
#pragma unroll
    for (int L = CH_MARCH_L; L <= 2 * CH_MARCH_L; ++L) {
        const unsigned long long items = (unsigned long long)nxy * (unsigned)((n + L - 1) / L);
        const unsigned long long rounds = (items + MARCH_SLOTS_FP32 - 1) / MARCH_SLOTS_FP32;
        if (items * br > bi * rounds) {
            best = L;
            bi = items;
            br = rounds;
        }
    }
    return best;
}

// 3-D estimate pass of EE2 on z-marching x-y tiles (ch_march.hip): f(y^{n+1})
// into the field f and basis column 0 (and the FP32 copy of y^{n+1} in the
// mixed form), with the partials of the estimate sums and of ||f||^2 and
// ||ghat||^2 over the instance's wblk range (partials of kind PK_STRIP).
hipError_t launch_est_march(const Table& t, int prec, const DevBuffers& b, const double* y0, const double* y1,
                            double* pout, hipStream_t s);

// 3-D LIM stage launch l (one stage of Fig. 1) on z-marching x-y tiles
// (ch_march.hip), with the launch bookkeeping of lim_launch.
hipError_t launch_lim_stage_march(const Table& t, const DevBuffers& b, const double* yin, double* yout, int l,
                                  bool timing, hipStream_t s);

// 3-D LIM estimate (eq. LIMest) on z-marching x-y tiles (ch_march.hip):
// partials of ||y^{n+1} - y_PC||^2 and ||y_PC||^2 over the instance's wblk
// range (partials of kind PK_STRIP).
hipError_t launch_est_lim_march(const Table& t, const DevBuffers& b, const double* y0, const double* y1, double* pout,
                                hipStream_t s);
