// Launchers of the 3-D marching kernels declared outside ch_internal.h.
#pragma once

#include "ch_internal.h"

// Rows (y) of the x-y block of a marching workgroup: 8 in FP64 (two x per
// thread), 16 in FP32 (four x per thread); the block is 64 wide.
constexpr int march_rows(int prec) { return prec == CH_FP64 ? 8 : 16; }

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
