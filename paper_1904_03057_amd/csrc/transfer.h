// Two-scale transfer between a grid and its halved grid (coarse-grid initial guess).
#pragma once
#include <hip/hip_runtime.h>

namespace tbs {

// One separable pass (prolongation coarse -> fine, or its adjoint, the restriction) along `axis`
// (0 x, 1 y, 2 z) of an FP64 array [z][y][x]; odims = output dimensions, nin = input length along
// the axis, n = odd spline degree, out = scale * result (accumulate: out += scale * result).
hipError_t launch_transfer(const double* in, double* out, const int odims[3], int nin, int axis, int prolong,
                           int periodic, int n, double scale, int accumulate, hipStream_t st);

}  // namespace tbs
