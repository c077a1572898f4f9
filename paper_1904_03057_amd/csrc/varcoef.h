// Variable-coefficient system operator (host-callable launcher and its argument block).
#pragma once
#include "common.h"

namespace tbs {

constexpr int kVcMaxQ = 8;   // Gauss points per cell and axis: ceil((3n + 1) / 2) <= 8 for n <= 5
constexpr int kVcMaxB = 6;   // B-splines per cell and axis: n + 1 <= 6

// One launch of F(c)_l = sum_k sum_m c_k (m_m f^{klm} + d_m w^{klm}) (all arrays [z][y][x]).
// bv[q][t], bd[q][t]: value and derivative of the t-th B-spline of a cell at its q-th Gauss point
// (unit cell), w[q]: the point's weight; ih2 = h_d^-2.
struct VarcoefArgs {
  int nx, ny, nz, zc;
  int tiles_x, tiles_y, nchunks, nblocks;
  const void* c;
  const void* d;
  const void* m;
  void* y;
  double bv[kVcMaxQ * kVcMaxB];
  double bd[kVcMaxQ * kVcMaxB];
  double w[kVcMaxQ];
  double ihx2, ihy2, ihz2;
};

// FP32 copies of the basis tables for the FP32 kernels (made on the host once per launch).
struct VarcoefTabF {
  float bv[kVcMaxQ * kVcMaxB];
  float bd[kVcMaxQ * kVcMaxB];
  float w[kVcMaxQ];
};

// Rows of outputs per wave (the y-extent of one strip).
constexpr int kVcTileY = 16;
// Output columns of one strip: the 64 lanes hold the strip's coefficient columns and an n-column halo.
constexpr int vc_tile_x(int n) { return 64 - 2 * n; }

// dt 0: FP64 arrays and arithmetic, 1: FP32.  bc: BC_PERIODIC or BC_DIRICHLET.
hipError_t launch_varcoef(const VarcoefArgs& a, int n, int bc, int dt, hipStream_t st);

}  // namespace tbs
