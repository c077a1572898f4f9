// Two-scale transfer between a grid and its halved grid, for the coarse-grid initial guess (the
// reduced-grid start of the Sec. 3 leg example).  For odd degree n the coarse B-spline space lies
// inside the fine one (two-scale relation, from the convolution row of Table 1):
//   prolongation  fine c_i   = sum_j C_j w_{i - p(j)}
//   restriction   coarse F_j = sum_k w_k f_{p(j) + k}      (the adjoint)
// with w_k = C(n+1, k + (n+1)/2) / 2^n, |k| <= (n+1)/2, and p(j) = 2j + 1 on a Dirichlet grid
// (coefficients that would fall outside the box are dropped), 2j on an even periodic grid.  Each
// launch is one separable pass along one axis of an FP64 array [z][y][x]; one thread per output
// element gathers its (at most n + 2) inputs, so no atomics and a fixed summation order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "transfer.h"

namespace tbs {

struct TransferArgs {
  const double* in;
  double* out;
  int ox, oy, oz;     // output dimensions (x, y, z)
  int nin;            // input length along the axis (the other two match the output)
  int axis;           // 0 x, 1 y, 2 z
  int prolong;        // 1 coarse -> fine, 0 fine -> coarse
  int off;            // p(j) = 2 j + off
  int periodic;
  int H;              // (n + 1) / 2
  double w[7];        // w[k + H]
  double scale;
  int accumulate;     // 1: out += result
};

__global__ __launch_bounds__(256) void transfer_kernel(TransferArgs a) {
  const int64_t total = (int64_t)a.ox * a.oy * a.oz;
  const int64_t ix = a.axis == 0 ? a.nin : a.ox;
  const int64_t iy = a.axis == 1 ? a.nin : a.oy;
  const int64_t stride = a.axis == 0 ? 1 : (a.axis == 1 ? ix : ix * iy);
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int x = (int)(t % a.ox);
    const int64_t rest = t / a.ox;
    const int y = (int)(rest % a.oy);
    const int z = (int)(rest / a.oy);
    const int o = a.axis == 0 ? x : (a.axis == 1 ? y : z);
    const int64_t base = (int64_t)(a.axis == 2 ? 0 : z) * ix * iy + (int64_t)(a.axis == 1 ? 0 : y) * ix +
                         (a.axis == 0 ? 0 : x);
    double acc = 0.0;
    for (int k = -a.H; k <= a.H; ++k) {
      int src;
      if (a.prolong) {  // fine o receives coarse j with 2 j + off + k = o
        int tt = o - a.off - k;
        if (a.periodic) {
          const int nf = 2 * a.nin;
          tt = ((tt % nf) + nf) % nf;
        }
        if (tt < 0 || (tt & 1)) continue;
        src = tt >> 1;
        if (src >= a.nin) continue;
      } else {  // coarse o gathers fine i = 2 o + off + k
        int i = 2 * o + a.off + k;
        if (a.periodic) {
          i = ((i % a.nin) + a.nin) % a.nin;
        } else if (i < 0 || i >= a.nin) {
          continue;
        }
        src = i;
      }
      acc = fma(a.w[k + a.H], a.in[base + (int64_t)src * stride], acc);
    }
    acc *= a.scale;
    a.out[t] = a.accumulate ? a.out[t] + acc : acc;
  }
}

hipError_t launch_transfer(const double* in, double* out, const int odims[3], int nin, int axis, int prolong,
                           int periodic, int n, double scale, int accumulate, hipStream_t st) {
  TransferArgs a{};
  a.in = in;
  a.out = out;
  a.ox = odims[0];
  a.oy = odims[1];
  a.oz = odims[2];
  a.nin = nin;
  a.axis = axis;
  a.prolong = prolong;
  a.off = periodic ? 0 : 1;
  a.periodic = periodic;
  a.H = (n + 1) / 2;
  double binom = 1.0;  // C(n+1, m), m = 0..n+1
  for (int m = 0; m <= n + 1; ++m) {
    a.w[m] = binom / (double)(1 << n);
    binom = binom * (n + 1 - m) / (m + 1);
  }
  a.scale = scale;
  a.accumulate = accumulate;
  const int64_t total = (int64_t)odims[0] * odims[1] * odims[2];
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(transfer_kernel, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace tbs
