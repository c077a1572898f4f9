// Shared device/host definitions of the tensor B-spline library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tbs {

// One-sided taps k = 0..n (symmetric filters) and the axis weights a_d = tau / h_d^2.
struct Taps {
  double m[6];
  double s[6];
  double ax, ay, az, tau;
};

// Device-resident solver scalars (written only by the single-block finalize kernels).
struct Scalars {
  double rr;      // r.r of the current recursive residual
  double pq;      // p.Ap of the current iteration
  double alpha;   // rr / pq of the last completed CG1
  double beta;    // rr_new / rr
  double bb;      // b.b
  double tol2;    // rtol^2 * b.b
  double rr0;     // r.r at start
  double out;     // scratch result (dot, norms)
  double out2;
  double alpha2;  // alpha of iteration nit-2 (one-kernel FP32 CG, two pending updates)
  int done;       // 1: converged, breakdown or trivial system -> every CG kernel returns at once
  int nit;        // completed CG iterations
  int status;     // 0 ok, -4 breakdown
  // x updates still to apply: 1 = alpha p_{nit-1}; 2 (one-kernel FP32 CG, which advances x every
  // second iteration) = alpha2 p_{nit-2}, then alpha p_{nit-1}
  int pending;
  // 1: x is zero and not read (set by FIN_INIT_XZERO; the first x update writes it, the x-update
  // kernels and the refinement update take it as zero until then)
  int xzero;
};
static_assert(sizeof(Scalars) <= 256, "a Scalars slot of the workspace is 256 bytes");

// CG1: one half of a Hestenes-Stiefel iteration (p, x update, q = A p, p.q); CGF: a whole iteration
// in one kernel (r update, p, x update, q = A p and the dot products p.q, r.q, q.q, r.r); RHSRES:
// the right-hand side b = M u of a source-free step and its residual r = b - A u in one pass.
enum Mode { M_APPLY = 0, M_RHS = 1, M_CG1 = 2, M_RESID = 3, M_CGF = 4, M_RHSRES = 5 };
enum Bc { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_ROBIN = 2 };

// Robin / penalty boundary on a box (BC_ROBIN): every 1-D factor of the operator is the truncated
// Toeplitz band plus a z x z corner block at each end (the high end mirrors the low end: row N-1-r,
// column N-1-c holds entry [r][c]).  cm: mass corner; cvx: corner of the x-pass's (Mx + Wx);
// cwy, cwz: corners of Wy, Wz; W_d = tau (h_d^-2 K_d + h_d^-1 E_d / (2 gamma)).  Row-major z x z.
constexpr int kRobinMaxZ = 5;
struct RobinCorner {
  int z;
  double cm[kRobinMaxZ * kRobinMaxZ];
  double cvx[kRobinMaxZ * kRobinMaxZ];
  double cwy[kRobinMaxZ * kRobinMaxZ];
  double cwz[kRobinMaxZ * kRobinMaxZ];
};

struct StencilArgs {
  int nx, ny, nz, zc;          // grid size and planes per z-chunk
  int tiles_x, tiles_y, nchunks, nblocks;
  Taps t;
  const void* in0;             // APPLY: u  RHS: u_prev  CG1: r  RESID: x
  const void* in1;             // RHS: q (nullable)  CG1, CGF: p_old
  const void* in2;             // CGF: q_old
  void* out0;                  // APPLY: y  RHS: b  CG1, CGF: q  RESID: r (nullable)
  void* out1;                  // CG1, CGF: p_new  RHSRES: b (f64)
  void* out2;                  // CGF: r_new
  void* io0;                   // CG1, CGF: x (lazy update, nullable)
  const double* bvec;          // RESID: b (RHSRES: formed in the kernel)
  double* part0;               // per-block partial sums (CG1, CGF: p.q, RESID: r.r)
  double* part1;               // RESID: b.b  CGF: r.q
  double* part2;               // CGF: q.q
  double* part3;               // CGF: r.r (of r_new)
  const Scalars* scal;         // CG1, CGF: alpha, beta, done, pending
  int first;                   // CG1, CGF: first iteration (p = r)
  int order;                   // tile order: 0 x-tiles fastest, 1 y-tiles fastest
  int nt_store;                // 1: outputs written with non-temporal stores
  RobinCorner rb;              // BC_ROBIN corner blocks
  double rscale;               // RESID: factor (a power of two) on the stored residual and its sums
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Round-to-nearest-even float -> bf16 on the bit pattern; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T> struct Io;
template <> struct Io<double> {
  template <typename Tc> __device__ static Tc ld(const void* p, int64_t i) { return (Tc)((const double*)p)[i]; }
  template <typename Tc> __device__ static void st(void* p, int64_t i, Tc v) { ((double*)p)[i] = (double)v; }
  template <typename Tc> __device__ static void st_nt(void* p, int64_t i, Tc v) {
    __builtin_nontemporal_store((double)v, (double*)p + i);
  }
};
template <> struct Io<float> {
  template <typename Tc> __device__ static Tc ld(const void* p, int64_t i) { return (Tc)((const float*)p)[i]; }
  template <typename Tc> __device__ static void st(void* p, int64_t i, Tc v) { ((float*)p)[i] = (float)v; }
  template <typename Tc> __device__ static void st_nt(void* p, int64_t i, Tc v) {
    __builtin_nontemporal_store((float)v, (float*)p + i);
  }
};
template <> struct Io<uint16_t> {  // bf16 storage
  template <typename Tc> __device__ static Tc ld(const void* p, int64_t i) {
    return (Tc)bf16_to_f32(((const uint16_t*)p)[i]);
  }
  template <typename Tc> __device__ static void st(void* p, int64_t i, Tc v) {
    ((uint16_t*)p)[i] = f32_to_bf16((float)v);
  }
  template <typename Tc> __device__ static void st_nt(void* p, int64_t i, Tc v) { st<Tc>(p, i, v); }
};

// Round a compute value to what the storage type keeps (identity except for bf16).
template <typename Ts, typename Tc> __device__ __forceinline__ Tc storage_round(Tc v) { return v; }
template <> __device__ __forceinline__ float storage_round<uint16_t, float>(float v) {
  return bf16_to_f32(f32_to_bf16(v));
}

// Wave-64 sum of doubles through cross-lane shuffles (fixed butterfly order: deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-to-tile map that keeps consecutive logical tiles on one XCD (blocks are dealt to the
// 8 XCDs round-robin, so block b runs on XCD b % 8).  Bijective for any G.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3, rem = G & 7;
  const int x = b & 7, i = b >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + i;
}

}  // namespace tbs
