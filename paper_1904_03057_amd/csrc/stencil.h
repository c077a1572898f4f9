// Launchers of the stencil tile engine and the vector/reduction kernels (host-callable).
#pragma once
#include "common.h"

#ifndef STENCIL_TY
#define STENCIL_TY 16
#endif
#ifndef STENCIL_APPLY_WX
#define STENCIL_APPLY_WX 1
#endif

#ifndef STENCIL_CG_TY
#define STENCIL_CG_TY 16
#endif
#ifndef STENCIL_CGF_TY
#define STENCIL_CGF_TY 48
#endif
#ifndef STENCIL_CG_PF
#define STENCIL_CG_PF 1
#endif
#ifndef STENCIL_RESID_TY
#define STENCIL_RESID_TY 16
#endif
#ifndef STENCIL_RESID_WY
#define STENCIL_RESID_WY 8
#endif
#ifndef STENCIL_F64_WY
#define STENCIL_F64_WY 8
#endif

namespace tbs {

constexpr int kTileX = 64;
constexpr int imin(int a, int b) { return a < b ? a : b; }
// smallest tile height of any stencil launch (the one-kernel CG iteration takes 16 rows or more in
// FP32, 8 or 16 in FP64): sizes the partial-sum buffers
constexpr int kTileY = imin(imin(STENCIL_RESID_TY, STENCIL_TY), imin(STENCIL_CG_TY, 8));
constexpr int kTileYPlan = 16;  // tile height the z-chunk plan assumes
constexpr int kLdsMax = 160 * 1024;  // LDS one workgroup may hold on gfx950

// Rows per row wave of the one-kernel CG iteration: four in FP32, two in FP64.
constexpr int cgf_rows_per_wave(int es) { return es == 4 ? 4 : 2; }

// LDS of the one-kernel CG iteration (degree n, tile height ty, 64 columns, es-byte compute type):
// staged plane (x halo of at most 8 columns a side: one 16-byte vector of bf16), the two x-pass
// planes, the p and r rings, the reduction slots, and the Robin corner tables and z-accumulators
// (one-element placeholders otherwise).  An upper bound of what the kernel declares (it asserts so).
constexpr int cgf_lds_bytes(int n, int ty, int bc, int es) {
  return es * ((ty + 2 * n) * (64 + 16) + 2 * (ty + 2 * n) * 64 + (2 * n + 3) * ty * 64) +
         8 * 4 * (ty / cgf_rows_per_wave(es)) +
         (bc == BC_ROBIN ? es * (4 * kRobinMaxZ * kRobinMaxZ + (2 * (n / 2) + 1) * ty * 64) : 2 * es);
}

// The one-kernel CG iteration's tile height: in FP32 the tallest of STENCIL_CGF_TY, 32 and 16 rows
// whose LDS fits one workgroup (row waves of four rows each: the registers per thread do not grow
// with the height, and a taller tile re-reads fewer halo rows of r, q and p); in FP64 16 rows, or 8
// where 16 do not fit (Robin quartic and quintic).
constexpr int cgf_tile_y(int n, int bc, int es) {
  return es == 4 ? (cgf_lds_bytes(n, STENCIL_CGF_TY, bc, 4) <= kLdsMax
                        ? STENCIL_CGF_TY
                        : (cgf_lds_bytes(n, 32, bc, 4) <= kLdsMax ? 32 : 16))
                 : (cgf_lds_bytes(n, 16, bc, 8) <= kLdsMax ? 16 : 8);
}

// Tile height per (mode, compute precision, degree, boundary): taller tiles re-read fewer halo
// rows.  The FP64 kernels take 16 rows in eight row waves of two rows (the FP64 ring and column
// windows of two rows leave room for more waves per SIMD than four rows in four waves).
constexpr int stencil_tile_y(int mode, int compute_bytes, int n, int bc) {
  return compute_bytes == 4
             ? ((mode == M_APPLY) ? 32
                                  : (mode == M_CG1 ? STENCIL_CG_TY : (mode == M_CGF ? cgf_tile_y(n, bc, 4) : 16)))
             : ((mode == M_RESID || mode == M_RHSRES) ? STENCIL_RESID_TY : (mode == M_CGF ? cgf_tile_y(n, bc, 8) : 16));
}
// Row waves per workgroup: four for the FP32 kernels, except the one-kernel CG iteration, whose
// waves keep four rows each (two in FP64); eight for the other FP64 kernels.
constexpr int stencil_tile_wy(int mode, int compute_bytes, int n, int bc) {
  return mode == M_CGF ? stencil_tile_y(mode, compute_bytes, n, bc) / cgf_rows_per_wave(compute_bytes)
                       : ((mode == M_RESID || mode == M_RHSRES) ? STENCIL_RESID_WY
                                                                   : (compute_bytes == 8 ? STENCIL_F64_WY : 4));
}
// One stencil launch of degree N for a (mode, input, compute, output) type combination and
// boundary condition BC; defined in stencil_kernel.h and instantiated per degree and boundary
// condition by stencil_inst.hip.
template <int N, int MODE, typename Tin, typename Tc, typename Tout, int BC>
hipError_t launch_bcx(const StencilArgs& a, bool vec, hipStream_t st);

template <int N, int BC>
hipError_t launch_rhsres_bc(const StencilArgs& a, bool vec, hipStream_t st);

template <int N, int MODE, typename Tin, typename Tc, typename Tout>
inline hipError_t launch_bc(const StencilArgs& a, int bc, bool vec, hipStream_t st) {
  if (bc == BC_PERIODIC) return launch_bcx<N, MODE, Tin, Tc, Tout, BC_PERIODIC>(a, vec, st);
  if (bc == BC_ROBIN) return launch_bcx<N, MODE, Tin, Tc, Tout, BC_ROBIN>(a, vec, st);
  return launch_bcx<N, MODE, Tin, Tc, Tout, BC_DIRICHLET>(a, vec, st);
}

// Number of workgroups (= partial sums written) of a stencil launch of this mode.
int stencil_blocks(const StencilArgs& a, int mode, int compute_bytes, int n, int bc);

// stencil.hip
hipError_t launch_apply(const StencilArgs& a, int n, int bc, int in_dt, int out_dt, hipStream_t st);
hipError_t launch_rhs(const StencilArgs& a, int n, int bc, int dt, hipStream_t st);
hipError_t launch_cg1(const StencilArgs& a, int n, int bc, int dt, hipStream_t st);
// CGF (one-kernel CG iteration): dt = 1 (all f32), 2 (f32 with p stored as bf16)
hipError_t launch_cgf(const StencilArgs& a, int n, int bc, int dt, hipStream_t st);
hipError_t launch_resid(const StencilArgs& a, int n, int bc, int r_dt, hipStream_t st);
// RHSRES: u (f64, in0) -> b = M u (f64, out1) and r = (b - A u) rscale (f32, out0), with the partial
// sums of r.r and (b rscale).(b rscale); periodic and Dirichlet only (hipErrorInvalidValue on Robin)
hipError_t launch_rhs_resid(const StencilArgs& a, int n, int bc, hipStream_t st);

// vector.hip
constexpr int kVecBlocks = 2048;   // grid of the elementwise kernels (= partial sums they write)
hipError_t launch_cg2(void* r, const void* q, int64_t n, int dt, double* part, const Scalars* s, hipStream_t st);
hipError_t launch_sub_norm(void* r, const void* b, const void* q, int64_t n, int dt, double* p0, double* p1,
                           hipStream_t st);
hipError_t launch_flush(void* x, const void* p0, const void* p1, int64_t n, int dt, const Scalars* s, hipStream_t st);
hipError_t launch_dot(const void* a, const void* b, int64_t n, int dt, double* part, hipStream_t st);
hipError_t launch_convert(const void* src, int sdt, void* dst, int ddt, int64_t n, hipStream_t st);
hipError_t launch_add_f32_to_f64(double* x, const float* d, int64_t n, hipStream_t st);
hipError_t launch_fill(void* x, int dt, int64_t n, hipStream_t st);  // zero fill
hipError_t launch_stream_copy(const void* src, void* dst, int64_t nbytes, hipStream_t st);
hipError_t launch_guess_combine(double* x, const double* u, const float* du, int64_t n, double scale,
                                hipStream_t st);  // x = u + scale du

// finalize kernels (single block, fixed-order reduction of partial sums)
enum FinOp { FIN_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_DOT = 3, FIN_NORMS = 4, FIN_CLEAR_PENDING = 5,
             FIN_FUSED = 6, FIN_INIT_XZERO = 7 };  // FIN_INIT_XZERO: FIN_INIT for x = 0 left unwritten
// Reduces the per-block partial sums p0 (and p1, p2, p3 where the op uses them) in a fixed order
// and updates the CG scalars.  FIN_FUSED takes p.q, r.q, q.q and r.r of a CGF launch.
hipError_t launch_finalize(int op, const double* p0, const double* p1, int count, Scalars* s, double rtol,
                           hipStream_t st, const double* p2 = nullptr, const double* p3 = nullptr);
// out[0] = sqrt(s->out), out[1] = sqrt(s->out2) (the norms of a FIN_NORMS reduction) in device memory
hipError_t launch_norms_out(const Scalars* s, double* out, hipStream_t st);

}  // namespace tbs
