// Dispatch of the stencil launches: (mode, dtype) combinations, basis degree n and boundary -> the
// kernel instances of stencil_kernel.h that stencil_inst.hip compiles per degree and boundary.
#include "common.h"
#include "stencil.h"

namespace tbs {

template <int MODE, typename Tin, typename Tc, typename Tout>
static hipError_t launch_n(const StencilArgs& a, int n, int bc, hipStream_t st) {
  // 16-byte vector staging needs rows made of whole vectors: Nx divisible by the vector width
  constexpr int ve = 16 / sizeof(Tin);
  const bool vec = (a.nx % ve) == 0;
  switch (n) {
    case 1: return launch_bc<1, MODE, Tin, Tc, Tout>(a, bc, vec, st);
    case 2: return launch_bc<2, MODE, Tin, Tc, Tout>(a, bc, vec, st);
    case 3: return launch_bc<3, MODE, Tin, Tc, Tout>(a, bc, vec, st);
    case 4: return launch_bc<4, MODE, Tin, Tc, Tout>(a, bc, vec, st);
    case 5: return launch_bc<5, MODE, Tin, Tc, Tout>(a, bc, vec, st);
  }
  return hipErrorInvalidValue;
}

int stencil_blocks(const StencilArgs& a, int mode, int compute_bytes, int n, int bc) {
  const int ty = stencil_tile_y(mode, compute_bytes, n, bc);
  const int wx = (mode == M_APPLY && compute_bytes == 4) ? STENCIL_APPLY_WX : 1;
  return ((a.nx + 64 * wx - 1) / (64 * wx)) * ((a.ny + ty - 1) / ty) * a.nchunks;
}

// dtype codes: 0 = f64, 1 = f32, 2 = bf16
hipError_t launch_apply(const StencilArgs& a, int n, int bc, int in_dt, int out_dt, hipStream_t st) {
  if (in_dt == 0 && out_dt == 0) return launch_n<M_APPLY, double, double, double>(a, n, bc, st);
  if (in_dt == 1 && out_dt == 1) return launch_n<M_APPLY, float, float, float>(a, n, bc, st);
  if (in_dt == 2 && out_dt == 1) return launch_n<M_APPLY, uint16_t, float, float>(a, n, bc, st);
  if (in_dt == 1 && out_dt == 0) return launch_n<M_APPLY, float, double, double>(a, n, bc, st);
  if (in_dt == 2 && out_dt == 0) return launch_n<M_APPLY, uint16_t, double, double>(a, n, bc, st);
  return hipErrorInvalidValue;
}

hipError_t launch_rhs(const StencilArgs& a, int n, int bc, int dt, hipStream_t st) {
  if (dt == 0) return launch_n<M_RHS, double, double, double>(a, n, bc, st);
  if (dt == 1) return launch_n<M_RHS, float, float, float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

// CG1: dt = 0 (all f64), 1 (all f32), 2 (f32 with p stored as bf16)
hipError_t launch_cg1(const StencilArgs& a, int n, int bc, int dt, hipStream_t st) {
  if (dt == 0) return launch_n<M_CG1, double, double, double>(a, n, bc, st);
  if (dt == 1) return launch_n<M_CG1, float, float, float>(a, n, bc, st);
  if (dt == 2) return launch_n<M_CG1, uint16_t, float, float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

hipError_t launch_cgf(const StencilArgs& a, int n, int bc, int dt, hipStream_t st) {
  if (dt == 0) return launch_n<M_CGF, double, double, double>(a, n, bc, st);
  if (dt == 1) return launch_n<M_CGF, float, float, float>(a, n, bc, st);
  if (dt == 2) return launch_n<M_CGF, uint16_t, float, float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

// RESID: FP64 x and b; r written as f64 (r_dt 0) or f32 (r_dt 1) when out0 != NULL
hipError_t launch_resid(const StencilArgs& a, int n, int bc, int r_dt, hipStream_t st) {
  if (r_dt == 0) return launch_n<M_RESID, double, double, double>(a, n, bc, st);
  if (r_dt == 1) return launch_n<M_RESID, double, double, float>(a, n, bc, st);
  return hipErrorInvalidValue;
}

hipError_t launch_rhs_resid(const StencilArgs& a, int n, int bc, hipStream_t st) {
  const bool vec = (a.nx % 2) == 0;  // 16-byte staging of the FP64 input
  if (bc == BC_ROBIN) return hipErrorInvalidValue;
  const bool per = bc == BC_PERIODIC;
  switch (n) {
    case 1: return per ? launch_rhsres_bc<1, BC_PERIODIC>(a, vec, st) : launch_rhsres_bc<1, BC_DIRICHLET>(a, vec, st);
    case 2: return per ? launch_rhsres_bc<2, BC_PERIODIC>(a, vec, st) : launch_rhsres_bc<2, BC_DIRICHLET>(a, vec, st);
    case 3: return per ? launch_rhsres_bc<3, BC_PERIODIC>(a, vec, st) : launch_rhsres_bc<3, BC_DIRICHLET>(a, vec, st);
    case 4: return per ? launch_rhsres_bc<4, BC_PERIODIC>(a, vec, st) : launch_rhsres_bc<4, BC_DIRICHLET>(a, vec, st);
    case 5: return per ? launch_rhsres_bc<5, BC_PERIODIC>(a, vec, st) : launch_rhsres_bc<5, BC_DIRICHLET>(a, vec, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tbs
