// Stencil kernels of one basis degree and one boundary condition: the build compiles this unit once
// per (TBS_DEGREE, TBS_BC) pair, so the fifteen kernel sets compile in parallel.
#include "stencil_kernel.h"

#if !defined(TBS_DEGREE) || !defined(TBS_BC)
#error "compile with -DTBS_DEGREE=<1..5> -DTBS_BC=<BC_PERIODIC|BC_DIRICHLET|BC_ROBIN>"
#endif

TBS_STENCIL_INSTANTIATE(TBS_DEGREE, tbs::TBS_BC)
