// Launcher of the refinement update that closes an inner FP32 CG solve (host-callable).
#pragma once
#include "common.h"

namespace tbs {

// out = base + scale (double)(d + alpha p_{nit-1}) with the inner solve's pending update applied in
// FP32 exactly as the CG flush would apply it to d (alpha, nit and the pending flag are read from s
// on the device); p_{nit-1} = (nit odd ? p1 : p0), dt 1 (FP32 p) or 2 (bf16 p).  out may equal base.
hipError_t launch_refine_add(double* out, const double* base, const float* d, const void* p0, const void* p1,
                             int64_t n, int dt, const Scalars* s, double scale, hipStream_t st);

}  // namespace tbs
