// Internal interface between the solver driver and the learned-guess network.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tbs.h"

// Computes the network's guess of u^{k+1} - u^k for (u_prev, q) (FP64 device arrays, q nullable)
// into the network's own output buffer and returns a device pointer to it (FP32, N values).
int tbs_net_guess_internal(tbs_net* net, const int64_t grid[3], int periodic, double tau, hipStream_t st,
                           const double* u_prev, const double* q, const float** du_out);
