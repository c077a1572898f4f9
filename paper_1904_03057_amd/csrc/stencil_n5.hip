// Stencil kernels of basis degree 5 (one translation unit per degree).
#include "stencil_kernel.h"

TBS_STENCIL_INSTANTIATE(5)
