// Stencil kernels of basis degree 4 (one translation unit per degree).
#include "stencil_kernel.h"

TBS_STENCIL_INSTANTIATE(4)
