// Streaming node-stencil kernels: the FP32 and mixed-precision
// instantiations.
#define OKD_STENCIL_PART 1
#include "k_stencil_impl.h"
