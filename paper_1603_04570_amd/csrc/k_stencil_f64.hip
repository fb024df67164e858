// Streaming node-stencil kernels: host-side shape tables and the FP64
// instantiations.
#define OKD_STENCIL_PART 0
#include "k_stencil_impl.h"
