// FP32 (mixed-precision path) instantiations of the residual kernels.
#define KT float
#define KSUF f32
#include "kernels_t.inc"
