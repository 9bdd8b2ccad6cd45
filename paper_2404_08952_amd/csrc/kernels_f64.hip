// FP64 instantiations of the residual kernels.
#define KT double
#define KSUF f64
#include "kernels_t.inc"
