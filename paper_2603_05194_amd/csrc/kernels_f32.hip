// FP32 instantiations of the field kernels and their launch wrappers (the mixed-precision bulk
// phase). The same sources as kernels.hip, compiled as a unit of their own so that the FP64 and
// FP32 halves of the library build in parallel.
#define BEC_UNIT_F32 1
#include "kernels.hip"
