// reflecting-boundary kernels, float32
#define GRF_T float
#define GRF_SUFFIX f32
#include "grf_inst_r2r.inc"
