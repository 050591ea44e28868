// reflecting-boundary kernels, float64
#define GRF_T double
#define GRF_SUFFIX f64
#include "grf_inst_r2r.inc"
