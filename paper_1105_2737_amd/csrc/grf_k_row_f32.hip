// row_f32 instantiations
#define GRF_T float
#define GRF_SUFFIX f32
#define GRF_ROWS 1
#include "grf_inst.inc"
