// row_f64 instantiations
#define GRF_T double
#define GRF_SUFFIX f64
#define GRF_ROWS 1
#include "grf_inst.inc"
