// Host-side helpers shared by the plan and batch parts of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "grf.h"

namespace grf {
namespace host {

extern thread_local std::string g_err;
grf_status fail(grf_status st, const std::string& msg);
grf_status hip_fail(hipError_t e, const char* what);
bool smooth235(long long n);
// W_L[i] = exp(2 pi i i / L) as interleaved (re, im) float64 values.
void table_values(int L, std::vector<double>& w);
// Device copy of W_L in float32 (dtype 0) or float64 (dtype 1).
grf_status make_table(int L, int dtype, void** out);

}  // namespace host
}  // namespace grf
