// Runtime-radix passes for transform lengths without a compile-time kernel:
// the radix plan generator, the workgroup geometry and the launches.
#include <algorithm>

#include "grf_dispatch.hpp"
#include "grf_generic.hpp"

namespace grf {

int radix_plan(int L, int* rad) {
  int n = L, e2 = 0, e3 = 0, e5 = 0;
  while (n % 2 == 0) { n /= 2; ++e2; }
  while (n % 3 == 0) { n /= 3; ++e3; }
  while (n % 5 == 0) { n /= 5; ++e5; }
  if (n != 1 || L < 1) return -1;
  int s = 0;
  while (e2 >= 3) { rad[s++] = 8; e2 -= 3; }
  if (e2 == 2) rad[s++] = 4;
  if (e2 == 1) rad[s++] = 2;
  while (e5-- > 0) rad[s++] = 5;
  while (e3-- > 0) rad[s++] = 3;
  return s;
}

namespace {

constexpr size_t kLdsBudget = 64 * 1024;        // two workgroups per CU
constexpr size_t kLdsMax = 160 * 1024;          // one workgroup's limit on gfx950

bool is_col(int pass) {
  return pass == PASS_COL_GEN_INV || pass == PASS_COL_LOAD_INV || pass == PASS_COL_LOAD_FWD;
}
bool is_row(int pass) {
  return pass == PASS_ROW_C2R || pass == PASS_ROW_R2C_GEN || pass == PASS_ROW_R2C_LOAD || pass == PASS_ROW_GEN_C2R;
}

template <typename T, int VPT>
hipError_t glaunch(int pass, const Args& a, long long nblocks, const GGeom& g, hipStream_t s) {
  const dim3 grid((unsigned)nblocks), block((unsigned)g.threads);
  const void* fn = nullptr;
  switch (pass) {
    case PASS_COL_GEN_INV: fn = reinterpret_cast<const void*>(&k_gcol<T, SRC_GEN, +1, VPT>); break;
    case PASS_COL_LOAD_INV: fn = reinterpret_cast<const void*>(&k_gcol<T, SRC_LOAD, +1, VPT>); break;
    case PASS_COL_LOAD_FWD: fn = reinterpret_cast<const void*>(&k_gcol<T, SRC_LOAD, -1, VPT>); break;
    case PASS_ROW_C2R: fn = reinterpret_cast<const void*>(&k_grow_c2r<T, SRC_LOAD, VPT>); break;
    case PASS_ROW_GEN_C2R: fn = reinterpret_cast<const void*>(&k_grow_c2r<T, SRC_GEN, VPT>); break;
    case PASS_ROW_R2C_GEN: fn = reinterpret_cast<const void*>(&k_grow_r2c<T, SRC_GEN, VPT>); break;
    case PASS_ROW_R2C_LOAD: fn = reinterpret_cast<const void*>(&k_grow_r2c<T, SRC_LOAD, VPT>); break;
    default: return hipErrorInvalidValue;
  }
  if (g.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds);
    if (e != hipSuccess) return e;
  }
  switch (pass) {
    case PASS_COL_GEN_INV: hipLaunchKernelGGL((k_gcol<T, SRC_GEN, +1, VPT>), grid, block, g.lds, s, a); break;
    case PASS_COL_LOAD_INV: hipLaunchKernelGGL((k_gcol<T, SRC_LOAD, +1, VPT>), grid, block, g.lds, s, a); break;
    case PASS_COL_LOAD_FWD: hipLaunchKernelGGL((k_gcol<T, SRC_LOAD, -1, VPT>), grid, block, g.lds, s, a); break;
    case PASS_ROW_C2R: hipLaunchKernelGGL((k_grow_c2r<T, SRC_LOAD, VPT>), grid, block, g.lds, s, a); break;
    case PASS_ROW_GEN_C2R: hipLaunchKernelGGL((k_grow_c2r<T, SRC_GEN, VPT>), grid, block, g.lds, s, a); break;
    case PASS_ROW_R2C_GEN: hipLaunchKernelGGL((k_grow_r2c<T, SRC_GEN, VPT>), grid, block, g.lds, s, a); break;
    default: hipLaunchKernelGGL((k_grow_r2c<T, SRC_LOAD, VPT>), grid, block, g.lds, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace

// Column passes: NT = ceil(L / vpt) threads per column, CP column pairs per
// workgroup sized so that the tile stays within 64 KB of LDS (at least one
// pair; a longer column takes one workgroup per CU), NT * CP <= 1024, and one
// padding slot per row when it fits.  Row passes: NT = ceil(M / vpt) threads per
// row, RB rows within 32 KB of LDS and 1024 threads, one padding element per
// row.  Limits: columns up to GRF_GENERIC_MAX_COL, half-rows up to
// GRF_GENERIC_MAX_ROW (the longest row takes one workgroup, 1024 threads).
GGeom generic_geom(int pass, int dtype, int L, int vpt) {
  GGeom g{};
  if (vpt != 4 && vpt != 8) return g;
  const size_t cplx = dtype == 0 ? 8 : 16;
  if (is_col(pass)) {
    if (L < 2 || L > GRF_GENERIC_MAX_COL) return g;
    g.nt = (L + vpt - 1) / vpt;
    const size_t pair = 2 * cplx;
    int cp = (int)std::max<size_t>(1, kLdsBudget / ((size_t)L * pair));
    cp = std::min(cp, 8);
    cp = std::min(cp, std::max(1, 1024 / g.nt));
    g.per_wg = cp;
    g.rs = ((size_t)L * (cp + 1) * pair <= std::max(kLdsBudget, (size_t)L * cp * pair)) ? cp + 1 : cp;
    g.lds = (size_t)L * g.rs * pair;
    g.threads = (g.nt * cp + 63) / 64 * 64;
  } else if (is_row(pass)) {
    const int M = L;
    if (M < 1 || M > GRF_GENERIC_MAX_ROW) return g;
    g.nt = (M + vpt - 1) / vpt;
    g.rs = M + 1;
    int rb = (int)std::max<size_t>(1, (32 * 1024) / ((size_t)g.rs * cplx));
    rb = std::min(rb, 16);
    rb = std::min(rb, std::max(1, 1024 / g.nt));
    g.per_wg = rb;
    g.lds = (size_t)rb * g.rs * cplx;
    g.threads = (g.nt * rb + 63) / 64 * 64;
  } else {
    return g;
  }
  if (g.lds > kLdsMax || g.threads > 1024) return GGeom{};
  return g;
}

hipError_t launch_generic(int pass, int dtype, const Args& a, long long nblocks, hipStream_t s) {
  const GGeom g = generic_geom(pass, dtype, a.gl, a.gvpt);
  if (g.threads <= 0) return hipErrorInvalidValue;
  if (a.gvpt == 4) return dtype == 0 ? glaunch<float, 4>(pass, a, nblocks, g, s) : glaunch<double, 4>(pass, a, nblocks, g, s);
  return dtype == 0 ? glaunch<float, 8>(pass, a, nblocks, g, s) : glaunch<double, 8>(pass, a, nblocks, g, s);
}

}  // namespace grf
