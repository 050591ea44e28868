// Instantiations of the last-axis pass that completes the column transform
// (RowXC2R) for the pairs of GRF_XC2R_PAIRS, with the radices of the column
// pass (ColCfg) and of the complex-to-real pass (RowCfg) of those lengths.
#include "grf_configs.hpp"
#include "grf_dispatch.hpp"
#include "grf_kernels.hpp"

namespace grf {

namespace {

template <typename T, int L, int M>
using XPass = RowXC2R<T, M, typename RowCfg<M>::Rad, L, ColCfg<L>::Rad::get(ColCfg<L>::Rad::count - 1)>;

template <typename T, int L, int M>
hipError_t xlaunch(const Args& a, long long nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_row_xc2r<T, M, typename RowCfg<M>::Rad, L, ColCfg<L>::Rad::get(ColCfg<L>::Rad::count - 1)>),
                     dim3((unsigned)nblocks), dim3(XPass<T, L, M>::THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace

XGeom xc2r_geom(int dtype, int n1, int M) {
#define GRF_X(L_, M_)                                                                        \
  if (n1 == L_ && M == M_)                                                                   \
    return dtype == 0 ? XGeom{XPass<float, L_, M_>::THREADS, XPass<float, L_, M_>::RB}      \
                      : XGeom{XPass<double, L_, M_>::THREADS, XPass<double, L_, M_>::RB};
  GRF_XC2R_PAIRS(GRF_X)
#undef GRF_X
  return XGeom{0, 0};
}

hipError_t launch_xc2r(int dtype, int n1, int M, const Args& a, long long nblocks, hipStream_t s) {
#define GRF_X(L_, M_) \
  if (n1 == L_ && M == M_) return dtype == 0 ? xlaunch<float, L_, M_>(a, nblocks, s) : xlaunch<double, L_, M_>(a, nblocks, s);
  GRF_XC2R_PAIRS(GRF_X)
#undef GRF_X
  return hipErrorInvalidValue;
}

}  // namespace grf
