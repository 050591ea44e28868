// Compile-time schedule per transform length.  The radix order, threads per
// transform and tile shapes here are the defaults the plan uses.
#pragma once
#include "grf_fft.hpp"

namespace grf {

// Column (leading-axis) transforms.  Radices stay <= 10 here: a thread holds
// a column pair, and a radix-16 butterfly on pairs keeps 32 complex values
// live, which costs occupancy.  The first radix sets the threads per column
// (L / R_0): 360, 384 and 768 start with 4 (twice the waves per CU of a
// first 8 in the same LDS; measured 1.19-1.40x faster generating passes).  The
// lengths the uneven batch also runs (64 ... 1024 in its lists) need orders
// whose thread counts fit its persistent kernel's tiles, since its plan-order
// bodies reproduce these bits (its 360 tiles were narrowed for 4-10-9).
template <int L> struct ColCfg;
#define GRF_COLCFG(L_, CP32_, CP64_, PAD_, ...)            \
  template <> struct ColCfg<L_> {                          \
    using Rad = Radices<__VA_ARGS__>;                      \
    static constexpr int CP32 = CP32_, CP64 = CP64_, PAD = PAD_; \
  };
GRF_COLCFG(4, 16, 16, 1, 4)
GRF_COLCFG(8, 16, 16, 1, 8)
GRF_COLCFG(12, 16, 16, 1, 3, 4)
GRF_COLCFG(16, 16, 16, 1, 4, 4)
GRF_COLCFG(24, 16, 16, 1, 4, 6)
GRF_COLCFG(32, 16, 16, 1, 8, 4)
GRF_COLCFG(48, 16, 8, 1, 6, 8)
GRF_COLCFG(64, 16, 8, 1, 8, 8)
GRF_COLCFG(96, 16, 8, 1, 8, 4, 3)
GRF_COLCFG(128, 16, 8, 1, 8, 4, 4)
GRF_COLCFG(180, 8, 4, 1, 5, 6, 6)
GRF_COLCFG(256, 8, 4, 1, 8, 8, 4)
GRF_COLCFG(360, 8, 4, 1, 4, 10, 9)
GRF_COLCFG(384, 8, 4, 1, 4, 8, 4, 3)
GRF_COLCFG(500, 4, 2, 1, 10, 10, 5)
GRF_COLCFG(512, 4, 2, 0, 8, 8, 8)
GRF_COLCFG(768, 4, 2, 1, 4, 8, 8, 3)
GRF_COLCFG(1000, 4, 2, 0, 10, 10, 10)
GRF_COLCFG(1024, 4, 2, 0, 8, 8, 4, 4)
#undef GRF_COLCFG

// Column passes that load a stored spectrum and transform it forward (the
// two-FFT filter pass and the adjoint): same radices, their own tile shapes.
template <int L> struct ColCfgF : ColCfg<L> {};
template <> struct ColCfgF<512> : ColCfg<512> {
  static constexpr int CP32 = 8, CP64 = 4, PAD = 1;
};

// Row (last-axis) transforms of half-length M.
template <int M> struct RowCfg;
#define GRF_ROWCFG(M_, RB32_, RB64_, ...)                  \
  template <> struct RowCfg<M_> {                          \
    using Rad = Radices<__VA_ARGS__>;                      \
    static constexpr int RB32 = RB32_, RB64 = RB64_, PADR = 0; \
  };
GRF_ROWCFG(2, 64, 64, 2)
GRF_ROWCFG(4, 64, 64, 4)
GRF_ROWCFG(8, 64, 64, 8)
GRF_ROWCFG(12, 32, 32, 3, 4)
GRF_ROWCFG(16, 32, 32, 4, 4)
GRF_ROWCFG(24, 32, 32, 4, 6)
GRF_ROWCFG(32, 32, 32, 8, 4)
GRF_ROWCFG(48, 16, 16, 6, 8)
GRF_ROWCFG(64, 16, 16, 8, 8)
GRF_ROWCFG(96, 16, 8, 8, 12)
GRF_ROWCFG(128, 16, 8, 16, 8)
GRF_ROWCFG(180, 4, 4, 5, 6, 6)
GRF_ROWCFG(192, 8, 4, 8, 8, 3)
GRF_ROWCFG(256, 8, 8, 8, 8, 4)
GRF_ROWCFG(360, 4, 4, 8, 5, 9)
GRF_ROWCFG(384, 4, 4, 8, 8, 6)
GRF_ROWCFG(500, 4, 2, 10, 10, 5)
GRF_ROWCFG(512, 4, 4, 8, 8, 8)
GRF_ROWCFG(1024, 4, 2, 16, 8, 8)
GRF_ROWCFG(2048, 2, 1, 16, 16, 8)
#undef GRF_ROWCFG

// Last-axis real-to-complex passes (white noise generation, upstream
// gradient): their own radix order and tile shape where measured faster.
template <int M> struct RowCfgG : RowCfg<M> {};
template <> struct RowCfgG<256> {
  using Rad = Radices<16, 16>;
  static constexpr int RB32 = 16, RB64 = 8, PADR = 0;
};

}  // namespace grf
