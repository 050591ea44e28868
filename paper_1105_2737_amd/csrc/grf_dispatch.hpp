// Per-length launch configurations and the dispatch interface between the
// host library and the kernel translation units.
//
// Column passes: Rad = radix order (first radix R_0 sets NT = L / R_0 threads
// per column), CP = column pairs per workgroup (float32 / float64), PAD = LDS
// row padding in column pairs.  Row passes: RB rows per workgroup.
#pragma once
#include <hip/hip_runtime.h>

#include "grf.h"
#include "grf_common.hpp"

namespace grf {

struct Args;

// Supported transform lengths (2^a 3^b 5^c):
//   column (leading-axis) lengths: GRF_COL_LENGTHS
//   row half-lengths M = N_d / 2:  GRF_ROW_LENGTHS
#define GRF_COL_LENGTHS(X) X(4) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(180) X(256) X(360) X(384) X(500) X(512) X(768) X(1000) X(1024)
#define GRF_ROW_LENGTHS(X) X(2) X(4) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(180) X(192) X(256) X(360) X(384) X(500) X(512) X(1024) X(2048)

// The passes (values as the GRF_PASS_* constants of the C interface).
enum PassKind {
  PASS_COL_GEN_INV = GRF_PASS_COL_GEN_INV,     // noise generation + inverse transform (one-FFT algorithm, axis 1)
  PASS_COL_LOAD_INV = GRF_PASS_COL_LOAD_INV,   // inverse transform of a stored spectrum (middle axis)
  PASS_COL_LOAD_FWD = GRF_PASS_COL_LOAD_FWD,   // forward transform (adjoint, middle axis)
  PASS_COL_FILTER = GRF_PASS_COL_FILTER,       // forward, filter, inverse (two-FFT algorithm, axis 1)
  PASS_COL_GRAD = GRF_PASS_COL_GRAD,           // forward transform + adjoint reduction (axis 1)
  PASS_ROW_C2R = GRF_PASS_ROW_C2R,             // last axis, complex-to-real inverse
  PASS_ROW_R2C_GEN = GRF_PASS_ROW_R2C_GEN,     // last axis, white noise + real-to-complex forward
  PASS_ROW_R2C_LOAD = GRF_PASS_ROW_R2C_LOAD,   // last axis, stored real rows + real-to-complex forward
  PASS_ROW_GEN_C2R = GRF_PASS_ROW_GEN_C2R,     // d = 1: whole fields, noise + filter + complex-to-real
  PASS_R2R_COL_GEN = GRF_PASS_R2R_COL_GEN,     // reflecting: coefficients + cosine transform, axis 1
  PASS_R2R_COL_LOAD = GRF_PASS_R2R_COL_LOAD,   // reflecting: cosine transform, middle axis
  PASS_R2R_ROW_LOAD = GRF_PASS_R2R_ROW_LOAD,   // reflecting: cosine transform, last axis
  PASS_R2R_ROW_GEN = GRF_PASS_R2R_ROW_GEN,     // reflecting, d = 1: coefficients + cosine transform
  PASS_COL_SEQ_INV = GRF_PASS_COL_SEQ_INV,     // as PASS_COL_GEN_INV, normals in the recursive draw order
  PASS_SPEC_FILTER = GRF_PASS_SPEC_FILTER,     // two-FFT, d = 1 and 3: filter on the transformed packed spectrum
  PASS_COL_GRAD3 = 100,                        // PASS_COL_GRAD for d = 3 (internal: adjoint only)
  PASS_COL_GRAD1 = 101,                        // PASS_COL_GRAD for the two-FFT algorithm (internal)
  // adjoint of the reflecting-boundary sampler (internal): cosine transforms
  // transposed (DCT-II), last axis and leading axes, the latter optionally
  // with the reduction (RED)
  PASS_R2R_ROW_FWD = 102,
  PASS_R2R_ROW_FWD_RED = 103,
  PASS_R2R_COL_FWD = 104,
  PASS_R2R_COL_FWD_RED = 105,
  PASS_COL_GRAD_SEQ = 106,                     // PASS_COL_GRAD / _GRAD3 in the recursive draw order
  PASS_COL_GRAD3_SEQ = 107,
  PASS_COL_FILTER3 = 109,                      // two-FFT, d = 3: PASS_COL_FILTER without the packed plane slot
  PASS_SPEC_FILTER0 = 110,                     // two-FFT, d = 3: the filter on the packed plane slots only
  PASS_COL_GEN_PART = 111,                     // PASS_COL_GEN_INV stopped before the transform's last stage
  PASS_ROW_XC2R = 112,                         // that last stage + PASS_ROW_C2R (after PASS_COL_GEN_PART or _SEQ_PART)
  PASS_COL_SEQ_PART = 113,                     // PASS_COL_SEQ_INV stopped before the transform's last stage
};

inline bool is_r2r_pass(int p) {
  return (p >= PASS_R2R_COL_GEN && p <= PASS_R2R_ROW_GEN) || (p >= PASS_R2R_ROW_FWD && p <= PASS_R2R_COL_FWD_RED);
}
// passes that take rows (last axis) rather than column tiles
inline bool is_row_pass(int p) {
  return p == PASS_ROW_C2R || p == PASS_ROW_R2C_GEN || p == PASS_ROW_R2C_LOAD || p == PASS_ROW_GEN_C2R ||
         p == PASS_R2R_ROW_LOAD || p == PASS_R2R_ROW_GEN || p == PASS_R2R_ROW_FWD || p == PASS_R2R_ROW_FWD_RED;
}

// Workgroup geometry of a pass at a given length (for grid sizing).
struct Geom {
  int threads;   // threads per workgroup
  int per_wg;    // column pairs (column passes) or rows (row passes) per workgroup
};

bool col_length_supported(int L);
bool row_length_supported(int M);
Geom pass_geom(int pass, int dtype, int L);

// Runtime-radix passes (grf_generic.hpp) for lengths that have no
// compile-time kernel: column passes (PASS_COL_GEN_INV, PASS_COL_LOAD_INV,
// PASS_COL_LOAD_FWD) of length L <= GRF_GENERIC_MAX_COL, row passes
// (PASS_ROW_C2R, PASS_ROW_R2C_GEN, PASS_ROW_R2C_LOAD and, for d = 1 with the
// one-FFT algorithm, PASS_ROW_GEN_C2R) of half-length M <= GRF_GENERIC_MAX_ROW.
#define GRF_GENERIC_MAX_COL 4096
#define GRF_GENERIC_MAX_ROW 8192
struct GGeom {
  int threads;    // threads per workgroup (0: unsupported)
  int per_wg;     // column pairs (column passes) or rows (row passes) per workgroup
  int nt;         // threads per transform
  int rs;         // LDS stride (column passes: pairs per row; row passes: elements per row)
  size_t lds;     // dynamic LDS bytes
};
// vpt: values per thread of a transform (4 or 8; NT = ceil(L / vpt)).
GGeom generic_geom(int pass, int dtype, int L, int vpt);
// Radix list of L (8s first, then 4 or 2, then 5s and 3s) into rad; returns
// the number of stages, -1 if L is not 2/3/5-smooth.
int radix_plan(int L, int* rad);
// a.gl .. a.grad must be set (transform length, geometry, values per thread,
// radix list).
hipError_t launch_generic(int pass, int dtype, const Args& a, long long nblocks, hipStream_t s);

// The d = 2 one-FFT sampler with the column transform's last stage moved into
// the last-axis pass (PASS_COL_GEN_PART or PASS_COL_SEQ_PART, then
// PASS_ROW_XC2R), for the (N_1, M) pairs listed; the two passes give the bits
// of PASS_COL_GEN_INV (PASS_COL_SEQ_INV) + PASS_ROW_C2R.
// (1024, 512) measured slower: 0.689 -> 0.702 ms per 1024^2 x 256 step, the
// last-axis pass gaining more than the column pass (last radix 4) loses.
#define GRF_XC2R_PAIRS(X) X(512, 256)
constexpr bool xc2r_col_length(int L) {
#define GRF_X(L_, M_) L == L_ ||
  return GRF_XC2R_PAIRS(GRF_X) false;
#undef GRF_X
}
struct XGeom {
  int threads;   // threads per workgroup (0: no kernel for the pair)
  int rows;      // rows per workgroup (the column transform's last radix)
};
XGeom xc2r_geom(int dtype, int n1, int M);
// a.rows = fields * N_1, a.tw = W_{N_1}, a.tw2 = W_{N_d}; nblocks = a.rows / rows.
hipError_t launch_xc2r(int dtype, int n1, int M, const Args& a, long long nblocks, hipStream_t s);

// Launch one pass over `nblocks` workgroups.  dtype: 0 = float32, 1 = float64.
hipError_t launch_pass(int pass, int dtype, int L, const Args& a, long long nblocks, hipStream_t s);

// Per-dtype implementations (defined in the kernel translation units).
hipError_t launch_col_f32(int pass, int L, const Args& a, long long nblocks, hipStream_t s);
hipError_t launch_col_f64(int pass, int L, const Args& a, long long nblocks, hipStream_t s);
hipError_t launch_row_f32(int pass, int M, const Args& a, long long nblocks, hipStream_t s);
hipError_t launch_row_f64(int pass, int M, const Args& a, long long nblocks, hipStream_t s);
Geom geom_col_f32(int pass, int L);
Geom geom_col_f64(int pass, int L);
Geom geom_row_f32(int pass, int M);
Geom geom_row_f64(int pass, int M);

// One-dimensional sampler (fields of N = 2M points, RB per workgroup): with
// partial == nullptr, workgroup w writes fields w*RB ..; otherwise the
// covariance epilogue, nblocks workgroups each writing 2M float64 partial sums.
hipError_t launch_gen1d(int dtype, int M, const Args& a, long long nblocks, double* partial, hipStream_t s);
hipError_t launch_gen1d_f32(int M, const Args& a, long long nblocks, double* partial, hipStream_t s);
hipError_t launch_gen1d_f64(int M, const Args& a, long long nblocks, double* partial, hipStream_t s);
Geom geom_gen1d(int dtype, int M);
Geom geom_gen1d_f32(int M);
Geom geom_gen1d_f64(int M);

// Reflecting boundaries (cosine / sine transforms): launch and geometry of the
// PASS_R2R_* passes (L: column length, or half-length M = N_d / 2 of a row
// pass), and the table a_n / z_n over the slot grid for a.recs[0] (out holds
// n1 * no * nd values of the working precision).
hipError_t launch_r2r(int pass, int dtype, int L, const Args& a, long long nblocks, hipStream_t s);
Geom geom_r2r(int pass, int dtype, int L);
hipError_t launch_r2r_table(int dtype, const Args& a, void* out, hipStream_t s);
hipError_t launch_r2r_f32(int pass, int L, const Args& a, long long nblocks, hipStream_t s);
hipError_t launch_r2r_f64(int pass, int L, const Args& a, long long nblocks, hipStream_t s);
Geom geom_r2r_f32(int pass, int L);
Geom geom_r2r_f64(int pass, int L);
hipError_t launch_r2r_table_f32(const Args& a, void* out, hipStream_t s);
hipError_t launch_r2r_table_f64(const Args& a, void* out, hipStream_t s);

// helper kernels (grf_util.hip)
// out[x] = scale * sum_{w < nw} partial[w * n + x], the sum taken in order of w.
hipError_t launch_cov_reduce(const double* partial, int nw, long long n, double scale, double* out, hipStream_t s);
// acc[x] += sum_{b < nb} f[b][0] * f[b][x] (fields of P values of the working
// precision, in float64, in order of b).
hipError_t launch_cov_accum(int dtype, const void* fields, int nb, long long P, double* acc, hipStream_t s);
// Device table of h for the record a.recs[0] over the plan's (row, m) grid,
// row stride M + 2, allocated into *out (synchronous).
grf_status build_filter_table(int dtype, Args a, double scale, void** out);
hipError_t launch_prep_recs(const double* theta, int batch, int kind, int d, double vol, FieldRec* out, int* err,
                            hipStream_t s);
hipError_t launch_reduce_partials(const double* partial, int batch, int nper, double* grad, hipStream_t s);
// Adjoint helpers: d = 1 reduction over the last-axis spectrum (nblocks =
// a.batch * a.ntile workgroups of 256 threads, one Philox block per thread),
// and the d = 3 noise gradient of the planes k_d = 0, N_d/2 from a.plane.
hipError_t launch_grad1d(int dtype, const Args& a, long long nblocks, hipStream_t s);
hipError_t launch_grad_plane(int dtype, const Args& a, hipStream_t s);
// Two-FFT algorithm, d = 1 and 3: the filter on the packed spectrum (one
// thread per slot, a.rows = rows of the chunk) and the adjoint's reduction
// over the packed spectra of g and z (a.ntile workgroups per field).
hipError_t launch_spec_filter(int dtype, const Args& a, long long nblocks, bool slot0, hipStream_t s);
hipError_t launch_grad_spec(int dtype, const Args& a, long long nblocks, hipStream_t s);
// One-FFT adjoint (d = 2, 3) on a spectrum transformed along every axis (grid
// lengths without a compile-time adjoint column kernel): a.ntile workgroups of
// 256 threads per field, one slot pair of a row per thread.
hipError_t launch_grad_gen(int dtype, const Args& a, long long nblocks, hipStream_t s);
// The one-FFT sampler's half-spectrum A = h xi before the inverse transforms
// (a.ntile workgroups per field).
hipError_t launch_debug_spectrum(int dtype, const Args& a, long long nblocks, hipStream_t s);
hipError_t launch_philox_raw(unsigned long long seed, const uint32_t* ctr, long long n, uint32_t* out, hipStream_t s);
hipError_t launch_noise(int dtype, unsigned long long seed, int tag, int rows, int nd, int batch, void* out,
                        hipStream_t s);

}  // namespace grf
