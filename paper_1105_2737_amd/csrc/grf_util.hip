// Helper kernels: per-field constants from device-resident parameters, the
// deterministic per-field reduction of adjoint partial sums, raw Philox output,
// the noise array of the contract, and the reductions of the covariance
// estimator.
#include "grf_dispatch.hpp"
#include "grf_host.hpp"
#include "grf_kernels.hpp"

namespace grf {

__global__ void k_prep_recs(const double* theta, int batch, int kind, int d, double vol, FieldRec* out,
                            int* err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  FieldRec r;
  if (make_field_rec(kind, d, vol, theta[3 * b + 0], theta[3 * b + 1], theta[3 * b + 2], &r) != 0) {
    // invalid parameters: the field comes out as NaN rather than silently wrong
    if (err != nullptr) atomicOr(err, 1);
    r = FieldRec{};
    r.kind = kind;
    r.c0 = __builtin_nan("");
    r.a = 1.0;
  }
  out[b] = r;
}

__global__ void k_reduce_partials(const double* partial, int batch, int nper, double* grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch * 3) return;
  const int b = i / 3, c = i % 3;
  double s = 0;
  for (int k = 0; k < nper; ++k) s += partial[((long long)b * nper + k) * 3 + c];
  grad[i] = s;
}

__global__ void k_philox_raw(unsigned long long seed, const uint32_t* ctr, long long n, uint32_t* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
  const uint4 x = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  out[4 * i] = x.x;
  out[4 * i + 1] = x.y;
  out[4 * i + 2] = x.z;
  out[4 * i + 3] = x.w;
}

// z of the contract for `batch` fields: [batch][rows][nd]
template <typename T>
__global__ void k_noise(unsigned long long seed, int tag, int rows, int nd, int batch, T* out) {
  const int nq = (nd + 3) / 4;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)batch * rows * nq;
  if (i >= total) return;
  const int q = (int)(i % nq);
  const long long rb = i / nq;
  const int row = (int)(rb % rows);
  const int b = (int)(rb / rows);
  const unsigned long long key = seed + (unsigned long long)b;
  T z[4];
  normals4<T>((uint32_t)q, (uint32_t)row, (uint32_t)tag, (uint32_t)key, (uint32_t)(key >> 32), z);
  T* p = out + ((long long)b * rows + row) * nd + 4 * q;
  for (int l = 0; l < 4 && 4 * q + l < nd; ++l) p[l] = z[l];
}


grf_status build_filter_table(int dtype, Args a, double scale, void** out) {
  a.scale = scale;
  const long long n = (long long)a.n1 * a.no * (a.M + 2);
  const size_t es = dtype == 0 ? 4 : 8;
  hipError_t e = hipMalloc(out, n * es);
  if (e != hipSuccess) return host::fail(GRF_ENOMEM, "hipMalloc of filter table failed");
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_filter_table<float>, grid, block, 0, 0, a, (float*)*out);
  else
    hipLaunchKernelGGL(k_filter_table<double>, grid, block, 0, 0, a, (double*)*out);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return host::hip_fail(e, "filter table");
  return GRF_OK;
}

hipError_t launch_prep_recs(const double* theta, int batch, int kind, int d, double vol, FieldRec* out, int* err,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_prep_recs, dim3((batch + 63) / 64), dim3(64), 0, s, theta, batch, kind, d, vol, out, err);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, int batch, int nper, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partials, dim3((batch * 3 + 255) / 256), dim3(256), 0, s, partial, batch, nper, grad);
  return hipGetLastError();
}

hipError_t launch_philox_raw(unsigned long long seed, const uint32_t* ctr, long long n, uint32_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_raw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, ctr, n, out);
  return hipGetLastError();
}

hipError_t launch_noise(int dtype, unsigned long long seed, int tag, int rows, int nd, int batch, void* out,
                        hipStream_t s) {
  const long long total = (long long)batch * rows * ((nd + 3) / 4);
  if (total <= 0) return hipSuccess;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_noise<float>, grid, block, 0, s, seed, tag, rows, nd, batch, (float*)out);
  else
    hipLaunchKernelGGL(k_noise<double>, grid, block, 0, s, seed, tag, rows, nd, batch, (double*)out);
  return hipGetLastError();
}

// out[x] = scale * sum_w partial[w * n + x], w in increasing order.
__global__ void k_cov_reduce(const double* partial, int nw, long long n, double scale, double* out) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  double acc = 0.0;
  for (int w = 0; w < nw; ++w) acc += partial[(long long)w * n + x];
  out[x] = acc * scale;
}

// acc[x] += sum_b f[b][0] f[b][x], b in increasing order, in float64.
template <typename T>
__global__ void k_cov_accum(const T* f, int nb, long long P, double* acc) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= P) return;
  double s = acc[x];
  for (int b = 0; b < nb; ++b) s += (double)f[(long long)b * P] * (double)f[(long long)b * P + x];
  acc[x] = s;
}

hipError_t launch_cov_reduce(const double* partial, int nw, long long n, double scale, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cov_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partial, nw, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_cov_accum(int dtype, const void* fields, int nb, long long P, double* acc, hipStream_t s) {
  if (P <= 0 || nb <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P + 255) / 256)), block(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_cov_accum<float>, grid, block, 0, s, (const float*)fields, nb, P, acc);
  else
    hipLaunchKernelGGL(k_cov_accum<double>, grid, block, 0, s, (const double*)fields, nb, P, acc);
  return hipGetLastError();
}

hipError_t launch_gen1d(int dtype, int M, const Args& a, long long nblocks, double* partial, hipStream_t s) {
  return dtype == 0 ? launch_gen1d_f32(M, a, nblocks, partial, s) : launch_gen1d_f64(M, a, nblocks, partial, s);
}

Geom geom_gen1d(int dtype, int M) { return dtype == 0 ? geom_gen1d_f32(M) : geom_gen1d_f64(M); }

hipError_t launch_r2r(int pass, int dtype, int L, const Args& a, long long nblocks, hipStream_t s) {
  return dtype == 0 ? launch_r2r_f32(pass, L, a, nblocks, s) : launch_r2r_f64(pass, L, a, nblocks, s);
}

Geom geom_r2r(int pass, int dtype, int L) { return dtype == 0 ? geom_r2r_f32(pass, L) : geom_r2r_f64(pass, L); }

hipError_t launch_r2r_table(int dtype, const Args& a, void* out, hipStream_t s) {
  return dtype == 0 ? launch_r2r_table_f32(a, out, s) : launch_r2r_table_f64(a, out, s);
}

}  // namespace grf
