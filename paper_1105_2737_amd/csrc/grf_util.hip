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

// grad[b][c] = sum_k partial[b][k][c]: one wave per field, lane l summing
// k = l, l + 64, ... in increasing order, then a fixed butterfly over the
// lanes, so the result depends on nper only (not on chunking or timing).
__global__ void __launch_bounds__(256) k_reduce_partials(const double* partial, int batch, int nper, double* grad) {
  const int lane = threadIdx.x & 63;
  const long long b = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= batch) return;   // whole waves leave together
  double s0 = 0, s1 = 0, s2 = 0;
  const double* p = partial + b * nper * 3;
  for (int k = lane; k < nper; k += 64) {
    s0 += p[3 * k];
    s1 += p[3 * k + 1];
    s2 += p[3 * k + 2];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
  }
  if (lane == 0) {
    grad[3 * b] = s0;
    grad[3 * b + 1] = s1;
    grad[3 * b + 2] = s2;
  }
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
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_partials, dim3((batch + 3) / 4), dim3(256), 0, s, partial, batch, nper, grad);
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
  if ((total + 255) / 256 > 0x7fffffffLL) return hipErrorInvalidValue;
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

// Adjoint for d = 1: the last-axis real-to-complex pass has left G = F[g] of
// each field at a.data (packed: slot 0 = (G_0, G_{N/2})).  Thread q of tile
// `tile` of field b takes the entries 2q and 2q+1, i.e. the Philox block q
// that generated them (block 0 also holds A_0 and A_{N/2}); the workgroup's
// sums go to a.partial[(b * ntile + tile) * 3 ..].  dL/dz to a.aux if asked.
template <typename T>
__global__ void __launch_bounds__(256) k_grad1d(Args a) {
  using V = C<T>;
  const int tile = blockIdx.x % a.ntile;
  const int b = blockIdx.x / a.ntile;
  const int q = tile * 256 + threadIdx.x;
  // counter order: block q holds the entries 2q, 2q + 1 (an odd N/2 leaves the
  // last block with one entry, its draws 2 and 3 unused)
  const int NQ = a.seq ? a.M / 2 : (a.M + 1) / 2;
  double acc0 = 0, acc1 = 0, acc2 = 0;
  if (q < NQ) {
    const FieldRec& rec = a.recs[b * a.rec_stride];
    const Filt<T> f = load_filt<T>(rec, 1.0);
    AdjAcc<T> ad(rec);
    T z[4];
    if (a.src == nullptr) {
      const unsigned long long key = a.seed + (unsigned long long)b;
      normals4<T, true>((uint32_t)q, 0u, (uint32_t)a.tag, (uint32_t)key, (uint32_t)(key >> 32), z);
    } else {
      const T* p = (const T*)a.src + (long long)b * a.nd + 4 * q;
      for (int e = 0; e < 4; ++e) z[e] = 4 * q + e < a.nd ? p[e] : (T)0;
    }
    const double il2 = a.il2[2];
    const T* ht = (const T*)a.htab;
    auto hk = [&](int k) -> T { return ht ? ht[k] : filt_h(f, (T)((double)k * k * il2)); };
    const V* G = (const V*)a.data + (long long)b * a.M;
    T* gz = a.aux ? (T*)a.aux + (long long)b * a.nd + 4 * q : nullptr;
    const T s = (T)0.70710678118654752440, s2 = (T)1.4142135623730950488;
    if (a.seq) {
      // draws 4q .. 4q+3: entries 2q+1 and 2q+2, or for the last block the
      // real entries 0 and N/2
      const int ka = 2 * q + 1, kb = 2 * q + 2;
      const T ha = hk(ka);
      const V Ga = G[ka];
      ad.add(2.0, (double)ha, (double)ka * ka * il2, mk<T>(s * z[0], s * z[1]), Ga);
      if (gz) {
        gz[0] = s2 * ha * Ga.x;
        gz[1] = s2 * ha * Ga.y;
      }
      if (kb < a.M) {
        const T hb = hk(kb);
        const V Gb = G[kb];
        ad.add(2.0, (double)hb, (double)kb * kb * il2, mk<T>(s * z[2], s * z[3]), Gb);
        if (gz) {
          gz[2] = s2 * hb * Gb.x;
          gz[3] = s2 * hb * Gb.y;
        }
      } else {
        const V G0 = G[0];
        const T h0 = hk(0), hm = hk(a.M);
        ad.add(1.0, (double)h0, 0.0, mk<T>(z[2], (T)0), mk<T>(G0.x, (T)0));
        ad.add(1.0, (double)hm, (double)a.M * a.M * il2, mk<T>(z[3], (T)0), mk<T>(G0.y, (T)0));
        if (gz) {
          gz[2] = h0 * G0.x;
          gz[3] = hm * G0.y;
        }
      }
      acc0 = ad.acc0 * rec.gs;
      acc1 = ad.acc1;
      acc2 = ad.acc2;
    } else {
    const int ka = 2 * q + 1, kb = 2 * q;
    if (ka < a.M) {
      const T ha = hk(ka);
      const V Ga = G[ka];
      ad.add(2.0, (double)ha, (double)ka * ka * il2, mk<T>(s * z[2], s * z[3]), Ga);
      if (gz) {
        gz[2] = s2 * ha * Ga.x;
        gz[3] = s2 * ha * Ga.y;
      }
    }
    const V Gb = G[kb];
    if (q > 0) {
      const T hb = hk(kb);
      ad.add(2.0, (double)hb, (double)kb * kb * il2, mk<T>(s * z[0], s * z[1]), Gb);
      if (gz) {
        gz[0] = s2 * hb * Gb.x;
        gz[1] = s2 * hb * Gb.y;
      }
    } else {   // the real entries A_0 = h_0 z_0 and A_{N/2} = h_{N/2} z_1
      const T h0 = hk(0), hm = hk(a.M);
      ad.add(1.0, (double)h0, 0.0, mk<T>(z[0], (T)0), mk<T>(Gb.x, (T)0));
      ad.add(1.0, (double)hm, (double)a.M * a.M * il2, mk<T>(z[1], (T)0), mk<T>(Gb.y, (T)0));
      if (gz) {
        gz[0] = h0 * Gb.x;
        gz[1] = hm * Gb.y;
      }
    }
    acc0 = ad.acc0 * rec.gs;
    acc1 = ad.acc1;
    acc2 = ad.acc2;
    }
  }
  __shared__ double red[3][4];
  for (int off = 32; off > 0; off >>= 1) {
    acc0 += __shfl_xor(acc0, off);
    acc1 += __shfl_xor(acc1, off);
    acc2 += __shfl_xor(acc2, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = acc0;
    red[1][wv] = acc1;
    red[2][wv] = acc2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double sacc = 0;
    for (int w = 0; w < 4; ++w) sacc += red[threadIdx.x][w];
    a.partial[((long long)b * a.ntile + tile) * 3 + threadIdx.x] = sacc;
  }
}

// Adjoint for d = 3, dL/dz of the two planes k_d = 0, N_d/2: from Z(k) and
// Z(-k) (stored by k_colg<..., D3>) G0 = (Z(k) + conj Z(-k)) / 2 and
// GM = (Z(k) - conj Z(-k)) / (2i); then the Hermitian arrangement backwards,
// as the d = 2 column kernel does for its plane slots.  One thread per
// (field, row) of a.batch fields.
template <typename T>
__global__ void k_grad_plane(Args a) {
  using V = C<T>;
  const long long R = (long long)a.n1 * a.no;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)a.batch * R) return;
  const int b = (int)(i / R), row = (int)(i % R);
  const int k1 = row / a.no, o = row % a.no;
  const int nrow = ((a.n1 - k1) % a.n1) * a.no + (a.no - o) % a.no;
  const V* Zp = (const V*)a.plane + (long long)b * R;
  const V Z = Zp[row], Zm = Zp[nrow];
  const V g0 = mk<T>((T)0.5 * (Z.x + Zm.x), (T)0.5 * (Z.y - Zm.y));
  const V gn = mk<T>((T)0.5 * (Z.y + Zm.y), (T)-0.5 * (Z.x - Zm.x));
  const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], 1.0);
  const int q1 = wrapk(k1, a.n1), qo = wrapk(o, a.no);
  const double p2b = (double)(q1 * q1) * a.il2[0] + (double)(qo * qo) * a.il2[1];
  const double p2n = p2b + (double)a.M * (double)a.M * a.il2[2];
  const T* hrow = a.htab ? (const T*)a.htab + (long long)row * (a.M + 2) : nullptr;
  const T hz = hrow ? hrow[0] : filt_h(f, (T)p2b);
  const T hn = hrow ? hrow[a.M] : filt_h(f, (T)p2n);
  const T s2 = (T)1.4142135623730950488;
  if (a.seq) {   // the draws of the plane entries (k, 0) and (k, N_d/2) of this row
    T* gzf = (T*)a.aux + (long long)b * a.field_stride * 2;
    const SeqDraw d0 = seq_draw(a, k1, o, 0), dn = seq_draw(a, k1, o, a.M);
    if (d0.kind == 0) {
      gzf[d0.j] = s2 * hz * g0.x;
      gzf[d0.j + 1] = s2 * hz * g0.y;
    } else if (d0.kind == 2) {
      gzf[d0.j] = hz * g0.x;
    }
    if (dn.kind == 0) {
      gzf[dn.j] = s2 * hn * gn.x;
      gzf[dn.j + 1] = s2 * hn * gn.y;
    } else if (dn.kind == 2) {
      gzf[dn.j] = hn * gn.x;
    }
    return;
  }
  T* gzr = (T*)a.aux + (long long)b * a.field_stride * 2 + (long long)row * a.nd;
  if (nrow == row) {
    gzr[0] = hz * g0.x;
    gzr[1] = hn * gn.x;
  } else if (row < nrow) {
    gzr[0] = s2 * hz * g0.x;
    gzr[1] = s2 * hz * g0.y;
  } else {   // slots of a mirrored row carry the Nyquist plane of its partner
    gzr[0] = s2 * hn * gn.x;
    gzr[1] = -s2 * hn * gn.y;
  }
}

// Two-FFT algorithm for d = 1 and 3 (Section 3, the first algorithm): the
// filter on the packed spectrum once every axis is forward transformed,
// A_k = h_k F[z]_k / sqrt(P) (the 1/sqrt(P) is in the filter's scale, or in
// the table).  One thread per slot (row, m) of a field, rows = the N_1 ... N_{d-1}
// leading indices.  Interior slots 0 < m < N_d/2 are scaled by h.  Slot 0 of
// row k holds Z = X(k, 0) + i X(k, N_d/2); both planes are Hermitian in k, so
// with W = Z(-k): X(k, 0) = (Z + conj W)/2 and X(k, N_d/2) = (Z - conj W)/(2i).
// The thread of the smaller of the rows k, -k filters both planes and writes
// both slots (A(-k) = conj A(k), since h is even).
// SLOT0: only the packed plane slots (one thread per row), the other slots
// having been filtered by the column pass.
template <typename T, bool SLOT0 = false>
__global__ void __launch_bounds__(256) k_spec_filter(Args a) {
  using V = C<T>;
  const long long R = (long long)a.n1 * a.no;
  const int M = a.M;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.rows * (SLOT0 ? 1 : M)) return;
  const int m = SLOT0 ? 0 : (int)(i % M);
  const long long grow = SLOT0 ? i : i / M;
  const long long b = grow / R;
  const int row = (int)(grow - b * R);
  const int k1 = row / a.no, o = row - (row / a.no) * a.no;
  const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], a.scale);
  const int q1 = wrapk(k1, a.n1), qo = wrapk(o, a.no);
  const T p2b = (T)(q1 * q1) * (T)a.il2[0] + (T)(qo * qo) * (T)a.il2[1];
  const T il2d = (T)a.il2[2];
  const T* hr = a.htab ? (const T*)a.htab + (long long)row * (M + 2) : nullptr;
  auto hv = [&](int mm) -> T { return hr ? hr[mm] : filt_h(f, p2b + (T)(mm * mm) * il2d); };
  V* base = (V*)a.data + b * R * M;
  if (m > 0) {
    V& x = base[(long long)row * M + m];
    const T h = hv(m);
    x = mk<T>(h * x.x, h * x.y);
    return;
  }
  const int pr = ((a.n1 - k1) % a.n1) * a.no + (a.no - o) % a.no;
  if (pr < row) return;
  const V z = base[(long long)row * M], w = base[(long long)pr * M];
  const V x0 = mk<T>((T)0.5 * (z.x + w.x), (T)0.5 * (z.y - w.y));
  const V xm = mk<T>((T)0.5 * (z.y + w.y), (T)-0.5 * (z.x - w.x));
  const T h0 = hv(0), hm = hv(M);
  const V a0 = mk<T>(h0 * x0.x, h0 * x0.y), am = mk<T>(hm * xm.x, hm * xm.y);
  base[(long long)row * M] = mk<T>(a0.x - am.y, a0.y + am.x);                      // A0 + i AM
  if (pr != row) base[(long long)pr * M] = mk<T>(a0.x + am.y, am.x - a0.y);      // conj A0 + i conj AM
}

// Adjoint of the two-FFT algorithm for d = 1 and 3: with G = F[g] (data) and
// xi = scale F[z] (src2), both packed and transformed along every axis, each
// half-spectrum entry adds w (h/2) dlogS/dtheta Re(xi conj G) (w = 2 for
// 0 < m < N_d/2, which stands for k and -k; in the planes m = 0, N_d/2 each
// k once).  Slot 0 is unpacked as in k_spec_filter; the thread of the pair
// (k, -k) counts both (w = 2), a self-mirrored row once.  Workgroup `tile`
// of field b takes slots tile * 256 ... of that field.
template <typename T>
__global__ void __launch_bounds__(256) k_grad_spec(Args a) {
  using V = C<T>;
  const int tile = blockIdx.x % a.ntile;
  const long long b = blockIdx.x / a.ntile;
  const long long R = (long long)a.n1 * a.no;
  const int M = a.M;
  const long long e = (long long)tile * 256 + threadIdx.x;
  double acc0 = 0, acc1 = 0, acc2 = 0;
  if (e < R * M) {
    const int m = (int)(e % M);
    const int row = (int)(e / M);
    const int k1 = row / a.no, o = row - (row / a.no) * a.no;
    const FieldRec& rec = a.recs[b * a.rec_stride];
    const Filt<T> f = load_filt<T>(rec, 1.0);
    AdjAcc<T> ad(rec);
    const int q1 = wrapk(k1, a.n1), qo = wrapk(o, a.no);
    const double p2b = (double)(q1 * q1) * a.il2[0] + (double)(qo * qo) * a.il2[1];
    const double il2d = a.il2[2];
    const T* hr = a.htab ? (const T*)a.htab + (long long)row * (M + 2) : nullptr;
    auto hv = [&](int mm) -> T { return hr ? hr[mm] : filt_h(f, (T)(p2b + (double)mm * mm * il2d)); };
    const V* G = (const V*)a.data + b * R * M;
    const V* X = (const V*)a.src2 + b * R * M;
    const T sc = (T)a.scale;
    if (m > 0) {
      const V x = X[(long long)row * M + m];
      ad.add(2.0, (double)hv(m), p2b + (double)m * m * il2d, mk<T>(sc * x.x, sc * x.y), G[(long long)row * M + m]);
    } else {
      const int pr = ((a.n1 - k1) % a.n1) * a.no + (a.no - o) % a.no;
      if (pr >= row) {
        const double w = pr == row ? 1.0 : 2.0;
        const V zx = X[(long long)row * M], wx = X[(long long)pr * M];
        const V zg = G[(long long)row * M], wg = G[(long long)pr * M];
        const V x0 = mk<T>((T)0.5 * sc * (zx.x + wx.x), (T)0.5 * sc * (zx.y - wx.y));
        const V xm = mk<T>((T)0.5 * sc * (zx.y + wx.y), (T)-0.5 * sc * (zx.x - wx.x));
        const V g0 = mk<T>((T)0.5 * (zg.x + wg.x), (T)0.5 * (zg.y - wg.y));
        const V gm = mk<T>((T)0.5 * (zg.y + wg.y), (T)-0.5 * (zg.x - wg.x));
        ad.add(w, (double)hv(0), p2b, x0, g0);
        ad.add(w, (double)hv(M), p2b + (double)M * M * il2d, xm, gm);
      }
    }
    acc0 = ad.acc0 * rec.gs;
    acc1 = ad.acc1;
    acc2 = ad.acc2;
  }
  __shared__ double red[3][4];
  for (int off = 32; off > 0; off >>= 1) {
    acc0 += __shfl_xor(acc0, off);
    acc1 += __shfl_xor(acc1, off);
    acc2 += __shfl_xor(acc2, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = acc0;
    red[1][wv] = acc1;
    red[2][wv] = acc2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double sacc = 0;
    for (int v = 0; v < 4; ++v) sacc += red[threadIdx.x][v];
    a.partial[(b * a.ntile + tile) * 3 + threadIdx.x] = sacc;
  }
}

// Adjoint of the one-FFT algorithm (d = 2, 3) at grid lengths without a
// compile-time adjoint column kernel: G = F[g] transformed along every axis by
// the runtime-radix passes and read back from memory (packed like the
// sampler's intermediate, slot 0 = Z(k) = G(k, 0) + i G(k, N_d/2)), instead of
// being formed inside the column transform.  Each thread takes the entries
// 2q, 2q + 1 of one row (one Philox block), regenerates their noise and h as
// gen_pair does, and adds w (h/2) dlogS/dtheta Re(xi conj G) (w = 2 for
// 0 < m < N_d/2).  Slot 0 is unpacked with the mirrored row:
// G(k, 0) = (Z(k) + conj Z(-k)) / 2, G(k, N_d/2) = (Z(k) - conj Z(-k)) / 2i;
// the lower row of a pair (k, -k) counts both (w = 2) and writes dL/dz of the
// first two normals of both rows, a self-mirrored row counts once.  dL/dz of
// an interior entry A = h s (z + i z') is 2 h s G.
template <typename T>
__global__ void __launch_bounds__(256) k_grad_gen(Args a) {
  using V = C<T>;
  const int tile = blockIdx.x % a.ntile;
  const int b = blockIdx.x / a.ntile;
  const int NQ = (a.M + 1) / 2;
  const long long R = (long long)a.n1 * a.no;
  const long long e = (long long)tile * 256 + threadIdx.x;
  double acc0 = 0, acc1 = 0, acc2 = 0;
  if (e < R * NQ) {
    const int row = (int)(e / NQ), q = (int)(e % NQ), m0 = 2 * q;
    const int k1 = row / a.no, o = row - k1 * a.no;
    const FieldRec& rec = a.recs[b * a.rec_stride];
    const Filt<T> f = load_filt<T>(rec, 1.0);
    AdjAcc<T> ad(rec);
    const unsigned long long key = a.seed + (unsigned long long)b;
    const uint32_t key0 = (uint32_t)key, key1 = (uint32_t)(key >> 32);
    const T* zsrc = (const T*)a.src;
    T z[4];
    load_z4<T>(a, zsrc, b, row, m0, key0, key1, z);
    const int q1 = wrapk(k1, a.n1), qo = wrapk(o, a.no);
    const double p2b = (double)(q1 * q1) * a.il2[0] + (double)(qo * qo) * a.il2[1];
    const double il2d = a.il2[2];
    // h by gen_pair's float expressions (or its table)
    const T* hr = a.htab ? (const T*)a.htab + (long long)row * (a.M + 2) : nullptr;
    const T p2bt = (T)(q1 * q1) * (T)a.il2[0] + (T)(qo * qo) * (T)a.il2[1];
    const T il2t = (T)a.il2[2];
    auto hv = [&](int m) -> T { return hr ? hr[m] : filt_h(f, p2bt + (T)(m * m) * il2t); };
    const V* Gf = (const V*)a.data + (long long)b * R * a.M;
    const V* G = Gf + (long long)row * a.M;
    T* gzf = a.aux ? (T*)a.aux + (long long)b * a.field_stride * 2 : nullptr;
    T* gz = gzf ? gzf + (long long)row * a.nd + 2 * m0 : nullptr;
    const T s = (T)0.70710678118654752440, s2 = (T)1.4142135623730950488;
    if (m0 + 1 < a.M) {
      const int m = m0 + 1;
      const T h1 = hv(m);
      const V G1 = G[m];
      ad.add(2.0, (double)h1, p2b + (double)m * m * il2d, mk<T>(s * z[2], s * z[3]), G1);
      if (gz) {
        gz[2] = s2 * h1 * G1.x;
        gz[3] = s2 * h1 * G1.y;
      }
    }
    if (m0 > 0) {
      const T h0 = hv(m0);
      const V G0 = G[m0];
      ad.add(2.0, (double)h0, p2b + (double)m0 * m0 * il2d, mk<T>(s * z[0], s * z[1]), G0);
      if (gz) {
        gz[0] = s2 * h0 * G0.x;
        gz[1] = s2 * h0 * G0.y;
      }
    } else {
      const int nrow = ((a.n1 - k1) % a.n1) * a.no + (a.no - o) % a.no;
      if (nrow >= row) {
        const T h0 = hv(0), hm = hv(a.M);
        const V zg = G[0], wg = Gf[(long long)nrow * a.M];
        const V g0 = mk<T>((T)0.5 * (zg.x + wg.x), (T)0.5 * (zg.y - wg.y));
        const V gm = mk<T>((T)0.5 * (zg.y + wg.y), (T)-0.5 * (zg.x - wg.x));
        const double pm = p2b + (double)a.M * a.M * il2d;
        if (nrow == row) {   // A(k, 0) = h z_0 and A(k, N_d/2) = h z_1, both real
          ad.add(1.0, (double)h0, p2b, mk<T>(z[0], (T)0), g0);
          ad.add(1.0, (double)hm, pm, mk<T>(z[1], (T)0), gm);
          if (gz) {
            gz[0] = h0 * g0.x;
            gz[1] = hm * gm.x;
          }
        } else {   // xi(k, 0) from this row's block, xi(k, N_d/2) from the mirrored row's
          T zz[4];
          load_z4<T>(a, zsrc, b, nrow, 0, key0, key1, zz);
          ad.add(2.0, (double)h0, p2b, mk<T>(s * z[0], s * z[1]), g0);
          ad.add(2.0, (double)hm, pm, mk<T>(s * zz[0], s * zz[1]), gm);
          if (gz) {
            gz[0] = s2 * h0 * g0.x;
            gz[1] = s2 * h0 * g0.y;
            T* gn = gzf + (long long)nrow * a.nd;
            gn[0] = s2 * hm * gm.x;
            gn[1] = s2 * hm * gm.y;
          }
        }
      }
    }
    acc0 = ad.acc0 * rec.gs;
    acc1 = ad.acc1;
    acc2 = ad.acc2;
  }
  __shared__ double red[3][4];
  for (int off = 32; off > 0; off >>= 1) {
    acc0 += __shfl_xor(acc0, off);
    acc1 += __shfl_xor(acc1, off);
    acc2 += __shfl_xor(acc2, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = acc0;
    red[1][wv] = acc1;
    red[2][wv] = acc2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double sacc = 0;
    for (int v = 0; v < 4; ++v) sacc += red[threadIdx.x][v];
    a.partial[((long long)b * a.ntile + tile) * 3 + threadIdx.x] = sacc;
  }
}

// The half-spectrum A = h xi that the one-FFT sampler transforms (noise,
// Hermitian arrangement and filter of Section 3's second algorithm), by the
// generating pass's own gen_pair, packed like the sampler's intermediate:
// [field][row][N_d/2], slot 0 = A(k, 0) + i A(k, N_d/2).  a.ntile workgroups
// per field, one slot pair (one Philox block) per thread; a workgroup never
// spans two fields, so the key is uniform over it, as gen_pair assumes.
template <typename T>
__global__ void __launch_bounds__(256) k_debug_spectrum(Args a) {
  const int b = blockIdx.x / a.ntile;
  const long long e = (long long)(blockIdx.x % a.ntile) * 256 + threadIdx.x;
  const int NQ = (a.M + 1) / 2;
  const long long R = (long long)a.n1 * a.no;
  if (e >= R * NQ) return;
  const int row = (int)(e / NQ), q = (int)(e % NQ);
  const int kk1 = row / a.no, o = row - kk1 * a.no;
  const Filt<T> f = load_filt<T>(a.recs[0], a.scale);
  const unsigned long long key = a.seed + (unsigned long long)b;
  C<T> A0, A1;
  gen_pair<T>(a, f, nullptr, b, (uint32_t)key, (uint32_t)(key >> 32), kk1, o, 2 * q, A0, A1);
  C<T>* out = (C<T>*)a.data + ((long long)b * R + row) * a.M + 2 * q;
  out[0] = A0;
  if (2 * q + 1 < a.M) out[1] = A1;
}

hipError_t launch_debug_spectrum(int dtype, const Args& a, long long nblocks, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_debug_spectrum<float>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_debug_spectrum<double>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_spec_filter(int dtype, const Args& a, long long nblocks, bool slot0, hipStream_t s) {
  if (dtype == 0 && slot0)
    hipLaunchKernelGGL((k_spec_filter<float, true>), dim3((unsigned)nblocks), dim3(256), 0, s, a);
  else if (dtype == 0)
    hipLaunchKernelGGL((k_spec_filter<float, false>), dim3((unsigned)nblocks), dim3(256), 0, s, a);
  else if (slot0)
    hipLaunchKernelGGL((k_spec_filter<double, true>), dim3((unsigned)nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_spec_filter<double, false>), dim3((unsigned)nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_grad_spec(int dtype, const Args& a, long long nblocks, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_grad_spec<float>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_grad_spec<double>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_grad_gen(int dtype, const Args& a, long long nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_grad_gen<float>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_grad_gen<double>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_grad1d(int dtype, const Args& a, long long nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_grad1d<float>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_grad1d<double>, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_grad_plane(int dtype, const Args& a, hipStream_t s) {
  const long long n = (long long)a.batch * a.n1 * a.no;
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_grad_plane<float>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(k_grad_plane<double>, grid, block, 0, s, a);
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
