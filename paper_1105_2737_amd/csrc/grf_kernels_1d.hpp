// One-dimensional sampling (d = 1) and the statistical covariance estimator.
//
// A 1D field of N = 2M points is a single row whose mirror is itself, so the
// one-FFT algorithm's Hermitian arrangement (Section 3) reduces to: the
// entries k = 0 and k = M are real, A_0 = h_0 z[0] and A_M = h_M z[1]; the
// interior entries are A_k = h_k (z[2k] + i z[2k+1]) / sqrt(2).  Gen1D
// generates these entries for RB fields straight into LDS (packed slot 0 =
// A_0 + i A_M, as in the multi-dimensional layout) and runs the last-axis
// complex-to-real transform on them, so a 1D field costs one write of its
// output.
//
// With COV the fields are not written: every workgroup accumulates
// phi(0) * phi(x) over the fields it generates, in float64, for the
// statistical covariance of Section 4 (the paper's estimator, averaged over
// the samples).  The partial sums of the workgroups are added in a fixed order
// by k_cov_reduce, so the estimate is deterministic.
#pragma once
#include "grf_kernels.hpp"

namespace grf {

template <typename T, int M, class Rad, int RB>
struct Gen1D {
  using V = C<T>;
  using E = Vec<T, 1>;
  using RL = RowLds<M>;
  static constexpr int NT = M / Rad::get(0);
  static constexpr int THREADS = (NT * RB + 63) / 64 * 64;
  static constexpr int R0 = Rad::get(0);
  static constexpr bool WAVE = (64 % NT) == 0;
  static constexpr int ROWS_BYTES = RB * RL::STRIDE * (int)sizeof(E);
  // Long rows read the twiddle table W_N through the caches instead of
  // staging it in LDS: at M = 2048 the 32 KB table halved the workgroups per
  // CU (measured: 4096-point fields 0.797 -> 0.660 ms per 65536, 3% faster at
  // M = 1024, 2% slower at M = 256).
  static constexpr bool TW_GLOBAL = M >= 1024;
  static constexpr int TW_BYTES = TW_GLOBAL ? 0 : 2 * M * (int)sizeof(V);
  static constexpr int LDS_BYTES = ROWS_BYTES + TW_BYTES + RB * (int)sizeof(T);
  using EN = Eng<T, M, Rad, NT, 1, 2, WAVE>;
  static_assert(M % 2 == 0, "a Philox block fills two complex entries");
  // the COV reduction reuses the rows area for M complex float64 values
  static_assert(ROWS_BYTES >= M * 16, "rows area too small for the reduction");

  // Entries of fields f0 .. f0 + nrows - 1 of the call into the LDS rows.
  __device__ __forceinline__ static void generate(const Args& a, long long f0, int nrows, E* sm, int tid) {
    constexpr int NQ = M / 2;   // Philox blocks per field (4 normals each)
    const T s = (T)0.70710678118654752440;
    const T il2 = (T)a.il2[2];
    for (int i = tid; i < nrows * NQ; i += blockDim.x) {
      const int rr = i / NQ, q = i % NQ;
      const long long b = f0 + rr;
      const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], a.scale);
      T z[4];
      if (a.src != nullptr) {
        const T* p = (const T*)a.src + b * (2 * M) + 4 * q;
        z[0] = p[0];
        z[1] = p[1];
        z[2] = p[2];
        z[3] = p[3];
      } else {
        const unsigned long long key = a.seed + (unsigned long long)b;
        normals4<T, false>((uint32_t)q, 0u, (uint32_t)a.tag, (uint32_t)key, (uint32_t)(key >> 32), z);
      }
      // h from the plan's table (families given by their density) or on the fly
      const T* ht = (const T*)a.htab;
      auto hk = [&](int k) -> T { return ht ? ht[k] : filt_h(f, (T)(k * k) * il2); };
      E* row = sm + rr * RL::STRIDE;
      if (a.seq) {
        // draw order of the recursive algorithm: block q holds draws 4q .. 4q+3,
        // i.e. entries 2q+1 and 2q+2 (real and imaginary parts), or for the
        // last block the real entries 0 and M (draws N - 2, N - 1)
        const int ka = 2 * q + 1, kb = 2 * q + 2;
        const T ha = hk(ka);
        row[RL::idx(ka)].v[0] = mk<T>(ha * s * z[0], ha * s * z[1]);
        if (kb < M) {
          const T hb = hk(kb);
          row[RL::idx(kb)].v[0] = mk<T>(hb * s * z[2], hb * s * z[3]);
        } else {
          row[0].v[0] = mk<T>(hk(0) * z[2], hk(M) * z[3]);
        }
        continue;
      }
      const int k1 = 2 * q + 1;
      const T h1 = hk(k1);
      row[RL::idx(k1)].v[0] = mk<T>(h1 * s * z[2], h1 * s * z[3]);
      const int k0 = 2 * q;
      if (k0 > 0) {
        const T h0 = hk(k0);
        row[RL::idx(k0)].v[0] = mk<T>(h0 * s * z[0], h0 * s * z[1]);
      } else {
        const T hz = hk(0), hn = hk(M);
        row[0].v[0] = mk<T>(hz * z[0], hn * z[1]);   // A_0 + i A_M
      }
    }
  }

  // Z_k of the complex-to-real transform for the thread's first-stage entries.
  __device__ __forceinline__ static void prepare(const E* rowp, const V* tw, int t, V (&x)[1][EN::REG]) {
#pragma unroll
    for (int m = 0; m < R0; ++m) {
      const int k = t + m * NT;
      const V xk = rowp[RL::idx(k)].v[0];
      if (k == 0) {
        x[0][m] = mk<T>(xk.x + xk.y, xk.x - xk.y);
      } else {
        const V xm = cconj(rowp[RL::idx(M - k)].v[0]);
        const V ek = cadd(xk, xm);
        const V ok = cmul(csub(xk, xm), tw[k]);
        x[0][m] = mk<T>(ek.x - ok.y, ek.y + ok.x);
      }
    }
  }

  // Sampling: workgroup bid writes fields bid*RB .. (complex index i of field
  // f at data + f*M + i: reals 2i and 2i+1).
  __device__ __forceinline__ static void run(const Args& a, int bid, char* smem) {
    E* sm = reinterpret_cast<E*>(smem);
    V* tws = reinterpret_cast<V*>(smem + ROWS_BYTES);   // LDS copy (short rows)
    const V* tw = TW_GLOBAL ? (const V*)a.tw2 : tws;
    const int tid = threadIdx.x;
    const int r = tid / NT, t = tid % NT;
    const long long f0 = (long long)bid * RB;
    const long long left = a.rows - f0;
    const int nrows = left < RB ? (int)left : RB;
    if constexpr (!TW_GLOBAL)
      for (int i = tid; i < 2 * M; i += blockDim.x) tws[i] = ((const V*)a.tw2)[i];
    generate(a, f0, nrows, sm, tid);
    __syncthreads();
    const bool act = r < nrows;
    V x[1][EN::REG];
    if (act) prepare(sm + r * RL::STRIDE, tw, t, x);
    __syncthreads();
    V* o = (V*)a.data + (f0 + r) * M;
    auto lds = [&](int i, int off = 0) -> E& { return sm[r * RL::STRIDE + RL::idx(i, off)]; };
    auto out = [&](int i, const E& e) { o[i] = e.v[0]; };
    EN::template run<+1>(x, t, act, lds, tw, out);
  }

  // The two-FFT algorithm on whole fields (Section 3, the first algorithm):
  // the white noise (tag 0, or given rows) as y_n = x_{2n} + i x_{2n+1} into
  // LDS, the forward length-M transform, then per pair (k, M - k) the
  // real-to-complex post-twiddle X_k = E_k + w^{-k} D_k and the filter
  // h_k / sqrt(P) in place (slot 0: A_0 + i A_M, both real), and the same
  // complex-to-real transform as the one-FFT path.
  __device__ __forceinline__ static void run_two_fft(const Args& a, int bid, char* smem) {
    E* sm = reinterpret_cast<E*>(smem);
    V* tws = reinterpret_cast<V*>(smem + ROWS_BYTES);
    const V* tw = TW_GLOBAL ? (const V*)a.tw2 : tws;
    const int tid = threadIdx.x;
    const int r = tid / NT, t = tid % NT;
    const long long f0 = (long long)bid * RB;
    const long long left = a.rows - f0;
    const int nrows = left < RB ? (int)left : RB;
    if constexpr (!TW_GLOBAL)
      for (int i = tid; i < 2 * M; i += blockDim.x) tws[i] = ((const V*)a.tw2)[i];
    constexpr int NQ = M / 2;   // Philox blocks per field
    for (int i = tid; i < nrows * NQ; i += blockDim.x) {
      const int rr = i / NQ, q = i % NQ;
      const long long b = f0 + rr;
      T z[4];
      if (a.src != nullptr) {
        const T* p = (const T*)a.src + b * (2 * M) + 4 * q;
        z[0] = p[0];
        z[1] = p[1];
        z[2] = p[2];
        z[3] = p[3];
      } else {
        const unsigned long long key = a.seed + (unsigned long long)b;
        normals4<T, false>((uint32_t)q, 0u, (uint32_t)a.tag, (uint32_t)key, (uint32_t)(key >> 32), z);
      }
      E* row = sm + rr * RL::STRIDE;
      row[RL::idx(2 * q)].v[0] = mk<T>(z[0], z[1]);
      row[RL::idx(2 * q + 1)].v[0] = mk<T>(z[2], z[3]);
    }
    __syncthreads();
    const bool act = r < nrows;
    auto lds = [&](int i, int off = 0) -> E& { return sm[r * RL::STRIDE + RL::idx(i, off)]; };
    V x[1][EN::REG];
    if (act) {
#pragma unroll
      for (int m = 0; m < R0; ++m) x[0][m] = lds(t + m * NT).v[0];
    }
    stage_sync<WAVE>();   // from here on a row's LDS area is used by its own threads only
    EN::template run<-1>(x, t, act, lds, tw, [&](int i, const E& e) { lds(i) = e; });
    stage_sync<WAVE>();
    if (act) {
      const long long b = f0 + r;
      const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], a.scale);
      const T* ht = (const T*)a.htab;
      const T il2 = (T)a.il2[2];
      auto hk = [&](int k) -> T { return ht ? ht[k] : filt_h(f, (T)(k * k) * il2); };
      for (int k = t; 2 * k <= M; k += NT) {
        if (k == 0) {
          const V y0 = lds(0).v[0];
          lds(0).v[0] = mk<T>(hk(0) * (y0.x + y0.y), hk(M) * (y0.x - y0.y));   // A_0 + i A_M
          continue;
        }
        const int km = M - k;
        const V yk = lds(k).v[0], ym = lds(km).v[0];
        const V ek = cscale(cadd(yk, cconj(ym)), (T)0.5);
        const V dk = cscale(csub(yk, cconj(ym)), (T)0.5);
        const V xk = cadd(ek, cmul(mk<T>(dk.y, -dk.x), cconj(tw[k])));
        const T hkk = hk(k);
        lds(k).v[0] = mk<T>(hkk * xk.x, hkk * xk.y);
        if (km != k) {
          const V em = cscale(cadd(ym, cconj(yk)), (T)0.5);
          const V dm = cscale(csub(ym, cconj(yk)), (T)0.5);
          const V xm = cadd(em, cmul(mk<T>(dm.y, -dm.x), cconj(tw[km])));
          const T hm = hk(km);
          lds(km).v[0] = mk<T>(hm * xm.x, hm * xm.y);
        }
      }
    }
    stage_sync<WAVE>();
    if (act) prepare(sm + r * RL::STRIDE, tw, t, x);
    stage_sync<WAVE>();
    V* o = (V*)a.data + (f0 + r) * M;
    auto out = [&](int i, const E& e) { o[i] = e.v[0]; };
    EN::template run<+1>(x, t, act, lds, tw, out);
  }

  // Covariance estimator: workgroup w takes the field blocks w, w + G, ...
  // (G = gridDim.x) of the a.rows fields, accumulates phi(0) phi(x) in
  // float64, adds its rows in order and writes M complex (= 2M real) partial
  // sums to partial + w * 2M.
  __device__ __forceinline__ static void run_cov(const Args& a, double* partial, char* smem) {
    E* sm = reinterpret_cast<E*>(smem);
    V* tws = reinterpret_cast<V*>(smem + ROWS_BYTES);   // LDS copy (short rows)
    const V* tw = TW_GLOBAL ? (const V*)a.tw2 : tws;
    T* phi0 = reinterpret_cast<T*>(smem + ROWS_BYTES + TW_BYTES);
    const int tid = threadIdx.x;
    const int r = tid / NT, t = tid % NT;
    constexpr int LAST = Rad::count - 1;
    constexpr int RL_ = Rad::get(LAST), NBL = EN::NB(LAST), LRL = M / RL_;
    double acc[NBL * RL_][2];
#pragma unroll
    for (int i = 0; i < NBL * RL_; ++i) acc[i][0] = acc[i][1] = 0.0;
    if constexpr (!TW_GLOBAL)
      for (int i = tid; i < 2 * M; i += blockDim.x) tws[i] = ((const V*)a.tw2)[i];
    for (long long blk = blockIdx.x; blk * RB < a.rows; blk += gridDim.x) {
      const long long f0 = blk * RB;
      const long long left = a.rows - f0;
      const int nrows = left < RB ? (int)left : RB;
      generate(a, f0, nrows, sm, tid);
      __syncthreads();
      const bool act = r < nrows;
      V x[1][EN::REG];
      if (act) prepare(sm + r * RL::STRIDE, tw, t, x);
      __syncthreads();
      auto lds = [&](int i, int off = 0) -> E& { return sm[r * RL::STRIDE + RL::idx(i, off)]; };
      auto none = [&](int, const E&) {};
      EN::template run<+1>(x, t, act, lds, tw, none);
      // x now holds the outputs i = t + b NT + m LRL of the last stage at
      // x[0][b R + m]; phi(0) is the real part of output 0 (thread t = 0).
      if (act && t == 0) phi0[r] = x[0][0].x;
      __syncthreads();
      if (act) {
        const double p0 = (double)phi0[r];
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
          if (NBL * NT == LRL || t + b * NT < LRL) {
#pragma unroll
            for (int m = 0; m < RL_; ++m) {
              acc[b * RL_ + m][0] += p0 * (double)x[0][b * RL_ + m].x;
              acc[b * RL_ + m][1] += p0 * (double)x[0][b * RL_ + m].y;
            }
          }
        }
      }
      __syncthreads();   // phi0 and the rows are rewritten by the next block
    }
    // rows of the workgroup added in order 0 .. RB-1, in the rows area
    double* red = reinterpret_cast<double*>(smem);
    for (int rr = 0; rr < RB; ++rr) {
      if (r == rr) {
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
          const int j = t + b * NT;
          if (NBL * NT == LRL || j < LRL) {
#pragma unroll
            for (int m = 0; m < RL_; ++m) {
              const int i = j + m * LRL;
              if (rr == 0) {
                red[2 * i] = acc[b * RL_ + m][0];
                red[2 * i + 1] = acc[b * RL_ + m][1];
              } else {
                red[2 * i] += acc[b * RL_ + m][0];
                red[2 * i + 1] += acc[b * RL_ + m][1];
              }
            }
          }
        }
      }
      __syncthreads();
    }
    double* pw = partial + (long long)blockIdx.x * 2 * M;
    for (int i = tid; i < 2 * M; i += blockDim.x) pw[i] = red[i];
  }
};

template <typename T, int M, class Rad, int RB>
__global__ void __launch_bounds__((Gen1D<T, M, Rad, RB>::THREADS)) k_gen1d(Args a) {
  using PS = Gen1D<T, M, Rad, RB>;
  __shared__ __align__(16) char smem[PS::LDS_BYTES];
  PS::run(a, blockIdx.x, smem);
}

template <typename T, int M, class Rad, int RB>
__global__ void __launch_bounds__((Gen1D<T, M, Rad, RB>::THREADS)) k_gen1d_two(Args a) {
  using PS = Gen1D<T, M, Rad, RB>;
  __shared__ __align__(16) char smem[PS::LDS_BYTES];
  PS::run_two_fft(a, blockIdx.x, smem);
}

template <typename T, int M, class Rad, int RB>
__global__ void __launch_bounds__((Gen1D<T, M, Rad, RB>::THREADS)) k_gen1d_cov(Args a, double* partial) {
  using PS = Gen1D<T, M, Rad, RB>;
  __shared__ __align__(16) char smem[PS::LDS_BYTES];
  PS::run_cov(a, partial, smem);
}

}  // namespace grf
