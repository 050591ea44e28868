// Transforms of any even 2/3/5-smooth length: the passes of the sampler for
// lengths that have no compile-time kernel (grf_configs.hpp).
//
// The same Stockham autosort recursion as the fixed-length engine (Eng in
// grf_kernels.hpp), with the radix list a runtime argument (Args::gs,
// Args::grad, produced on the host by a generator: radices 8 first, then
// 4 or 2, then 5 and 3).  Every stage goes LDS -> registers -> LDS: each
// thread loads the inputs of its butterflies, the workgroup synchronises, the
// thread writes the outputs, the workgroup synchronises.  NT = ceil(L / VPT)
// threads per transform (VPT = 4 or 8 values per thread, a tuning choice; 4
// untuned), so
// a thread holds at most VPT + R values of a stage (NB(R) = ceil(VPT / R)
// butterflies); the radix is dispatched per stage to a body compiled for it,
// so that these values stay in registers.  Twiddles
// W_L are read from the plan's table in global memory (cached).  Transform
// data live in dynamic LDS: column passes take CP column pairs per workgroup
// (one Vec<T, 2> per row), row passes RB rows (one complex per element).
#pragma once
#include "grf_kernels.hpp"

namespace grf {

// One stage of radix R (Ns = product of the radices before it) over the
// transform whose element i is acc(i); act: this thread holds a transform.
template <typename T, int NC, int R, int DIR, int VPT, class Acc>
__device__ __forceinline__ void gstage(Acc acc, int t, int NT, int L, int Ns, const C<T>* tw, int tws, bool act) {
  using V = C<T>;
  using E = Vec<T, NC>;
  constexpr int NB = (VPT + R - 1) / R;
  const int LR = L / R;
  const int tstep = L / (Ns * R);
  // j / Ns by one float product: (j + 1/2) / Ns lies at least 1 / (2 Ns) from
  // an integer, and for j < L <= 2^20 the product's relative error (below
  // 2^-22) moves it by less than that, so its integer part is exact (an
  // integer division by a runtime value costs ~25 VALU instructions)
  const float ins = 1.0f / (float)Ns;
  auto quo = [&](int j) -> int { return (int)(((float)j + 0.5f) * ins); };
  V v[NB][NC][R];
  V w[NB][R];   // the butterflies' twiddles (w[i][0] unused)
  if (act) {
    // every LDS value and twiddle of the thread's butterflies requested
    // before any is used, so that their latencies overlap
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (j < LR) {
        const int k = j - quo(j) * Ns;
#pragma unroll
        for (int m = 0; m < R; ++m) {
          const E e = acc(j + m * LR);
#pragma unroll
          for (int c = 0; c < NC; ++c) v[i][c][m] = e.v[c];
        }
        if (Ns > 1) {
#pragma unroll
          for (int m = 1; m < R; ++m) w[i][m] = tw[tws * (m * k * tstep)];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (j < LR) {
        if (Ns > 1) {
#pragma unroll
          for (int m = 1; m < R; ++m) {
#pragma unroll
            for (int c = 0; c < NC; ++c) v[i][c][m] = ctw<DIR>(v[i][c][m], w[i][m]);
          }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) Dft<R, DIR, V>::run(v[i][c]);
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if (j < LR) {
        const int q = quo(j);
        const int base = q * Ns * R + (j - q * Ns);
#pragma unroll
        for (int m = 0; m < R; ++m) {
          E e;
#pragma unroll
          for (int c = 0; c < NC; ++c) e.v[c] = v[i][c][m];
          acc(base + m * Ns) = e;
        }
      }
    }
  }
  __syncthreads();
}

// The whole transform of length L = prod a.grad[0 .. a.gs-1], in place in
// LDS (natural order in and out).
template <typename T, int NC, int DIR, int VPT, class Acc>
__device__ __forceinline__ void grun(const Args& a, Acc acc, int t, int NT, int L, const C<T>* tw, int tws, bool act) {
  int Ns = 1;
  for (int s = 0; s < a.gs; ++s) {
    const int R = a.grad[s];
    switch (R) {
      case 2: gstage<T, NC, 2, DIR, VPT>(acc, t, NT, L, Ns, tw, tws, act); break;
      case 3: gstage<T, NC, 3, DIR, VPT>(acc, t, NT, L, Ns, tw, tws, act); break;
      case 4: gstage<T, NC, 4, DIR, VPT>(acc, t, NT, L, Ns, tw, tws, act); break;
      case 5: gstage<T, NC, 5, DIR, VPT>(acc, t, NT, L, Ns, tw, tws, act); break;
      default: gstage<T, NC, 8, DIR, VPT>(acc, t, NT, L, Ns, tw, tws, act); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------
// Column pass of length L = a.gl along a leading axis: CP = a.gcp column pairs
// per workgroup, NT = a.gnt threads per column; source = the one-FFT
// algorithm's noise generation (Hermitian arrangement + filter, gen_pair) or a
// global load; direction DIR.  Tiles, fields and the XCD-grouped order as in
// ColPass.
template <typename T, int SRC, int DIR, int VPT>
__global__ void __launch_bounds__(1024) k_gcol(Args a) {
  using V = C<T>;
  using E = Vec<T, 2>;
  extern __shared__ __align__(16) char gsm[];
  E* sm = reinterpret_cast<E*>(gsm);
  const int L = a.gl, CP = a.gcp, NT = a.gnt, RS = a.grs;
  const int tid = threadIdx.x;
  const int cp = tid % CP;
  const int t = tid / CP;
  int bid = col_block(a.order);
  const int tile = bid % a.ntile;
  bid /= a.ntile;
  const int fx = bid % a.nfixed;
  const int b = bid / a.nfixed;
  const int m0 = (tile * CP + cp) * 2;
  const bool act = (t < NT) && (m0 < a.M);
  const bool two = (m0 + 1) < a.M;
  const bool al = (a.M & 1) == 0;
  V* base = (V*)a.data + (long long)b * a.field_stride + (long long)fx * a.stride_fixed + m0;
  auto acc = [&](int i) -> E& { return sm[i * RS + cp]; };
  if (act) {
    if constexpr (SRC == SRC_GEN) {
      const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], a.scale);
      const unsigned long long key = a.seed + (unsigned long long)b;
      const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
      for (int k = t; k < L; k += NT) {
        E e;
        gen_pair<T>(a, f, (const T*)a.src, b, k0, k1, k, fx, m0, e.v[0], e.v[1]);
        acc(k) = e;
      }
    } else {
      // NT = ceil(L / VPT): the thread's elements are t + i NT, i < VPT; all
      // loads issued before the first LDS store
      E xr[VPT];
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = t + i * NT;
        if (k < L) ld_pair<T>(base + (long long)k * a.stride_ax, two, al, xr[i].v[0], xr[i].v[1]);
      }
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = t + i * NT;
        if (k < L) acc(k) = xr[i];
      }
    }
  }
  __syncthreads();
  grun<T, 2, DIR, VPT>(a, acc, t, NT, L, (const V*)a.tw, 1, act);
  if (act) {
    for (int k = t; k < L; k += NT) st_pair<T>(base + (long long)k * a.stride_ax, two, al, acc(k));
  }
}

// ---------------------------------------------------------------------------
// Last-axis complex-to-real pass of half-length M = a.gl: RB = a.gcp rows per
// workgroup, NT = a.gnt threads per row.  Row data X_k (packed slot 0 =
// (X_0, X_M)) become Z_k = E_k + i O_k as in RowC2R, Z is inverse transformed
// (length M, twiddles W_M = W_{N_d}[2 i]) and z_n is stored as
// (x[2n], x[2n+1]).  SRC_GEN (d = 1, the rows are whole fields): the row's
// half-spectrum is generated first (the one-FFT arrangement with the filter),
// then transformed the same way.
template <typename T, int SRC, int VPT>
__global__ void __launch_bounds__(1024) k_grow_c2r(Args a) {
  using V = C<T>;
  using E = Vec<T, 1>;
  extern __shared__ __align__(16) char gsm[];
  E* sm = reinterpret_cast<E*>(gsm);
  const int M = a.gl, RB = a.gcp, NT = a.gnt, RS = a.grs;
  const int tid = threadIdx.x;
  const int r = tid / NT;
  const int t = tid % NT;
  const long long row = (long long)blockIdx.x * RB + r;
  const bool act = (r < RB) && (row < a.rows);
  const V* tw2 = (const V*)a.tw2;
  V* o = (V*)a.data + row * M;
  auto acc = [&](int i) -> E& { return sm[r * RS + i]; };
  if (act) {
    if constexpr (SRC == SRC_GEN) {
      // each row is a field (its own key): entries m0, m0 + 1 from one Philox
      // block (gen_pair)
      const long long b = row;
      const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], a.scale);
      const unsigned long long key = a.seed + (unsigned long long)b;
      const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
      for (int q = t; 2 * q < M; q += NT) {
        V A0, A1;
        gen_pair<T, false, false>(a, f, (const T*)a.src, (int)b, k0, k1, 0, 0, 2 * q, A0, A1);
        acc(2 * q).v[0] = A0;
        if (2 * q + 1 < M) acc(2 * q + 1).v[0] = A1;
      }
    } else {
      // NT = ceil(M / VPT): elements t + i NT, i < VPT, all loads issued first
      V xr[VPT];
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = t + i * NT;
        if (k < M) xr[i] = o[k];
      }
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = t + i * NT;
        if (k < M) acc(k).v[0] = xr[i];
      }
    }
  }
  // the pre-twiddle's factors, requested before the barrier: the thread's
  // pairs are k = t + i NT with 2k <= M, i.e. i <= VPT / 2
  constexpr int NPT = VPT / 2 + 1;
  V wk[NPT], wm[NPT];
  if (act) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int k = t + i * NT;
      if (k > 0 && 2 * k <= M) {
        wk[i] = tw2[k];
        wm[i] = tw2[M - k];
      }
    }
  }
  __syncthreads();
  // pre-twiddle, pairs (k, M - k) by one thread (in place)
  if (act) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int k = t + i * NT;
      if (2 * k > M) continue;
      if (k == 0) {
        const V x0 = acc(0).v[0];
        acc(0).v[0] = mk<T>(x0.x + x0.y, x0.x - x0.y);
        continue;
      }
      const int km = M - k;
      const V xk = acc(k).v[0], xm = acc(km).v[0];
      {
        const V c = cconj(xm);
        const V ek = cadd(xk, c);
        const V ok = cmul(csub(xk, c), wk[i]);
        acc(k).v[0] = mk<T>(ek.x - ok.y, ek.y + ok.x);
      }
      if (km != k) {
        const V c = cconj(xk);
        const V ek = cadd(xm, c);
        const V ok = cmul(csub(xm, c), wm[i]);
        acc(km).v[0] = mk<T>(ek.x - ok.y, ek.y + ok.x);
      }
    }
  }
  __syncthreads();
  grun<T, 1, +1, VPT>(a, acc, t, NT, M, tw2, 2, act);
  if (act) {
    for (int n = t; n < M; n += NT) o[n] = acc(n).v[0];
  }
}

// ---------------------------------------------------------------------------
// Last-axis real-to-complex pass of half-length M = a.gl (the two-FFT
// algorithm's white noise, or a stored real row): y_n = x_{2n} + i x_{2n+1},
// forward transform, then X_k = E_k + w^{-k} D_k as in RowR2C, slot 0 =
// (X_0, X_M).  The generated noise: Philox block (q, row, tag, 0) of field b
// gives slots 4q .. 4q + 3 of the row.
template <typename T, int SRC, int VPT>
__global__ void __launch_bounds__(1024) k_grow_r2c(Args a) {
  using V = C<T>;
  using E = Vec<T, 1>;
  extern __shared__ __align__(16) char gsm[];
  E* sm = reinterpret_cast<E*>(gsm);
  const int M = a.gl, RB = a.gcp, NT = a.gnt, RS = a.grs;
  const int tid = threadIdx.x;
  const int r = tid / NT;
  const int t = tid % NT;
  const long long row = (long long)blockIdx.x * RB + r;
  const bool act = (r < RB) && (row < a.rows);
  const V* tw2 = (const V*)a.tw2;
  auto acc = [&](int i) -> E& { return sm[r * RS + i]; };
  if (act) {
    if constexpr (SRC == SRC_LOAD) {
      const V* src = (const V*)a.src + row * M;
      V xr[VPT];
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = t + i * NT;
        if (k < M) xr[i] = src[k];
      }
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = t + i * NT;
        if (k < M) acc(k).v[0] = xr[i];
      }
    } else {
      const long long b = row / a.rows_per_field;
      const int frow = (int)(row - b * a.rows_per_field);
      const unsigned long long key = a.seed + (unsigned long long)b;
      for (int q = t; 2 * q < M; q += NT) {
        T z[4];
        normals4<T>((uint32_t)q, (uint32_t)frow, (uint32_t)a.tag, (uint32_t)key, (uint32_t)(key >> 32), z);
        acc(2 * q).v[0] = mk<T>(z[0], z[1]);
        if (2 * q + 1 < M) acc(2 * q + 1).v[0] = mk<T>(z[2], z[3]);
      }
    }
  }
  __syncthreads();
  constexpr int NPT = VPT / 2 + 1;
  V wk[NPT], wm[NPT];
  if (act) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int k = t + i * NT;
      if (k > 0 && 2 * k <= M) {
        wk[i] = tw2[k];
        wm[i] = tw2[M - k];
      }
    }
  }
  grun<T, 1, -1, VPT>(a, acc, t, NT, M, tw2, 2, act);
  if (act) {
    V* o = (V*)a.data + row * M;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int k = t + i * NT;
      if (2 * k > M) continue;
      if (k == 0) {
        const V y0 = acc(0).v[0];
        o[0] = mk<T>(y0.x + y0.y, y0.x - y0.y);
        continue;
      }
      const int km = M - k;
      const V yk = acc(k).v[0], ym = acc(km).v[0];
      const V ek = cscale(cadd(yk, cconj(ym)), (T)0.5);
      const V dk = cscale(csub(yk, cconj(ym)), (T)0.5);
      const V dki = mk<T>(dk.y, -dk.x);
      o[k] = cadd(ek, cmul(dki, cconj(wk[i])));
      if (km != k) {
        const V em = cscale(cadd(ym, cconj(yk)), (T)0.5);
        const V dm = cscale(csub(ym, cconj(yk)), (T)0.5);
        const V dmi = mk<T>(dm.y, -dm.x);
        o[km] = cadd(em, cmul(dmi, cconj(wm[i])));
      }
    }
  }
}

}  // namespace grf
