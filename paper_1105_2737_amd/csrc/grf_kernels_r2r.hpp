// Reflecting boundaries: cosine (Neumann) and sine (Dirichlet) transforms in
// place of the FFT, the variant named in the introduction and at the start of
// Section 3.
//
// On the cell-centred grid x_j = (j + 1/2) l / N of each axis, a field is
//     phi_j = sum_n a_n z_n prod_i b_i(n_i, j_i)
// over the slot grid (the field's own shape).  Slot n of a cosine axis is the
// mode cos(pi n (j + 1/2) / N) of frequency n / (2l); slot n of a sine axis is
// the mode sin(pi (N - n)(j + 1/2) / N) of frequency (N - n) / (2l); and
// a_n = h(p_n) prod_i sqrt(c(n_i)), c(0) = 1, c(n >= 1) = 2, with h the
// periodic filter sigma sqrt(S(p) / |D|).  z: Philox normals with tag 2,
// indexed by slot as the periodic noise is indexed by point.
//
// sin(pi (N - n)(j + 1/2) / N) = (-1)^j cos(pi n (j + 1/2) / N), so every axis
// is the DCT-III  x_j = sum_{k<N} X_k cos(pi k (j + 1/2) / N)  of the slots,
// with the sign (-1)^j on the output of a sine axis.  A DCT-III of length N
// is one inverse DFT of length N (Makhoul, IEEE Trans. ASSP 28 (1980)):
//     Y_0 = X_0,  Y_k = (1/2) e^{i pi k / (2N)} (X_k - i X_{N-k}),
//     v_m = sum_k Y_k e^{2 pi i k m / N},  x_{2n} = v_n,  x_{2n+1} = v_{N-1-n}.
// Y is linear over the complex numbers in X, so a column pass transforms two
// real columns at once as the real and imaginary parts of one complex column
// (the column pair layout of the periodic passes, unchanged).  Along the last
// axis X is real, Y is Hermitian (Y_{N-k} = conj Y_k, Y_{N/2} = X_{N/2} / sqrt 2)
// and the DFT is the half-length complex-to-real transform of the periodic
// path.
//
// Layout: the field's own (real, last axis contiguous), in place in the
// output.  Passes: generation + axis-1 DCT (column pass), middle-axis DCT
// (d = 3, column pass), last-axis DCT (row pass); d = 1 is one row pass that
// generates its rows.
#pragma once
#include "grf_kernels.hpp"

namespace grf {

// sqrt(c(n)): 1 for slot 0, sqrt 2 otherwise.
template <typename T>
__device__ __forceinline__ T slot_w(int n) {
  return n == 0 ? (T)1 : (T)1.4142135623730950488;
}

// a_n / z_n at slot (n1, no, nd) (axis 1, middle, last); the three factors
// and h in a fixed order, so that the table and the on-the-fly route give the
// same bits.
template <typename T>
__device__ __forceinline__ T r2r_coef(const Args& a, const Filt<T>& f, int n1, int no, int nd) {
  const int k1 = (a.bcmask & 1) ? a.n1 - n1 : n1;
  const int ko = (a.bcmask & 2) ? a.no - no : no;
  const int kd = (a.bcmask & 4) ? a.nd - nd : nd;
  // p^2 = sum (k_i / (2 l_i))^2
  const T p2 = (T)0.25 * ((T)(k1 * k1) * (T)a.il2[0] + (T)(ko * ko) * (T)a.il2[1] + (T)(kd * kd) * (T)a.il2[2]);
  T w = slot_w<T>(nd);
  if (a.n1 > 1) w = w * slot_w<T>(n1);
  if (a.no > 1) w = w * slot_w<T>(no);
  return filt_h(f, p2) * w;
}

// Four consecutive coefficients of row `row` (= n1 * no + no index), last-axis
// slots s .. s + 3 (s a multiple of 4) of field b.  UNIFORM_KEY: every lane of
// the wavefront works on the same field (column passes).
template <typename T, bool UNIFORM_KEY>
__device__ __forceinline__ void r2r_gen4(const Args& a, const Filt<T>& f, int b, uint32_t k0, uint32_t k1, int n1,
                                         int no, int s, T* x) {
  const int row = n1 * a.no + no;
  T z[4];
  if (a.src == nullptr) {
    normals4<T, UNIFORM_KEY>((uint32_t)(s >> 2), (uint32_t)row, (uint32_t)a.tag, k0, k1, z);
  } else {
    const T* p = (const T*)a.src + (long long)b * a.field_stride * 2 + (long long)row * a.nd + s;
#pragma unroll
    for (int e = 0; e < 4; ++e) z[e] = p[e];
  }
  if (a.htab != nullptr) {
    struct alignas(4 * sizeof(T)) P4 { T v[4]; };
    const P4 h = *reinterpret_cast<const P4*>((const T*)a.htab + (long long)row * a.nd + s);
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = h.v[e] * z[e];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = r2r_coef<T>(a, f, n1, no, s + e) * z[e];
  }
}

// Table of a_n / z_n over the slot grid ([rows][N_d], the field's layout) for
// the record a.recs[0].
template <typename T>
__global__ void k_r2r_table(Args a, T* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long P = (long long)a.n1 * a.no * a.nd;
  if (i >= P) return;
  const int s = (int)(i % a.nd);
  const long long row = i / a.nd;
  const Filt<T> f = load_filt<T>(a.recs[0], 1.0);
  out[i] = r2r_coef<T>(a, f, (int)(row / a.no), (int)(row % a.no), s);
}

// Column pass: DCT-III along a leading axis of length L over tiles of CP
// column pairs (4 reals of the last axis per thread and row).  SRC_GEN
// generates the coefficients (axis 1); SRC_LOAD reads the field.
template <typename T, int L, class Rad, int CP, int PAD, int SRC>
struct R2RCol {
  using V = C<T>;
  using E = Vec<T, 2>;
  static constexpr int NT = L / Rad::get(0);
  static constexpr int THREADS = (NT * CP + 63) / 64 * 64;
  static constexpr int RS = CP + PAD;
  static constexpr int R0 = Rad::get(0);
  static constexpr int LDS_BYTES = L * RS * (int)sizeof(E) + 2 * L * (int)sizeof(V);
  using EN = Eng<T, L, Rad, NT, 2, 1>;
  static_assert(L % 2 == 0, "even lengths only");
  // straight-line generation for long columns, as in the periodic column pass
  static constexpr bool GEN_STRAIGHT = L >= 500;

  __device__ __forceinline__ static void run(const Args& a, int bid, char* smem) {
    E* sm = reinterpret_cast<E*>(smem);
    V* tw = reinterpret_cast<V*>(smem + L * RS * sizeof(E));
    V* tq = tw + L;
    const int tid = threadIdx.x;
    const int cp = tid % CP;
    const int t = tid / CP;
    const int tile = bid % a.ntile;
    bid /= a.ntile;
    const int fx = bid % a.nfixed;
    const int b = bid / a.nfixed;
    const int m0 = (tile * CP + cp) * 2;
    const bool act = (t < NT) && (m0 < a.M);
    const bool two = (m0 + 1) < a.M;
    const bool al = (a.M & 1) == 0;
    V* base = (V*)a.data + (long long)b * a.field_stride + (long long)fx * a.stride_fixed + m0;
    for (int i = tid; i < L; i += blockDim.x) {
      tw[i] = ((const V*)a.tw)[i];
      tq[i] = ((const V*)a.tq)[i];
    }
    V x[2][EN::REG];
    if (act) {
      if constexpr (SRC == SRC_GEN) {
        const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], 1.0);
        const unsigned long long key = a.seed + (unsigned long long)b;
        const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
        if (GEN_STRAIGHT && a.src == nullptr && a.htab != nullptr && al) {
          // straight-line: the coefficient loads of all rows first, then the
          // R0 independent Philox blocks (same products as r2r_gen4)
          struct alignas(4 * sizeof(T)) P4 { T v[4]; };
          P4 hc[R0];
#pragma unroll
          for (int m = 0; m < R0; ++m)
            hc[m] = *reinterpret_cast<const P4*>((const T*)a.htab +
                                                 (long long)((t + m * NT) * a.no + fx) * a.nd + 2 * m0);
          T z[R0][4];
#pragma unroll
          for (int m = 0; m < R0; ++m)
            normals4<T, true>((uint32_t)(m0 >> 1), (uint32_t)((t + m * NT) * a.no + fx), (uint32_t)a.tag, k0, k1,
                              z[m]);
#pragma unroll
          for (int m = 0; m < R0; ++m) {
            x[0][m] = mk<T>(hc[m].v[0] * z[m][0], hc[m].v[1] * z[m][1]);
            x[1][m] = mk<T>(hc[m].v[2] * z[m][2], hc[m].v[3] * z[m][3]);
          }
        } else {
#pragma unroll
          for (int m = 0; m < R0; ++m) {
            T v[4];
            r2r_gen4<T, true>(a, f, b, k0, k1, t + m * NT, fx, 2 * m0, v);
            x[0][m] = mk<T>(v[0], v[1]);
            x[1][m] = mk<T>(v[2], v[3]);
          }
        }
      } else {
#pragma unroll
        for (int m = 0; m < R0; ++m)
          ld_pair<T>(base + (long long)(t + m * NT) * a.stride_ax, two, al, x[0][m], x[1][m]);
      }
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        E e;
        e.v[0] = x[0][m];
        e.v[1] = x[1][m];
        sm[(t + m * NT) * RS + cp] = e;
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int k = t + m * NT;
        if (k > 0) {
          const E pr = sm[(L - k) * RS + cp];
          const V q = tq[k];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const V xk = x[c][m], xp = pr.v[c];
            x[c][m] = cmul(mk<T>(xk.x + xp.y, xk.y - xp.x), q);   // (X_k - i X_{L-k}) q
          }
        }
      }
    }
    __syncthreads();
    const bool neg = a.sine != 0;
    auto lds = [&](int i) -> E& { return sm[i * RS + cp]; };
    auto out = [&](int i, const E& e) {
      const int j = 2 * i < L ? 2 * i : 2 * (L - 1 - i) + 1;
      E o = e;
      if (neg && (j & 1)) {
        o.v[0] = mk<T>(-e.v[0].x, -e.v[0].y);
        o.v[1] = mk<T>(-e.v[1].x, -e.v[1].y);
      }
      st_pair<T>(base + (long long)j * a.stride_ax, two, al, o);
    };
    EN::template run<+1>(x, t, act, lds, tw, out);
  }
};

template <typename T, int L, class Rad, int CP, int PAD, int SRC>
__global__ void __launch_bounds__((R2RCol<T, L, Rad, CP, PAD, SRC>::THREADS)) k_r2r_col(Args a) {
  using PS = R2RCol<T, L, Rad, CP, PAD, SRC>;
  __shared__ __align__(16) char smem[PS::LDS_BYTES];
  PS::run(a, col_block(a.order), smem);
}

// Row pass: DCT-III along the last axis (N = 2M reals per row), RB rows per
// workgroup.  SRC_LOAD reads, for each first-stage entry k of the half-length
// inverse DFT, the reals X_k, X_{N-k}, X_{M-k}, X_{M+k} straight from global
// memory (unit stride across lanes, so coalesced); SRC_GEN (d = 1: a row is a
// field) generates the row into LDS first, since a Philox block yields four
// consecutive slots.  The DFT's outputs v_{2i} + i v_{2i+1} go through LDS so
// that each thread writes output pairs (x_{2n}, x_{2n+1}) = (v_n, +-v_{N-1-n})
// as one vector (measured: 25% faster than four-byte stores of each v_m
// straight to its place).
template <typename T, int M, class Rad, int RB, int SRC>
struct R2RRow {
  using V = C<T>;
  using E = Vec<T, 1>;
  using RL = RowLds<M>;
  static constexpr int N = 2 * M;
  static constexpr int NT = M / Rad::get(0);
  static constexpr int THREADS = (NT * RB + 63) / 64 * 64;
  static constexpr int R0 = Rad::get(0);
  static constexpr bool WAVE = (64 % NT) == 0;
  static constexpr int ROWS_BYTES = RB * RL::STRIDE * (int)sizeof(E);
  // The d = 1 kernel (SRC_GEN) reads W_N of long rows through the caches
  // rather than from LDS, as the periodic 1D kernel does (measured at 4096
  // points: 0.838 -> 0.747 ms per 65536 fields); the load pass keeps the LDS
  // copy (2.5% slower without it at 128 x 4096).
  static constexpr bool TW_GLOBAL = SRC == SRC_GEN && M >= 1024;
  // alpha_k, beta_k (2M values) after W_N in LDS for short rows: read from
  // global memory right before their use, the loads went out one at a time
  // (M = 128: the pass 33% slower); long rows keep them in the caches (their
  // LDS would cost occupancy)
  static constexpr bool AB_LDS = !TW_GLOBAL && M <= 512;
  static constexpr int LDS_BYTES =
      ROWS_BYTES + (TW_GLOBAL ? 0 : N * (int)sizeof(V)) + (AB_LDS ? 2 * M * (int)sizeof(V) : 0);
  using EN = Eng<T, M, Rad, NT, 1, 2, WAVE>;
  static_assert(M % 2 == 0, "a Philox block fills two complex slots");

  // Z_k of the complex-to-real transform from X_k, X_{N-k}, X_{M-k}, X_{M+k}
  // (k = 0: X_0 and X_M in x0, x1).  With Y_k = q_k (X_k - i X_{N-k}),
  // q_k = (1/2) e^{i pi k / (2N)}, the half-length transform's input is
  //   Z_k = Y_k + conj Y_{M-k} + i W_N^k (Y_k - conj Y_{M-k})
  //       = (X_k - i X_{N-k}) alpha_k + (X_{M-k} + i X_{M+k}) beta_k
  // with alpha_k = q_k (1 + i W_N^k), beta_k = conj(q_{M-k}) (1 - i W_N^k),
  // tabulated after the q_k (ab = tq + M + 1: alpha_k at k, beta_k at M + k).
  __device__ __forceinline__ static V prep(int k, T x0, T x1, T x2, T x3, const V* ab) {
    if (k == 0) {
      const T y0 = x0, ym = x1 * (T)0.70710678118654752440;
      return mk<T>(y0 + ym, y0 - ym);
    }
    return cadd(cmul(mk<T>(x0, -x1), ab[k]), cmul(mk<T>(x2, x3), ab[M + k]));
  }

  __device__ __forceinline__ static void run(const Args& a, int bid, char* smem) {
    E* sm = reinterpret_cast<E*>(smem);
    V* tws = reinterpret_cast<V*>(smem + ROWS_BYTES);
    const V* tw = TW_GLOBAL ? (const V*)a.tw2 : tws;
    const V* abg = (const V*)a.tq + (M + 1);
    const V* ab = AB_LDS ? tws + N : abg;
    const int tid = threadIdx.x;
    const int r = tid / NT, t = tid % NT;
    const long long row0 = (long long)bid * RB;
    const long long left = a.rows - row0;
    const int nrows = left < RB ? (int)left : RB;
    const bool act = r < nrows;
    V* g = (V*)a.data + row0 * M;
    TwFill<V, TW_GLOBAL ? 1 : N, THREADS> twf;
    TwFill<V, AB_LDS ? 2 * M : 1, THREADS> abf;
    if (!TW_GLOBAL && tid < THREADS) twf.load((const V*)a.tw2, tid);
    if (AB_LDS && tid < THREADS) abf.load(abg, tid);
    V x[1][EN::REG];
    if constexpr (SRC == SRC_GEN) {
      constexpr int NQ = M / 2;   // Philox blocks per row
      for (int i = tid; i < nrows * NQ; i += blockDim.x) {
        const int rr = i / NQ, q = i % NQ;
        const int b = (int)(row0 + rr);
        const Filt<T> f = load_filt<T>(a.recs[b * a.rec_stride], 1.0);
        const unsigned long long key = a.seed + (unsigned long long)b;
        T v[4];
        r2r_gen4<T, false>(a, f, b, (uint32_t)key, (uint32_t)(key >> 32), 0, 0, 4 * q, v);
        E* rowp = sm + rr * RL::STRIDE;
        rowp[RL::idx(2 * q)].v[0] = mk<T>(v[0], v[1]);
        rowp[RL::idx(2 * q + 1)].v[0] = mk<T>(v[2], v[3]);
      }
      if (!TW_GLOBAL && tid < THREADS) twf.store(tws, tid);
      if (AB_LDS && tid < THREADS) abf.store(tws + N, tid);
      __syncthreads();
      const E* rowp = sm + r * RL::STRIDE;
      auto X = [&](int i) -> T {
        const V c = rowp[RL::idx(i >> 1)].v[0];
        return (i & 1) ? c.y : c.x;
      };
      if (act) {
#pragma unroll
        for (int m = 0; m < R0; ++m) {
          const int k = t + m * NT;
          x[0][m] = k == 0 ? prep(0, X(0), X(M), (T)0, (T)0, ab) : prep(k, X(k), X(N - k), X(M - k), X(M + k), ab);
        }
      }
      __syncthreads();   // the rows area is reused by the transform
    } else {
      const T* xr = (const T*)(g + (long long)r * M);
      T xa[R0], xb[R0], xc[R0], xd[R0];
      if (act) {
#pragma unroll
        for (int m = 0; m < R0; ++m) {
          const int k = t + m * NT;
          xa[m] = xr[k];
          xb[m] = xr[k == 0 ? M : N - k];
          xc[m] = xr[k == 0 ? 0 : M - k];
          xd[m] = xr[M + k];
        }
      }
      if (!TW_GLOBAL && tid < THREADS) twf.store(tws, tid);
      if (AB_LDS && tid < THREADS) abf.store(tws + N, tid);
      __syncthreads();
      if (act) {
#pragma unroll
        for (int m = 0; m < R0; ++m) x[0][m] = prep(t + m * NT, xa[m], xb[m], xc[m], xd[m], ab);
      }
    }
    auto lds = [&](int i, int off = 0) -> E& { return sm[r * RL::STRIDE + RL::idx(i, off)]; };
    auto none = [&](int, const E&) {};
    EN::template run<+1>(x, t, act, lds, tw, none);
    // x holds the outputs i = t + b NT + m LRL of the last stage at x[0][b R + m];
    // they go to LDS, and each thread writes pairs (x_{2n}, x_{2n+1}) = (v_n, +-v_{N-1-n})
    constexpr int LAST = Rad::count - 1;
    constexpr int RL_ = Rad::get(LAST), NBL = EN::NB(LAST), LRL = M / RL_;
    __syncthreads();
    if (act) {
#pragma unroll
      for (int b = 0; b < NBL; ++b) {
        const int j = t + b * NT;
        if (NBL * NT == LRL || j < LRL) {
#pragma unroll
          for (int m = 0; m < RL_; ++m) sm[r * RL::STRIDE + RL::idx(j + m * LRL)].v[0] = x[0][b * RL_ + m];
        }
      }
    }
    __syncthreads();
    if (act) {
      // c_u = v_{2u} + i v_{2u+1}: output pairs 2u and 2u + 1 are
      // (v_{2u}, +-v_{N-1-2u}) = (c_u.x, +-c_{M-1-u}.y) and
      // (v_{2u+1}, +-v_{N-2-2u}) = (c_u.y, +-c_{M-1-u}.x), one vector store
      const E* rowp = sm + r * RL::STRIDE;
      const T sg = a.sine ? (T)-1 : (T)1;
      struct alignas(4 * sizeof(T)) P4 { T v[4]; };
      P4* o = reinterpret_cast<P4*>(g + (long long)r * M);
#pragma unroll
      for (int u = t; u < M / 2; u += NT) {
        const V c0 = rowp[RL::idx(u)].v[0];
        const V c1 = rowp[RL::idx(M - 1 - u)].v[0];
        P4 w;
        w.v[0] = c0.x;
        w.v[1] = sg * c1.y;
        w.v[2] = c0.y;
        w.v[3] = sg * c1.x;
        o[u] = w;
      }
    }
  }
};

template <typename T, int M, class Rad, int RB, int SRC>
__global__ void __launch_bounds__((R2RRow<T, M, Rad, RB, SRC>::THREADS)) k_r2r_row(Args a) {
  using PS = R2RRow<T, M, Rad, RB, SRC>;
  __shared__ __align__(16) char smem[PS::LDS_BYTES];
  PS::run(a, blockIdx.x, smem);
}


// ---------------------------------------------------------------------------
// Adjoint.  phi = B (a * z), B the product of the axis bases, so for an
// upstream gradient g:  dL/dz = a * B^T g  and
// dL/dtheta = sum_n (B^T g)_n z_n (a_n / 2) d log S / d theta (p_n).
// B^T along an axis is the DCT-II  X_k = sum_j x_j cos(pi k (j + 1/2) / N)
// of the axis data (times (-1)^j first on a sine axis), again one DFT of
// length N (Makhoul): v_n = x_{2n}, v_{N-1-n} = x_{2n+1}, V = DFT(v) (forward),
// X_k = Re(e^{-i pi k / (2N)} V_k).  Two real columns packed as one complex
// column give A_k = (V_k + conj V_{N-k}) / 2 and B_k = (V_k - conj V_{N-k}) / (2i)
// for the two; a real row gives V from the half-length transform, and
// X_k = Re(W_k), X_{N-k} = -Im(W_k) with W_k = e^{-i pi k / (2N)} V_k.

// squared frequency (float64) of slot (n1, no, nd), for d log S
__device__ __forceinline__ double r2r_p2(const Args& a, int n1, int no, int nd) {
  const int k1 = (a.bcmask & 1) ? a.n1 - n1 : n1;
  const int ko = (a.bcmask & 2) ? a.no - no : no;
  const int kd = (a.bcmask & 4) ? a.nd - nd : nd;
  return 0.25 * ((double)k1 * k1 * a.il2[0] + (double)ko * ko * a.il2[1] + (double)kd * kd * a.il2[2]);
}

// The reduction step of four consecutive slots (row = n1 * no + no index,
// last-axis slots s .. s + 3) of field b with G = (B^T g) there: regenerate
// z (or read it from a.src2), add the terms, write dL/dz to a.aux if asked.
// PRE: the coefficients a_n of the four slots come from cpre (loaded by the
// caller from the plan's table) instead of a load here.
template <typename T, bool UNIFORM_KEY, bool PRE = false>
__device__ __forceinline__ void r2r_adj4(const Args& a, const Filt<T>& f, AdjAcc<T>& ad, int b, uint32_t k0,
                                         uint32_t k1, int n1, int no, int s, const T* G, int nvalid,
                                         const T* cpre = nullptr) {
  const int row = n1 * a.no + no;
  T z[4];
  if (a.src2 == nullptr) {
    normals4<T, UNIFORM_KEY>((uint32_t)(s >> 2), (uint32_t)row, (uint32_t)a.tag, k0, k1, z);
  } else {
    const T* p = (const T*)a.src2 + (long long)b * a.field_stride * 2 + (long long)row * a.nd + s;
#pragma unroll
    for (int e = 0; e < 4; ++e) z[e] = e < nvalid ? p[e] : (T)0;
  }
  T* gz = a.aux ? (T*)a.aux + (long long)b * a.field_stride * 2 + (long long)row * a.nd + s : nullptr;
  if constexpr (sizeof(T) == 4) {
    // float32: the four slots' terms c = a_n z G / 2, c dlogS/dl and
    // c dlogS/dnu formed and summed in float32 (p^2 by the float expression
    // of r2r_coef, dlogS as in AdjAcc::add2f), one float64 add per sum
    const int k1 = (a.bcmask & 1) ? a.n1 - n1 : n1;
    const int ko = (a.bcmask & 2) ? a.no - no : no;
    const float p2r = (float)(k1 * k1) * (float)a.il2[0] + (float)(ko * ko) * (float)a.il2[1];
    const float il2d = (float)a.il2[2];
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (e < nvalid) {
        const float c = PRE ? (float)cpre[e]
                            : a.htab ? ((const float*)a.htab)[(long long)row * a.nd + s + e]
                                     : r2r_coef<float>(a, f, n1, no, s + e);
        const int kd = (a.bcmask & 4) ? a.nd - (s + e) : s + e;
        const float pf = 0.25f * (p2r + (float)(kd * kd) * il2d);
        float dl, dn = 0.0f;
        if (ad.gauss) {
          dl = fmaf(ad.gl1f, pf, ad.gl0f);
        } else {
          const float u = fmaf(ad.rbf, pf, ad.raf);
          const float iu = __builtin_amdgcn_rcpf(u);
          dl = fmaf(ad.gl1f, iu, ad.gl0f);
          if (ad.has_nu) dn = ad.gn0f - __builtin_amdgcn_logf(u) * 0.693147180559945309f - ad.gn1f * iu;
        }
        const float cc = 0.5f * c * ((float)z[e] * (float)G[e]);
        s0 += cc;
        s1 = fmaf(cc, dl, s1);
        s2 = fmaf(cc, dn, s2);
        if (gz) gz[e] = c * G[e];
      }
    }
    ad.acc0 += (double)s0;
    ad.acc1 += (double)s1;
    ad.acc2 += (double)s2;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (e < nvalid) {
        const T c = PRE ? cpre[e]
                        : a.htab ? ((const T*)a.htab)[(long long)row * a.nd + s + e] : r2r_coef<T>(a, f, n1, no, s + e);
        ad.add(1.0, (double)c, r2r_p2(a, n1, no, s + e), mk<T>(z[e], (T)0), mk<T>(G[e], (T)0));
        if (gz) gz[e] = c * G[e];
      }
    }
  }
}

// Column pass: DCT-II along a leading axis, in place (RED = false) or, on
// axis 1, followed by the reduction (RED = true: nothing is written back; the
// workgroup's sums go to a.partial[((b * nfixed + fx) * ntile + tile) * 3 ..]).
template <typename T, int L, class Rad, int CP, int PAD, bool RED>
struct R2RColF {
  using V = C<T>;
  using E = Vec<T, 2>;
  static constexpr int NT = L / Rad::get(0);
  static constexpr int THREADS = (NT * CP + 63) / 64 * 64;
  static constexpr int NW = THREADS / 64;
  static constexpr int RS = CP + PAD;
  static constexpr int R0 = Rad::get(0);
  static constexpr int LDS_BYTES = L * RS * (int)sizeof(E) + 2 * L * (int)sizeof(V) + 3 * NW * (int)sizeof(double);
  using EN = Eng<T, L, Rad, NT, 2, 1>;
  static_assert(L % 2 == 0, "even lengths only");

  __device__ __forceinline__ static void run(const Args& a, int bid, char* smem) {
    E* sm = reinterpret_cast<E*>(smem);
    V* tw = reinterpret_cast<V*>(smem + L * RS * sizeof(E));
    V* tq = tw + L;
    double* red = reinterpret_cast<double*>(tq + L);
    const int tid = threadIdx.x;
    const int cp = tid % CP;
    const int t = tid / CP;
    const int tile = bid % a.ntile;
    const int rest = bid / a.ntile;
    const int fx = rest % a.nfixed;
    const int b = rest / a.nfixed;
    const int m0 = (tile * CP + cp) * 2;
    const bool act = (t < NT) && (m0 < a.M);
    const bool two = (m0 + 1) < a.M;
    const bool al = (a.M & 1) == 0;
    V* base = (V*)a.data + (long long)b * a.field_stride + (long long)fx * a.stride_fixed + m0;
    for (int i = tid; i < L; i += blockDim.x) {
      tw[i] = ((const V*)a.tw)[i];
      tq[i] = ((const V*)a.tq)[i];
    }
    const bool neg = a.sine != 0;
    V x[2][EN::REG];
    if (act) {
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int mm = t + m * NT;
        const int j = 2 * mm < L ? 2 * mm : 2 * (L - 1 - mm) + 1;   // v_mm = x_j
        ld_pair<T>(base + (long long)j * a.stride_ax, two, al, x[0][m], x[1][m]);
        if (neg && (j & 1)) {
          x[0][m] = mk<T>(-x[0][m].x, -x[0][m].y);
          x[1][m] = mk<T>(-x[1][m].x, -x[1][m].y);
        }
      }
    }
    // the reduction's coefficients a_n from the plan's table, requested here
    // so that their latency overlaps the transform
    T cq[RED ? R0 : 1][4];
    const bool pre = RED && act && a.htab != nullptr;
    if constexpr (RED) {
      if (pre) {
#pragma unroll
        for (int m = 0; m < R0; ++m) {
          const T* cp4 = (const T*)a.htab + (long long)((t + m * NT) * a.no + fx) * a.nd + 2 * m0;
          cq[m][0] = cp4[0];
          cq[m][1] = cp4[1];
          cq[m][2] = two ? cp4[2] : (T)0;
          cq[m][3] = two ? cp4[3] : (T)0;
        }
      }
    }
    __syncthreads();   // the twiddle tables
    auto lds = [&](int i) -> E& { return sm[i * RS + cp]; };
    auto none = [&](int, const E&) {};
    EN::template run<-1>(x, t, act, lds, tw, none);
    constexpr int LAST = Rad::count - 1;
    constexpr int RL_ = Rad::get(LAST), NBL = EN::NB(LAST), LRL = L / RL_;
    __syncthreads();
    if (act) {
#pragma unroll
      for (int bb = 0; bb < NBL; ++bb) {
        const int j = t + bb * NT;
        if (NBL * NT == LRL || j < LRL) {
#pragma unroll
          for (int m = 0; m < RL_; ++m) {
            E e;
            e.v[0] = x[0][bb * RL_ + m];
            e.v[1] = x[1][bb * RL_ + m];
            sm[(j + m * LRL) * RS + cp] = e;
          }
        }
      }
    }
    __syncthreads();
    double acc0 = 0, acc1 = 0, acc2 = 0;
    if (act) {
      const FieldRec& rec = a.recs[b * a.rec_stride];
      const Filt<T> f = load_filt<T>(rec, 1.0);
      AdjAcc<T> ad(rec);
      const unsigned long long key = a.seed + (unsigned long long)b;
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int k = t + m * NT;
        const E vk = sm[k * RS + cp];
        const E vm = sm[((L - k) % L) * RS + cp];
        const V q = mk<T>((T)2 * tq[k].x, (T)-2 * tq[k].y);   // e^{-i pi k / (2L)}
        T X[4];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const V A = mk<T>((T)0.5 * (vk.v[c].x + vm.v[c].x), (T)0.5 * (vk.v[c].y - vm.v[c].y));
          const V B = mk<T>((T)0.5 * (vk.v[c].y + vm.v[c].y), (T)-0.5 * (vk.v[c].x - vm.v[c].x));
          X[2 * c] = fmat(q.x, A.x, -(q.y * A.y));
          X[2 * c + 1] = fmat(q.x, B.x, -(q.y * B.y));
        }
        if constexpr (RED) {
          if (pre)
            r2r_adj4<T, true, true>(a, f, ad, b, (uint32_t)key, (uint32_t)(key >> 32), k, fx, 2 * m0, X, two ? 4 : 2,
                                    cq[m]);
          else
            r2r_adj4<T, true>(a, f, ad, b, (uint32_t)key, (uint32_t)(key >> 32), k, fx, 2 * m0, X, two ? 4 : 2);
        } else {
          E o;
          o.v[0] = mk<T>(X[0], X[1]);
          o.v[1] = mk<T>(X[2], X[3]);
          st_pair<T>(base + (long long)k * a.stride_ax, two, al, o);
        }
      }
      acc0 = ad.acc0 * rec.gs;
      acc1 = ad.acc1;
      acc2 = ad.acc2;
    }
    if constexpr (RED) {
      for (int off = 32; off > 0; off >>= 1) {
        acc0 += __shfl_xor(acc0, off);
        acc1 += __shfl_xor(acc1, off);
        acc2 += __shfl_xor(acc2, off);
      }
      const int lane = tid & 63, wv = tid >> 6;
      if (lane == 0) {
        red[wv] = acc0;
        red[NW + wv] = acc1;
        red[2 * NW + wv] = acc2;
      }
      __syncthreads();
      if (tid < 3) {
        double sacc = 0;
        for (int w = 0; w < NW; ++w) sacc += red[tid * NW + w];
        a.partial[((long long)(b * a.nfixed + fx) * a.ntile + tile) * 3 + tid] = sacc;
      }
    }
  }
};

template <typename T, int L, class Rad, int CP, int PAD, bool RED>
__global__ void __launch_bounds__((R2RColF<T, L, Rad, CP, PAD, RED>::THREADS)) k_r2r_colf(Args a) {
  using PS = R2RColF<T, L, Rad, CP, PAD, RED>;
  __shared__ __align__(16) char smem[PS::LDS_BYTES];
  PS::run(a, col_block(a.order), smem);
}

// Row pass: DCT-II along the last axis of the rows of a.src into a.data
// (RED = false), or (RED = true, d = 1, a row is a field) followed by the
// reduction: each row's sums go to a.partial[field * 3 ..].
template <typename T, int M, class Rad, int RB, bool RED>
struct R2RRowF {
  using V = C<T>;
  using E = Vec<T, 1>;
  using RL = RowLds<M>;
  static constexpr int N = 2 * M;
  static constexpr int NT = M / Rad::get(0);
  static constexpr int THREADS = (NT * RB + 63) / 64 * 64;
  static constexpr int R0 = Rad::get(0);
  static constexpr bool WAVE = (64 % NT) == 0;
  static constexpr int ROWS_BYTES = RB * RL::STRIDE * (int)sizeof(E);
  static constexpr int RED_BYTES = RED ? 3 * THREADS * (int)sizeof(double) : 0;
  static constexpr bool TW_GLOBAL = RED && M >= 1024;   // as R2RRow: the d = 1 kernel only
  static constexpr int TW_BYTES = TW_GLOBAL ? 0 : N * (int)sizeof(V);
  static constexpr int LDS_BYTES = ROWS_BYTES + TW_BYTES + RED_BYTES;
  using EN = Eng<T, M, Rad, NT, 1, 2, WAVE>;

  __device__ __forceinline__ static void run(const Args& a, int bid, char* smem) {
    E* sm = reinterpret_cast<E*>(smem);
    V* tws = reinterpret_cast<V*>(smem + ROWS_BYTES);
    const V* tw = TW_GLOBAL ? (const V*)a.tw2 : tws;
    double* red = reinterpret_cast<double*>(smem + ROWS_BYTES + TW_BYTES);
    const V* tq = (const V*)a.tq;
    const int tid = threadIdx.x;
    const int r = tid / NT, t = tid % NT;
    const long long row0 = (long long)bid * RB;
    const long long left = a.rows - row0;
    const int nrows = left < RB ? (int)left : RB;
    const bool act = r < nrows;
    TwFill<V, TW_GLOBAL ? 1 : N, THREADS> twf;
    if (tid < THREADS) {
      if (!TW_GLOBAL) twf.load((const V*)a.tw2, tid);
      copy_in<T, M, RB * M, THREADS>((const V*)a.src + row0 * M, sm, nrows * M, tid);
      if (!TW_GLOBAL) twf.store(tws, tid);
    }
    __syncthreads();
    E* rowp = sm + r * RL::STRIDE;
    auto X = [&](int i) -> T {
      const V c = rowp[RL::idx(i >> 1)].v[0];
      return (i & 1) ? c.y : c.x;
    };
    const bool neg = a.sine != 0;
    // v_m = x_rho(m) (times (-1)^rho(m) on a sine axis), z_n = v_{2n} + i v_{2n+1}
    auto v = [&](int m) -> T {
      const int j = m < M ? 2 * m : 2 * (N - 1 - m) + 1;
      const T xv = X(j);
      return (neg && (j & 1)) ? -xv : xv;
    };
    V x[1][EN::REG];
    if (act) {
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int n = t + m * NT;
        x[0][m] = mk<T>(v(2 * n), v(2 * n + 1));
      }
    }
    __syncthreads();
    auto lds = [&](int i, int off = 0) -> E& { return rowp[RL::idx(i, off)]; };
    auto none = [&](int, const E&) {};
    EN::template run<-1>(x, t, act, lds, tw, none);
    constexpr int LAST = Rad::count - 1;
    constexpr int RL_ = Rad::get(LAST), NBL = EN::NB(LAST), LRL = M / RL_;
    __syncthreads();
    if (act) {
#pragma unroll
      for (int bb = 0; bb < NBL; ++bb) {
        const int j = t + bb * NT;
        if (NBL * NT == LRL || j < LRL) {
#pragma unroll
          for (int m = 0; m < RL_; ++m) rowp[RL::idx(j + m * LRL)].v[0] = x[0][bb * RL_ + m];
        }
      }
    }
    __syncthreads();
    // V_k = E_k + e^{-2 pi i k / N} O_k from Z_k and Z_{M-k}; W_k = e^{-i pi k/(2N)} V_k
    T xo[R0][2];
    T xm = (T)0;
    if (act) {
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int k = t + m * NT;
        const V zk = rowp[RL::idx(k)].v[0];
        const V zc = cconj(rowp[RL::idx(k == 0 ? 0 : M - k)].v[0]);
        const V Ek = mk<T>((T)0.5 * (zk.x + zc.x), (T)0.5 * (zk.y + zc.y));
        const V Ok = mk<T>((T)0.5 * (zk.y - zc.y), (T)-0.5 * (zk.x - zc.x));
        const V Vk = cadd(Ek, cmul(Ok, cconj(tw[k])));
        const V q = mk<T>((T)2 * tq[k].x, (T)-2 * tq[k].y);
        const V W = cmul(q, Vk);
        xo[m][0] = W.x;    // X_k
        xo[m][1] = -W.y;   // X_{N-k} (k > 0)
      }
      if (t == 0) {   // k = M: V_M = Re Z_0 - Im Z_0 (real), X_M = V_M / sqrt 2
        const V z0 = rowp[RL::idx(0)].v[0];
        xm = (z0.x - z0.y) * (T)0.70710678118654752440;
      }
    }
    __syncthreads();
    auto Xw = [&](int i, T val) {   // real i of the row, in the RowLds layout of pairs
      const int c = RL::idx(i >> 1);
      reinterpret_cast<T*>(&rowp[c].v[0])[i & 1] = val;
    };
    if (act) {
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int k = t + m * NT;
        Xw(k, xo[m][0]);
        if (k > 0) Xw(N - k, xo[m][1]);
      }
      if (t == 0) Xw(M, xm);
    }
    __syncthreads();
    if constexpr (!RED) {
      if (act) {
        V* o = (V*)a.data + (row0 + r) * M;
        for (int n = t; n < M; n += NT) o[n] = rowp[RL::idx(n)].v[0];
      }
    } else {
      double acc0 = 0, acc1 = 0, acc2 = 0;
      if (act) {
        const int b = (int)(row0 + r);
        const FieldRec& rec = a.recs[b * a.rec_stride];
        const Filt<T> f = load_filt<T>(rec, 1.0);
        AdjAcc<T> ad(rec);
        const unsigned long long key = a.seed + (unsigned long long)b;
        // the thread's slots 4 q4 .. 4 q4 + 3, q4 = t + i NT < M / 2; their
        // coefficients from the plan's table all requested before the first
        // is used
        constexpr int NQ4 = (R0 + 1) / 2;
        T cq[NQ4][4];
        const bool pre = a.htab != nullptr;
        if (pre) {
#pragma unroll
          for (int i = 0; i < NQ4; ++i) {
            const int q4 = t + i * NT;
            if (q4 < M / 2) {
#pragma unroll
              for (int e = 0; e < 4; ++e) cq[i][e] = ((const T*)a.htab)[4 * q4 + e];
            }
          }
        }
#pragma unroll
        for (int i = 0; i < NQ4; ++i) {
          const int q4 = t + i * NT;
          if (q4 < M / 2) {
            const V p0 = rowp[RL::idx(2 * q4)].v[0], p1 = rowp[RL::idx(2 * q4 + 1)].v[0];
            const T G[4] = {p0.x, p0.y, p1.x, p1.y};
            if (pre)
              r2r_adj4<T, false, true>(a, f, ad, b, (uint32_t)key, (uint32_t)(key >> 32), 0, 0, 4 * q4, G, 4, cq[i]);
            else
              r2r_adj4<T, false>(a, f, ad, b, (uint32_t)key, (uint32_t)(key >> 32), 0, 0, 4 * q4, G, 4);
          }
        }
        acc0 = ad.acc0 * rec.gs;
        acc1 = ad.acc1;
        acc2 = ad.acc2;
      }
      red[tid] = acc0;
      red[THREADS + tid] = acc1;
      red[2 * THREADS + tid] = acc2;
      __syncthreads();
      if (act && t == 0) {
        for (int c = 0; c < 3; ++c) {
          double sacc = 0;
          for (int i = 0; i < NT; ++i) sacc += red[c * THREADS + r * NT + i];
          a.partial[(row0 + r) * 3 + c] = sacc;
        }
      }
    }
  }
};

template <typename T, int M, class Rad, int RB, bool RED>
__global__ void __launch_bounds__((R2RRowF<T, M, Rad, RB, RED>::THREADS)) k_r2r_rowf(Args a) {
  using PS = R2RRowF<T, M, Rad, RB, RED>;
  __shared__ __align__(16) char smem[PS::LDS_BYTES];
  PS::run(a, blockIdx.x, smem);
}

}  // namespace grf
