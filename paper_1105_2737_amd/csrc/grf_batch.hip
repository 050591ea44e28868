// Persistent launches for batches of fields of different sizes (d = 2,
// one-FFT algorithm, float32).  See grf_batch.hpp.
//
// Both passes reuse the kernel bodies of the single-plan sampler (ColPass,
// and RowC2RStaged, the LDS-staged form of RowC2R with the same arithmetic),
// so a field sampled in a batch with the plan path's radix order has the same
// bits as the same field sampled by a plan.  In the two-launch route column
// workgroups have 256 threads and at most ~48 KB of LDS (three per CU at the
// column bodies' register use), row workgroups 512 threads and at most ~70 KB
// (two per CU), and each length has two tile shapes (the second with half the
// columns / rows per workgroup).  The one-launch kernel (512 threads, two
// workgroups per CU) has four bodies per length: those two tile shapes and two
// of another radix order (another number of threads per transform).  The
// autotuner chooses among them.
#include "grf_batch.hpp"
#include "grf_configs.hpp"
#include "grf_kernels.hpp"

#include <type_traits>

namespace grf {

// (length, column pairs variant 0, variant 1)
#define GRF_BATCH_COL(X) X(64, 32, 16) X(96, 16, 8) X(128, 16, 8) X(180, 7, 4) X(256, 8, 4) \
  X(360, 2, 1) X(500, 4, 2) X(512, 4, 2) X(1000, 2, 1) X(1024, 2, 1)
// (half-length, rows variant 0, variant 1)
#define GRF_BATCH_ROW(X) X(32, 128, 64) X(48, 64, 32) X(64, 64, 32) X(96, 42, 21) X(128, 64, 32) \
  X(180, 14, 7) X(256, 16, 8) X(360, 11, 5) X(500, 10, 5) X(512, 8, 4)

// Another radix order, i.e. another number of threads per transform (L / R_0),
// per length: variants 2 and 3 of the one-launch kernel's bodies (tile shapes
// CPA / RBA and CPB / RBB), variants 0 and 1 being the plan path's radix
// order with two tile shapes.  A field's bits depend on its radix order, not
// on its tile shape.
template <int L> struct BatchAltCol;
#define GRF_ALTCOL(L_, CPA_, CPB_, ...)                   \
  template <> struct BatchAltCol<L_> {                    \
    using Rad = Radices<__VA_ARGS__>;                     \
    static constexpr int CPA = CPA_, CPB = CPB_;          \
  };
GRF_ALTCOL(64, 32, 16, 4, 4, 4)
GRF_ALTCOL(96, 21, 10, 4, 8, 3)
GRF_ALTCOL(128, 16, 8, 4, 8, 4)
GRF_ALTCOL(180, 16, 8, 6, 6, 5)
GRF_ALTCOL(256, 8, 4, 4, 8, 8)
GRF_ALTCOL(360, 8, 4, 6, 6, 10)
GRF_ALTCOL(500, 4, 2, 5, 10, 10)
GRF_ALTCOL(512, 4, 2, 4, 8, 4, 4)
GRF_ALTCOL(1000, 4, 2, 8, 5, 5, 5)
GRF_ALTCOL(1024, 2, 1, 4, 4, 8, 8)
#undef GRF_ALTCOL
template <int M> struct BatchAltRow;
#define GRF_ALTROW(M_, RBA_, RBB_, ...)                   \
  template <> struct BatchAltRow<M_> {                    \
    using Rad = Radices<__VA_ARGS__>;                     \
    static constexpr int RBA = RBA_, RBB = RBB_;          \
  };
GRF_ALTROW(32, 64, 32, 4, 8)
GRF_ALTROW(48, 64, 32, 8, 6)
GRF_ALTROW(64, 32, 16, 4, 4, 4)
GRF_ALTROW(96, 21, 10, 4, 4, 6)
GRF_ALTROW(128, 32, 16, 8, 4, 4)
GRF_ALTROW(180, 16, 8, 6, 6, 5)
GRF_ALTROW(256, 32, 16, 16, 16)
GRF_ALTROW(360, 12, 6, 9, 5, 8)
GRF_ALTROW(500, 5, 2, 5, 10, 10)
GRF_ALTROW(512, 16, 8, 16, 8, 4)
#undef GRF_ALTROW

// (FLY = false: the per-field filter is evaluated by the per-row route; the
// straight-line form's registers would be the whole persistent kernel's)
template <int L, int CP, bool ALT = false>
using BColPass = ColPass<float, L, typename std::conditional<ALT, BatchAltCol<L>, ColCfg<L>>::type::Rad, CP,
                         ColCfg<L>::PAD, SRC_GEN, +1, false>;
template <int M, int RB, bool ALT = false>
using BRowPass = RowC2RStaged<float, M, typename std::conditional<ALT, BatchAltRow<M>, RowCfg<M>>::type::Rad, RB, 0>;

// LDS of the largest body
#define GRF_COL_LDS(L_, A_, B_) (BColPass<L_, A_>::LDS_BYTES > BColPass<L_, B_>::LDS_BYTES ? BColPass<L_, A_>::LDS_BYTES : BColPass<L_, B_>::LDS_BYTES),
#define GRF_ROW_LDS(M_, A_, B_) (BRowPass<M_, A_>::LDS_BYTES > BRowPass<M_, B_>::LDS_BYTES ? BRowPass<M_, A_>::LDS_BYTES : BRowPass<M_, B_>::LDS_BYTES),
constexpr int col_lds_list[] = {GRF_BATCH_COL(GRF_COL_LDS) 0};
constexpr int row_lds_list[] = {GRF_BATCH_ROW(GRF_ROW_LDS) 0};
constexpr int max_of(const int* a, int n) {
  int m = 0;
  for (int i = 0; i < n; ++i) m = a[i] > m ? a[i] : m;
  return m;
}
constexpr int COL_LDS = max_of(col_lds_list, sizeof(col_lds_list) / sizeof(int));
constexpr int ROW_LDS = max_of(row_lds_list, sizeof(row_lds_list) / sizeof(int));
static_assert(COL_LDS <= 52 * 1024, "three column workgroups per CU");
static_assert(ROW_LDS <= 80 * 1024, "two row workgroups per CU");

#define GRF_CHECK_THREADS(L_, A_, B_) static_assert(BColPass<L_, A_>::THREADS <= BATCH_COL_THREADS, "too many threads");
GRF_BATCH_COL(GRF_CHECK_THREADS)
#undef GRF_CHECK_THREADS
#define GRF_CHECK_THREADS(M_, A_, B_) static_assert(BRowPass<M_, A_>::THREADS <= BATCH_ROW_THREADS, "too many threads");
GRF_BATCH_ROW(GRF_CHECK_THREADS)
#undef GRF_CHECK_THREADS

__device__ __forceinline__ Args batch_args(const BatchField& f, const BatchField* F, int field, float* out,
                                           const float2* tw) {
  Args a;
  a.data = (void*)(out + f.out_off);
  a.src = nullptr;
  a.aux = nullptr;
  a.partial = nullptr;
  a.recs = &F[field].rec;
  a.tw = tw + f.tw1;
  a.tw2 = tw + f.twd;
  a.htab = nullptr;            // per-field parameters: h is computed on the fly
  a.seed = f.seed;
  a.field_stride = (long long)f.n1 * f.M;
  a.stride_ax = f.M;
  a.stride_fixed = f.M;
  a.rows = f.n1;
  a.il2[0] = f.il2[0];
  a.il2[1] = f.il2[1];
  a.il2[2] = f.il2[2];
  a.scale = 1.0;
  a.rec_stride = 0;
  a.batch = 1;
  a.n1 = f.n1;
  a.no = 1;
  a.nd = f.nd;
  a.M = f.M;
  a.ntile = f.ntile;
  a.nfixed = 1;
  a.rows_per_field = f.n1;
  a.tag = 1;
  a.order = 0;
  a.tq = nullptr;
  a.sine = 0;
  a.bcmask = 0;
  a.seq = 0;
  a.plane = nullptr;
  a.src2 = nullptr;
  return a;
}

// One body per (length, tile shape), compiled as a separate function so that
// each gets its own register allocation (inlined into one switch, the
// allocator handles all bodies together and spills).
// TAG separates the bodies of the two kernels, so that each is compiled under
// its own kernel's register limit.
template <int L, int CP, int TAG = 0, bool ALT = false>
__device__ __attribute__((noinline)) void bcol_body(const BatchField* F, int field, int sub, float* out,
                                                    const float2* tw, char* smem) {
  const Args a = batch_args(F[field], F, field, out, tw);
  BColPass<L, CP, ALT>::run(a, sub, smem);
}
template <int M, int RB, int TAG = 0, bool ALT = false>
__device__ __attribute__((noinline)) void brow_body(const BatchField* F, int field, int sub, float* out,
                                                    const float2* tw, char* smem) {
  const Args a = batch_args(F[field], F, field, out, tw);
  BRowPass<M, RB, ALT>::run(a, sub, smem);
}

// Next work item of the workgroup (uniform); -1 when the queue is drained.
__device__ __forceinline__ int next_item(int* counter, int n, int* s_item) {
  if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
  __syncthreads();
  const int i = *s_item;
  __syncthreads();
  return i < n ? i : -1;
}

// Column items come in XCD_QUEUES queues (queue q = items[qoff[q] .. qoff[q+1]),
// counter counters[q]): a workgroup starts on the queue of its XCD (workgroup
// i runs on XCD i mod 8 under round-robin dispatch), so that the adjacent
// tiles of a field, which share cache lines, meet in one L2; when its queue is
// drained it helps with the others.
__global__ void __launch_bounds__(BATCH_COL_THREADS)
k_batch_col(const BatchField* __restrict__ F, const BatchItem* __restrict__ items, const int* __restrict__ qoff,
            const float2* tw, float* out, int* counters) {
  __shared__ __align__(16) char smem[COL_LDS];
  __shared__ int s_item;
  const int x0 = (int)(blockIdx.x % XCD_QUEUES);
  for (int j = 0; j < XCD_QUEUES; ++j) {
    const int q = (x0 + j) % XCD_QUEUES;
    const int base = qoff[q], n = qoff[q + 1] - base;
    int* counter = counters + q;
    for (int i = next_item(counter, n, &s_item); i >= 0; i = next_item(counter, n, &s_item)) {
      const BatchItem w = items[base + i];
      const BatchField& f = F[w.field];
      const int key = f.n1 * 4 + f.cvar;
      switch (key) {
#define GRF_CASE(L_, A_, B_)                                                  \
  case L_ * 4 + 0: bcol_body<L_, A_>(F, w.field, w.sub, out, tw, smem); break; \
  case L_ * 4 + 1: bcol_body<L_, B_>(F, w.field, w.sub, out, tw, smem); break;
        GRF_BATCH_COL(GRF_CASE)
#undef GRF_CASE
        default: break;
      }
      __syncthreads();  // the next item reuses the LDS
    }
  }
}

__global__ void __launch_bounds__(BATCH_ROW_THREADS)
k_batch_row(const BatchField* __restrict__ F, const BatchItem* __restrict__ items, int n, const float2* tw,
            float* out, int* counter) {
  __shared__ __align__(16) char smem[ROW_LDS];
  __shared__ int s_item;
  for (int i = next_item(counter, n, &s_item); i >= 0; i = next_item(counter, n, &s_item)) {
    const BatchItem w = items[i];
    const BatchField& f = F[w.field];
    const int key = f.M * 4 + f.rvar;
    switch (key) {
#define GRF_CASE(M_, A_, B_)                                                  \
  case M_ * 4 + 0: brow_body<M_, A_>(F, w.field, w.sub, out, tw, smem); break; \
  case M_ * 4 + 1: brow_body<M_, B_>(F, w.field, w.sub, out, tw, smem); break;
      GRF_BATCH_ROW(GRF_CASE)
#undef GRF_CASE
      default: break;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One persistent launch for both passes.  (length, column pairs variant 0,
// variant 1) of the column bodies at up to 512 threads; the row bodies are
// those of k_batch_row.
#define GRF_BATCH_ONE_COL(X) X(64, 64, 32) X(96, 42, 21) X(128, 32, 16) X(180, 14, 7) X(256, 16, 8) \
  X(360, 5, 2) X(500, 8, 4) X(512, 8, 4) X(1000, 4, 2) X(1024, 4, 2)

constexpr int max4(int a, int b, int c, int d) {
  const int x = a > b ? a : b, y = c > d ? c : d;
  return x > y ? x : y;
}
#define GRF_ONE_LDS(L_, A_, B_)                                                                          \
  max4(BColPass<L_, A_>::LDS_BYTES, BColPass<L_, B_>::LDS_BYTES,                                        \
       BColPass<L_, BatchAltCol<L_>::CPA, true>::LDS_BYTES, BColPass<L_, BatchAltCol<L_>::CPB, true>::LDS_BYTES),
constexpr int one_lds_list[] = {GRF_BATCH_ONE_COL(GRF_ONE_LDS) 0};
#undef GRF_ONE_LDS
#define GRF_ALT_ROW_LDS(M_, A_, B_)                                                                      \
  max4(BRowPass<M_, BatchAltRow<M_>::RBA, true>::LDS_BYTES, BRowPass<M_, BatchAltRow<M_>::RBB, true>::LDS_BYTES, 0, 0),
constexpr int alt_row_lds_list[] = {GRF_BATCH_ROW(GRF_ALT_ROW_LDS) 0};
#undef GRF_ALT_ROW_LDS
constexpr int ONE_COL_LDS = max_of(one_lds_list, sizeof(one_lds_list) / sizeof(int));
constexpr int ONE_ROW_LDS = max_of(alt_row_lds_list, sizeof(alt_row_lds_list) / sizeof(int)) > ROW_LDS
                                ? max_of(alt_row_lds_list, sizeof(alt_row_lds_list) / sizeof(int))
                                : ROW_LDS;
constexpr int ONE_LDS = ONE_COL_LDS > ONE_ROW_LDS ? ONE_COL_LDS : ONE_ROW_LDS;
static_assert(ONE_LDS <= 80 * 1024, "two one-launch workgroups per CU");
#define GRF_CHECK_THREADS(L_, A_, B_)                                                                   \
  static_assert(BColPass<L_, A_>::THREADS <= BATCH_ONE_THREADS, "too many threads");                    \
  static_assert(BColPass<L_, BatchAltCol<L_>::CPA, true>::THREADS <= BATCH_ONE_THREADS, "too many threads");
GRF_BATCH_ONE_COL(GRF_CHECK_THREADS)
#undef GRF_CHECK_THREADS
#define GRF_CHECK_THREADS(M_, A_, B_) \
  static_assert(BRowPass<M_, BatchAltRow<M_>::RBA, true>::THREADS <= BATCH_ONE_THREADS, "too many threads");
GRF_BATCH_ROW(GRF_CHECK_THREADS)
#undef GRF_CHECK_THREADS

// The XCD this workgroup runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (XCD_QUEUES - 1));
}

// A workgroup takes the items of its own XCD's queue only, so that the
// column items that write a field's spectrum and the row items that read it
// run under one L2: a column item's stores are complete at the L2 once each
// thread has waited for its memory counter, before the readiness count is
// raised; a row item's first loads of that spectrum follow the wait (no CU
// holds those lines in its L1 before, since nothing reads them earlier in the
// launch).  Queue order (host): column items of a group of fields before the
// row items of that group, so every column item a row item waits for has
// been taken by a running workgroup.
__global__ void __launch_bounds__(BATCH_ONE_THREADS, 4)
k_batch_one(const BatchField* __restrict__ F, const BatchItem* __restrict__ items, const int* __restrict__ qoff,
            const float2* tw, float* out, int* counters, int* done, int* err) {
  __shared__ __align__(16) char smem[ONE_LDS];
  __shared__ int s_item, s_skip;
  const int q = xcc_id();
  const int base = qoff[q], n = qoff[q + 1] - base;
  int* counter = counters + q;
  for (int i = next_item(counter, n, &s_item); i >= 0; i = next_item(counter, n, &s_item)) {
    const BatchItem w = items[base + i];
    const BatchField& f = F[w.field];
    if (w.sub >= 0) {
      switch (f.n1 * 4 + f.cvar) {
#define GRF_CASE(L_, A_, B_)                                                                                 \
  case L_ * 4 + 0: bcol_body<L_, A_, 1>(F, w.field, w.sub, out, tw, smem); break;                              \
  case L_ * 4 + 1: bcol_body<L_, B_, 1>(F, w.field, w.sub, out, tw, smem); break;                              \
  case L_ * 4 + 2: bcol_body<L_, BatchAltCol<L_>::CPA, 1, true>(F, w.field, w.sub, out, tw, smem); break;       \
  case L_ * 4 + 3: bcol_body<L_, BatchAltCol<L_>::CPB, 1, true>(F, w.field, w.sub, out, tw, smem); break;
        GRF_BATCH_ONE_COL(GRF_CASE)
#undef GRF_CASE
        default: break;
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this thread's stores have reached the L2
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_fetch_add(done + w.field, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (threadIdx.x == 0) {
        int skip = 0;
        for (int it = 0; __hip_atomic_load(done + w.field, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < f.ntile;
             ++it) {
          if (it >= BATCH_ONE_SPIN_LIMIT) {
            atomicOr(err, 1);
            skip = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        s_skip = skip;
      }
      __syncthreads();
      if (!s_skip) {
        switch (f.M * 4 + f.rvar) {
#define GRF_CASE(M_, A_, B_)                                                                                   \
  case M_ * 4 + 0: brow_body<M_, A_, 1>(F, w.field, -w.sub - 1, out, tw, smem); break;                           \
  case M_ * 4 + 1: brow_body<M_, B_, 1>(F, w.field, -w.sub - 1, out, tw, smem); break;                           \
  case M_ * 4 + 2: brow_body<M_, BatchAltRow<M_>::RBA, 1, true>(F, w.field, -w.sub - 1, out, tw, smem); break;    \
  case M_ * 4 + 3: brow_body<M_, BatchAltRow<M_>::RBB, 1, true>(F, w.field, -w.sub - 1, out, tw, smem); break;
          GRF_BATCH_ROW(GRF_CASE)
#undef GRF_CASE
          default: break;
        }
      }
    }
    __syncthreads();   // the next item reuses the LDS
  }
}

// mask |= 1 << XCD of each workgroup (the mask is cleared by a launch before).
__global__ void k_xcc_seen(int* mask) {
  if (threadIdx.x == 0) atomicOr(mask, 1 << xcc_id());
}

__global__ void k_reset_counters(int* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

int batch_col_cp(int L, int var) {
  switch (L) {
#define GRF_X(L_, A_, B_) \
  case L_: return var == 0 ? A_ : B_;
    GRF_BATCH_COL(GRF_X)
#undef GRF_X
    default: return 0;
  }
}
int batch_row_rb(int M, int var) {
  switch (M) {
#define GRF_X(M_, A_, B_) \
  case M_: return var == 0 ? A_ : var == 1 ? B_ : var == 2 ? BatchAltRow<M_>::RBA : BatchAltRow<M_>::RBB;
    GRF_BATCH_ROW(GRF_X)
#undef GRF_X
    default: return 0;
  }
}
int batch_one_cp(int L, int var) {
  switch (L) {
#define GRF_X(L_, A_, B_) \
  case L_: return var == 0 ? A_ : var == 1 ? B_ : var == 2 ? BatchAltCol<L_>::CPA : BatchAltCol<L_>::CPB;
    GRF_BATCH_ONE_COL(GRF_X)
#undef GRF_X
    default: return 0;
  }
}
bool batch_col_supported(int L) { return batch_col_cp(L, 0) > 0; }
bool batch_row_supported(int M) { return batch_row_rb(M, 0) > 0; }

hipError_t launch_batch_col(const BatchField* fields, const BatchItem* items, const int* qoff, const void* twpool,
                            float* out, int* counters, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_col, dim3(nwg), dim3(BATCH_COL_THREADS), 0, s, fields, items, qoff,
                     (const float2*)twpool, out, counters);
  return hipGetLastError();
}
hipError_t launch_batch_row(const BatchField* fields, const BatchItem* items, int nitems, const void* twpool,
                            float* out, int* counter, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_row, dim3(nwg), dim3(BATCH_ROW_THREADS), 0, s, fields, items, nitems,
                     (const float2*)twpool, out, counter);
  return hipGetLastError();
}
hipError_t launch_batch_one(const BatchField* fields, const BatchItem* items, const int* qoff, const void* twpool,
                            float* out, int* counters, int* done, int* err, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_one, dim3(nwg), dim3(BATCH_ONE_THREADS), 0, s, fields, items, qoff,
                     (const float2*)twpool, out, counters, done, err);
  return hipGetLastError();
}
const void* k_batch_one_ptr() { return reinterpret_cast<const void*>(&k_batch_one); }
hipError_t launch_xcc_seen(int* mask, int nwg, hipStream_t s) {
  hipError_t e = launch_reset_counters(mask, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xcc_seen, dim3(nwg), dim3(64), 0, s, mask);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}
const void* k_batch_col_ptr() { return reinterpret_cast<const void*>(&k_batch_col); }
const void* k_batch_row_ptr() { return reinterpret_cast<const void*>(&k_batch_row); }

hipError_t launch_reset_counters(int* counters, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(1024), 0, s, counters, n);
  return hipGetLastError();
}

}  // namespace grf
