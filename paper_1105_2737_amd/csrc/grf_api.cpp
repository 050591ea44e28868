// Host side of the C ABI declared in include/grf.h: argument validation, plan
// tables and the sequence of passes for each entry point.
//
// Pass sequences (packed half-spectrum layout, in place in the output buffer):
//   one-FFT algorithm (Section 3), d = 2:
//       column noise generation + inverse transform along axis 1
//       -> last-axis complex-to-real
//   one-FFT algorithm, d = 3: as above with an inverse transform along axis 2
//       between the two
//   two-FFT algorithm (Section 3), d = 2:
//       last-axis white noise + real-to-complex
//       -> axis 1 forward, multiply by h / sqrt(P), axis 1 inverse
//       -> last-axis complex-to-real
//   adjoint of the one-FFT algorithm, d = 2:
//       last-axis real-to-complex of dL/dphi -> axis 1 forward + reduction
//       -> per-field sum of the partials
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "grf.h"
#include "grf_dispatch.hpp"
#include "grf_host.hpp"
#include "grf_kernels.hpp"
#include "grf_tune_cache.hpp"

using grf::Args;
using grf::FieldRec;

// The kernel of one pass of a plan, as chosen by the tuner or the cache: the
// compile-time kernel of its length, or the runtime-radix kernel with a radix
// order and a number of values per thread.
struct TuneChoice {
  bool generic = false;
  int vpt = 8;
  int ns = 0;
  int rad[16] = {};
};

struct grf_plan_s {
  grf_plan_desc desc;
  int d;
  int n1, no, nd, M;        // N_1, middle (N_2 if d = 3 else 1), last, last/2
  long long P;              // points per field
  double vol;
  double il2[3];
  int dtype;
  size_t esz;               // bytes per real element
  void* tw_col1 = nullptr;  // W_{N_1}
  void* tw_col2 = nullptr;  // W_{N_2} (d = 3)
  void* tw_row = nullptr;   // W_{N_d}
  FieldRec* rec_dev = nullptr;
  void* htab = nullptr;     // filter table h[row][m] (row stride M + 2) of the default parameters
  bool table_only = false;  // PAPER / TABULATED: h exists only as the table
  // reflecting boundaries (cosine / sine transforms); htab then holds a_n / z_n
  // over the slot grid [rows][N_d]
  bool reflect = false;
  int sinemask = 0;         // sine axes: bit 0 axis 1, bit 1 middle axis, bit 2 last axis
  void* tq_col1 = nullptr;  // (1/2) e^{i pi k / (2N)} of each axis
  void* tq_col2 = nullptr;
  void* tq_row = nullptr;   // last axis: q_k, k <= M, then the forward pass's alpha_k, beta_k (make_row_rtable)
  int device = 0;
  bool listed = true;       // every axis has compile-time kernels (else the runtime-radix passes)
  std::map<long long, TuneChoice> tune;   // per (pass, transform length): the tuner's or the cache's choice
  mutable bool tuning = false;            // the tuner's view: the unsplit passes (UnsplitScope)
};

namespace grf {
namespace host {

thread_local std::string g_err;

grf_status fail(grf_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

grf_status hip_fail(hipError_t e, const char* what) {
  return fail(GRF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool smooth235(long long n) {
  if (n <= 0) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

void table_values(int L, std::vector<double>& w) {
  w.resize(2 * (size_t)L);
  for (int i = 0; i < L; ++i) {
    // reduce i/L to an angle in [-pi, pi] before cos/sin for accuracy
    long long ii = i;
    if (2 * ii > L) ii -= L;
    const double ang = 2.0 * M_PI * (double)ii / (double)L;
    w[2 * i] = std::cos(ang);
    w[2 * i + 1] = std::sin(ang);
  }
}

// W_L[i] = exp(2 pi i i / L) in float64, stored in the working precision.
grf_status make_table(int L, int dtype, void** out) {
  std::vector<double> w;
  table_values(L, w);
  const size_t bytes = (size_t)L * 2 * (dtype == GRF_F32 ? 4 : 8);
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return fail(GRF_ENOMEM, "hipMalloc of twiddle table failed");
  if (dtype == GRF_F32) {
    std::vector<float> f(w.begin(), w.end());
    e = hipMemcpy(*out, f.data(), bytes, hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(*out, w.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "twiddle upload");
  return GRF_OK;
}

// Pre-twiddles (1/2) e^{i pi k / (2N)}, k = 0 .. count - 1, of the cosine
// transform of length N, in float64, stored in the working precision.
grf_status make_qtable(int N, int count, int dtype, void** out) {
  std::vector<double> w(2 * (size_t)count);
  for (int k = 0; k < count; ++k) {
    const double ang = M_PI * (double)k / (2.0 * (double)N);
    w[2 * k] = 0.5 * std::cos(ang);
    w[2 * k + 1] = 0.5 * std::sin(ang);
  }
  const size_t bytes = (size_t)count * 2 * (dtype == GRF_F32 ? 4 : 8);
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return fail(GRF_ENOMEM, "hipMalloc of twiddle table failed");
  if (dtype == GRF_F32) {
    std::vector<float> f(w.begin(), w.end());
    e = hipMemcpy(*out, f.data(), bytes, hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(*out, w.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "twiddle upload");
  return GRF_OK;
}

// The last axis's table: q_k = (1/2) e^{i pi k / (2N)}, k = 0..M (N = 2M), then
// the forward pass's combined factors alpha_k = q_k (1 + i W_N^k) and
// beta_k = conj(q_{M-k}) (1 - i W_N^k), k = 0..M-1 (see R2RRow::prep), all in
// float64, rounded once.
grf_status make_row_rtable(int N, int dtype, void** out) {
  const int M = N / 2;
  std::vector<double> w(2 * (size_t)(3 * M + 1));
  auto q = [&](int k, double& re, double& im) {
    const double ang = M_PI * (double)k / (2.0 * (double)N);
    re = 0.5 * std::cos(ang);
    im = 0.5 * std::sin(ang);
  };
  for (int k = 0; k <= M; ++k) q(k, w[2 * k], w[2 * k + 1]);
  for (int k = 0; k < M; ++k) {
    long long kk = k;
    if (2 * kk > N) kk -= N;
    const double ang = 2.0 * M_PI * (double)kk / (double)N;
    const double wr = std::cos(ang), wi = std::sin(ang);
    double qr, qi, mr, mi;
    q(k, qr, qi);
    q(M - k, mr, mi);
    // 1 + i w = (1 - wi) + i wr;  1 - i w = (1 + wi) - i wr
    const double ar = 1.0 - wi, ai = wr, br = 1.0 + wi, bi = -wr;
    double* al = &w[2 * (size_t)(M + 1 + k)];
    double* be = &w[2 * (size_t)(2 * M + 1 + k)];
    al[0] = qr * ar - qi * ai;
    al[1] = qr * ai + qi * ar;
    be[0] = mr * br + mi * bi;   // conj(q_{M-k}) = mr - i mi
    be[1] = mr * bi - mi * br;
  }
  const size_t bytes = w.size() * (dtype == GRF_F32 ? 4 : 8);
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return fail(GRF_ENOMEM, "hipMalloc of twiddle table failed");
  if (dtype == GRF_F32) {
    std::vector<float> f(w.begin(), w.end());
    e = hipMemcpy(*out, f.data(), bytes, hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(*out, w.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "twiddle upload");
  return GRF_OK;
}

}  // namespace host
}  // namespace grf

namespace {

using grf::host::fail;
using grf::host::g_err;
using grf::host::hip_fail;
using grf::host::make_qtable;
using grf::host::make_row_rtable;
using grf::host::make_table;
using grf::host::smooth235;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

long long chunk_fields(const grf_plan_s* p, long long batch);

// Workspace layout: [records][partials][spectrum of one chunk of fields]
// [d = 3 adjoint: plane values Z of one chunk | two-FFT adjoint: the white
// noise's spectrum of one chunk]
struct WsLayout {
  size_t recs, partial, spec, plane, spec2, total;
};

// Adjoint: workgroups of the reduction pass per field (each leaves three
// partial sums) and, for d = 1, 2, its column tiles.
struct AdjTiles {
  int ntile;     // tiles per fixed index (d = 2, 3) or per field (d = 1)
  int nper;      // partial sums per field / 3
};
AdjTiles adj_tiles(const grf_plan_s* p) {
  if (p->reflect) {
    if (p->d == 1) return AdjTiles{1, 1};
    const grf::Geom g = grf::pass_geom(grf::PASS_R2R_COL_FWD_RED, p->dtype, p->n1);
    const int nt = (p->M + 2 * g.per_wg - 1) / (2 * g.per_wg);
    return AdjTiles{nt, nt * p->no};
  }
  if (p->desc.alg == GRF_ALG_TWO_FFT && (p->d != 2 || !p->listed)) {
    const long long slots = (long long)p->n1 * p->no * p->M;
    const int nt = (int)((slots + 255) / 256);
    return AdjTiles{nt, nt};
  }
  if (p->d == 1) {
    const int nt = ((p->M + 1) / 2 + 255) / 256;
    return AdjTiles{nt, nt};
  }
  if (!p->listed) {   // k_grad_gen: one slot pair per thread
    const long long slots = (long long)p->n1 * p->no * ((p->M + 1) / 2);
    const int nt = (int)((slots + 255) / 256);
    return AdjTiles{nt, nt};
  }
  const grf::Geom g = grf::pass_geom(p->d == 3 ? grf::PASS_COL_GRAD3 : grf::PASS_COL_GRAD, p->dtype, p->n1);
  if (g.per_wg <= 0) return AdjTiles{1, 1};   // no adjoint kernel for this length (grf_backward refuses it)
  const int nt = (p->M + 2 * g.per_wg - 1) / (2 * g.per_wg);
  return AdjTiles{nt, nt * p->no};
}

WsLayout ws_layout(const grf_plan_s* p, long long batch, int op) {
  WsLayout w{};
  w.recs = 0;
  size_t off = align256((size_t)batch * sizeof(FieldRec));
  w.partial = off;
  if (op == GRF_OP_BACKWARD) {
    off += align256((size_t)batch * adj_tiles(p).nper * 3 * sizeof(double));
    w.spec = off;
    const long long C = chunk_fields(p, batch);
    off += align256((size_t)C * p->P * p->esz);
    w.plane = off;
    if (p->d == 3) off += align256((size_t)C * p->n1 * p->no * 2 * p->esz);
    w.spec2 = off;
    if (p->desc.alg == GRF_ALG_TWO_FFT) off += align256((size_t)C * p->P * p->esz);
  } else {
    w.spec = off;
    w.plane = off;
    w.spec2 = off;
  }
  w.total = off;
  return w;
}

grf_status check_stream_device(const grf_plan_s* p) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device) return fail(GRF_EINVAL, "plan was created on another device");
  return GRF_OK;
}

// Per-field constants: from device theta (prep kernel) or the plan default.
grf_status field_records(const grf_plan_s* p, const double* theta, long long batch, void* workspace,
                         size_t ws_bytes, hipStream_t s, const FieldRec** recs, int* stride) {
  if (theta == nullptr) {
    *recs = p->rec_dev;
    *stride = 0;
    return GRF_OK;
  }
  if (p->table_only) return fail(GRF_EUNSUPPORTED, "per-field parameters need a parametric covariance family");
  if (workspace == nullptr || ws_bytes < (size_t)batch * sizeof(FieldRec))
    return fail(GRF_EINVAL, "workspace too small for per-field parameters");
  FieldRec* out = (FieldRec*)workspace;
  hipError_t e = grf::launch_prep_recs(theta, (int)batch, p->desc.cov_kind, p->d, p->vol, out, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "per-field constants");
  *recs = out;
  *stride = 1;
  return GRF_OK;
}

Args base_args(const grf_plan_s* p, long long batch) {
  Args a;
  std::memset(&a, 0, sizeof(a));
  a.field_stride = p->P / 2;
  a.batch = (int)batch;
  a.n1 = p->n1;
  a.no = p->no;
  a.nd = p->nd;
  a.M = p->M;
  a.il2[0] = p->il2[0];
  a.il2[1] = p->il2[1];
  a.il2[2] = p->il2[2];
  a.scale = 1.0;
  a.nfixed = 1;
  a.rows_per_field = (int)(p->P / p->nd);
  return a;
}

// Column passes take their tiles in XCD-grouped order (GRF_XCD=0 turns it off).
int xcd_order() {
  const char* e = std::getenv("GRF_XCD");
  return (e && e[0] == '0') ? 0 : 1;
}

bool is_adjoint_col_pass(int pass) {
  return pass == grf::PASS_COL_GRAD || pass == grf::PASS_COL_GRAD3 || pass == grf::PASS_COL_GRAD1 ||
         pass == grf::PASS_COL_GRAD_SEQ || pass == grf::PASS_COL_GRAD3_SEQ;
}

// Fields per workgroup of the adjoint's column pass (each workgroup runs one
// column tile of that many consecutive fields, so that it reads its rows of
// the filter table once from HBM per run).  Measured on MI355X (adjoint of
// 1024^2 x 64 / 512^2 x 256 / 256^3 x 16, fields per workgroup 1, 2, 4, 8):
// 0.273 / 0.246 / 0.255 / 0.273 ms, 0.242 / 0.246 / 0.265 / 0.313 ms and
// 1.69 / 1.73 / 1.82 / 1.83 ms: two pay off only where the table (2.1 MB at
// 1024^2) no longer stays in an XCD's 4 MB L2 while the fields stream
// through it; a 3D plan has no table.  GRF_ADJ_FPW overrides.
int adjoint_fields_per_wg(const Args& a, size_t esz) {
  if (const char* e = std::getenv("GRF_ADJ_FPW")) {
    const int v = std::atoi(e);
    if (v >= 1) return v;
  }
  const long long table = (long long)a.n1 * a.no * (a.M + 2) * (long long)esz;
  return (a.htab != nullptr && table > (1ll << 20)) ? 2 : 1;
}

// A pass whose transform length has no compile-time kernel runs on the
// runtime-radix kernels (column passes, the last-axis passes, the d = 1
// one-launch sampler of the one-FFT algorithm).
bool fixed_length(int pass, int L) {
  if (pass == grf::PASS_SPEC_FILTER || pass == grf::PASS_SPEC_FILTER0) return true;
  if (grf::is_r2r_pass(pass)) return true;   // the reflecting passes exist for the listed lengths only
  if (grf::is_row_pass(pass)) return grf::row_length_supported(L);
  return grf::col_length_supported(L);
}

long long tune_key(int pass, int L) { return (long long)pass * 1000000 + L; }

const TuneChoice* tune_choice(const grf_plan_s* p, int pass, int L) {
  const auto it = p->tune.find(tune_key(pass, L));
  return it == p->tune.end() ? nullptr : &it->second;
}

grf_status run_generic(const grf_plan_s* p, int pass, int L, Args a, long long batch, hipStream_t s,
                       const TuneChoice* tc) {
  // untuned: 8 values per thread in float32, 4 in float64 (measured on
  // MI355X with the generator's radix order over 12 workloads in d = 1, 2, 3:
  // float32 sampling 1.03-1.37x faster with 8, float64 mostly 3-11% faster
  // with 4), the other where a transform does not fit the first (more than
  // 1024 threads, or too much LDS)
  int vpt = tc ? tc->vpt : (p->dtype == GRF_F32 ? 8 : 4);
  grf::GGeom g = grf::generic_geom(pass, p->dtype, L, vpt);
  if (g.threads <= 0 && !tc) {
    vpt = 12 - vpt;
    g = grf::generic_geom(pass, p->dtype, L, vpt);
  }
  if (g.threads <= 0) return fail(GRF_EUNSUPPORTED, "no kernel for this transform length and pass");
  a.gl = L;
  a.gcp = g.per_wg;
  a.gnt = g.nt;
  a.grs = g.rs;
  a.gvpt = vpt;
  if (tc) {
    a.gs = tc->ns;
    for (int i = 0; i < tc->ns; ++i) a.grad[i] = tc->rad[i];
  } else {
    a.gs = grf::radix_plan(L, a.grad);
  }
  if (a.gs < 0) return fail(GRF_EINVAL, "transform length is not 2/3/5-smooth");
  long long nblocks;
  if (grf::is_row_pass(pass)) {
    nblocks = (a.rows + g.per_wg - 1) / g.per_wg;
  } else {
    a.ntile = (a.M + 2 * g.per_wg - 1) / (2 * g.per_wg);
    nblocks = (long long)a.ntile * a.nfixed * batch;
    a.order = xcd_order();
  }
  if (nblocks <= 0) return GRF_OK;
  if (nblocks > 0x7fffffffLL) return fail(GRF_EINVAL, "batch too large for one launch");
  hipError_t e = grf::launch_generic(pass, p->dtype, a, nblocks, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return GRF_OK;
}

grf_status run_pass(const grf_plan_s* p, int pass, int L, Args a, long long nfixed_blocks_per_field,
                    long long batch, hipStream_t s) {
  (void)nfixed_blocks_per_field;
  if (pass == grf::PASS_ROW_XC2R) {
    const grf::XGeom g = grf::xc2r_geom(p->dtype, p->n1, p->M);
    if (g.threads <= 0) return fail(GRF_EUNSUPPORTED, "no kernel for this transform length and pass");
    const long long nblocks = a.rows / g.rows;
    if (nblocks <= 0) return GRF_OK;
    hipError_t e = grf::launch_xc2r(p->dtype, p->n1, p->M, a, nblocks, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return GRF_OK;
  }
  const TuneChoice* tc = tune_choice(p, pass, L);
  if (tc ? tc->generic : !fixed_length(pass, L)) return run_generic(p, pass, L, a, batch, s, tc);
  const grf::Geom g = grf::pass_geom(pass, p->dtype, L);
  if (g.threads <= 0) return fail(GRF_EUNSUPPORTED, "no kernel for this length");
  long long nblocks;
  if (pass == grf::PASS_SPEC_FILTER) {
    nblocks = (a.rows * a.M + g.threads - 1) / g.threads;
  } else if (pass == grf::PASS_SPEC_FILTER0) {
    nblocks = (a.rows + g.threads - 1) / g.threads;
  } else if (grf::is_row_pass(pass)) {
    nblocks = (a.rows + g.per_wg - 1) / g.per_wg;
  } else {
    a.ntile = (a.M + 2 * g.per_wg - 1) / (2 * g.per_wg);
    a.fpw = is_adjoint_col_pass(pass) && pass != grf::PASS_COL_GRAD_SEQ && pass != grf::PASS_COL_GRAD3_SEQ
                ? adjoint_fields_per_wg(a, p->esz)
                : 1;
    nblocks = (long long)a.ntile * a.nfixed * ((batch + a.fpw - 1) / a.fpw);
    a.order = xcd_order();
  }
  if (nblocks <= 0) return GRF_OK;
  if (nblocks > 0x7fffffffLL) return fail(GRF_EINVAL, "batch too large for one launch");
  hipError_t e = grf::launch_pass(pass, p->dtype, L, a, nblocks, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return GRF_OK;
}

// One launch of the sampler: pass kind, transform length, arguments and the
// fields first .. first + count - 1 of the call that it covers.
struct PassLaunch {
  int pass;
  int L;
  Args a;
  long long first = 0;
  long long count = 0;
};

// Fields per chunk: the sampler runs all its passes on one chunk of fields
// before the next, and a chunk is sized to the 256 MB last-level cache
// (Infinity Cache) of the device, so that each pass reads what the previous
// one wrote from that cache rather than from HBM.  GRF_CHUNK_BYTES overrides.
long long chunk_fields(const grf_plan_s* p, long long batch) {
  long long bytes = 256ll << 20;
  if (const char* e = std::getenv("GRF_CHUNK_BYTES")) {
    const long long v = std::atoll(e);
    if (v > 0) bytes = v;
  }
  long long c = bytes / (p->P * (long long)p->esz);
  if (c < 1) c = 1;
  if (c > batch) c = batch;
  return c;
}

grf_status run_launch(const grf_plan_s* p, const PassLaunch& pl, hipStream_t s) {
  return run_pass(p, pl.pass, pl.L, pl.a, 0, pl.count, s);
}

// The tuner chooses per pass between the compile-time kernel and
// runtime-radix ones on the unsplit sequence (column generation + plain
// complex-to-real); the split route runs where both keep the compile-time
// kernels.  While a scope lives, the plan's sequences are the unsplit ones.
struct UnsplitScope {
  const grf_plan_s* p;
  const bool prev;
  explicit UnsplitScope(const grf_plan_s* q) : p(q), prev(q->tuning) { p->tuning = true; }
  ~UnsplitScope() { p->tuning = prev; }
};

// d = 2 one-FFT (either draw order) on a pair of lengths that has the split
// kernels (the column transform's last stage in the last-axis pass), with
// both passes on their compile-time kernels.  GRF_SPLIT=0 keeps the unsplit
// passes.
bool split_route(const grf_plan_s* p) {
  if (p->d != 2 || p->reflect || p->desc.alg != GRF_ALG_ONE_FFT || !p->listed || p->tuning) return false;
  if (grf::xc2r_geom(p->dtype, p->n1, p->M).threads <= 0) return false;
  if (const char* e = std::getenv("GRF_SPLIT"))
    if (e[0] == '0') return false;
  const bool seq = p->desc.draw_order == GRF_DRAW_RECURSIVE;
  const TuneChoice* c = tune_choice(p, seq ? grf::PASS_COL_SEQ_INV : grf::PASS_COL_GEN_INV, p->n1);
  const TuneChoice* r = tune_choice(p, grf::PASS_ROW_C2R, p->M);
  return !(c && c->generic) && !(r && r->generic);
}

// The passes of the sampler over fields c0 .. c0 + nb - 1 (zsrc == nullptr
// generates the noise); field c0 + j uses key seed + c0 + j, so a chunk gives
// the same bits as the same fields in a larger call.
void chunk_passes(const grf_plan_s* p, uint64_t seed, const void* zsrc, long long c0, long long nb,
                  const FieldRec* recs, int rstride, void* out, std::vector<PassLaunch>& v) {
  const size_t fbytes = (size_t)p->P * p->esz;
  Args a = base_args(p, nb);
  a.data = (char*)out + c0 * fbytes;
  a.src = zsrc ? (const char*)zsrc + c0 * fbytes : nullptr;
  a.recs = rstride ? recs + c0 : recs;
  a.rec_stride = rstride;
  a.seed = seed + (uint64_t)c0;
  a.htab = rstride == 0 ? p->htab : nullptr;
  auto push = [&](int pass, int L, const Args& x) {
    PassLaunch pl;
    pl.pass = pass;
    pl.L = L;
    pl.a = x;
    pl.first = c0;
    pl.count = nb;
    v.push_back(pl);
  };
  if (p->reflect) {
    // cosine / sine transforms: coefficients + axis 1, (middle axis,) last axis
    a.tag = 2;
    a.bcmask = p->sinemask;
    Args r = a;
    r.tw2 = p->tw_row;
    r.tq = p->tq_row;
    r.sine = (p->sinemask >> 2) & 1;
    if (p->d == 1) {
      r.rows = nb;
      push(grf::PASS_R2R_ROW_GEN, p->M, r);
      return;
    }
    Args c = a;
    c.tw = p->tw_col1;
    c.tq = p->tq_col1;
    c.sine = p->sinemask & 1;
    c.stride_ax = (long long)p->no * p->M;
    c.stride_fixed = p->M;
    c.nfixed = p->no;
    push(grf::PASS_R2R_COL_GEN, p->n1, c);
    if (p->d == 3) {
      Args m = c;
      m.src = nullptr;
      m.tw = p->tw_col2;
      m.tq = p->tq_col2;
      m.sine = (p->sinemask >> 1) & 1;
      m.stride_ax = p->M;
      m.stride_fixed = (long long)p->no * p->M;
      m.nfixed = p->n1;
      push(grf::PASS_R2R_COL_LOAD, p->no, m);
    }
    r.src = nullptr;
    r.rows = nb * (p->P / p->nd);
    push(grf::PASS_R2R_ROW_LOAD, p->M, r);
    return;
  }
  const bool seq = p->desc.draw_order == GRF_DRAW_RECURSIVE;
  if (p->d == 1) {
    // one launch of whole fields: noise, filter and complex-to-real transform
    // (the two-FFT algorithm: white noise and its forward transform first)
    const bool two = p->desc.alg == GRF_ALG_TWO_FFT;
    a.tag = two ? 0 : seq ? 3 : 1;
    a.seq = seq;
    if (two) a.scale = 1.0 / std::sqrt((double)p->P);   // the table, where there is one, carries it
    a.tw2 = p->tw_row;
    a.rows = nb;
    if (two && !grf::row_length_supported(p->M)) {
      // no one-launch kernel for this length: white noise + real-to-complex,
      // the filter on the spectrum, complex-to-real
      Args f = a;
      f.htab = p->table_only ? p->htab : nullptr;
      push(zsrc ? grf::PASS_ROW_R2C_LOAD : grf::PASS_ROW_R2C_GEN, p->M, a);
      push(grf::PASS_SPEC_FILTER, 0, f);
      Args c = a;
      c.src = nullptr;
      push(grf::PASS_ROW_C2R, p->M, c);
      return;
    }
    push(grf::PASS_ROW_GEN_C2R, p->M, a);
    return;
  }
  if (p->desc.alg == GRF_ALG_ONE_FFT) {
    a.tag = seq ? 3 : 1;
    a.seq = seq;
    a.tw = p->tw_col1;
    if (p->d == 2) {
      a.stride_ax = p->M;
      a.stride_fixed = p->M;
      a.nfixed = 1;
    } else {
      a.stride_ax = (long long)p->no * p->M;
      a.stride_fixed = p->M;
      a.nfixed = p->no;
    }
    if (split_route(p)) {
      // the column transform's last stage in the last-axis pass
      push(seq ? grf::PASS_COL_SEQ_PART : grf::PASS_COL_GEN_PART, p->n1, a);
      Args b = a;
      b.src = nullptr;
      b.tw = p->tw_col1;
      b.tw2 = p->tw_row;
      b.rows = nb * (long long)p->n1;
      push(grf::PASS_ROW_XC2R, p->M, b);
      return;
    }
    push(seq ? grf::PASS_COL_SEQ_INV : grf::PASS_COL_GEN_INV, p->n1, a);
    if (p->d == 3) {
      Args m = a;
      m.src = nullptr;
      m.tw = p->tw_col2;
      m.stride_ax = p->M;
      m.stride_fixed = (long long)p->no * p->M;
      m.nfixed = p->n1;
      push(grf::PASS_COL_LOAD_INV, p->no, m);
    }
  } else if (p->d != 2) {
    // two-FFT, d = 3 (d = 1 is one launch, above): last-axis R2C, then the
    // leading axes
    Args r = a;
    r.tag = 0;
    r.tw2 = p->tw_row;
    r.rows = nb * (p->P / p->nd);
    push(zsrc ? grf::PASS_ROW_R2C_LOAD : grf::PASS_ROW_R2C_GEN, p->M, r);
    Args m = a, c = a;
    m.src = c.src = nullptr;
    m.tw = p->tw_col2;
    m.stride_ax = p->M;
    m.stride_fixed = (long long)p->no * p->M;
    m.nfixed = p->n1;
    c.tw = p->tw_col1;
    c.stride_ax = (long long)p->no * p->M;
    c.stride_fixed = p->M;
    c.nfixed = p->no;
    Args f = a;
    f.src = nullptr;
    f.rows = nb * (p->P / p->nd);
    f.scale = 1.0 / std::sqrt((double)p->P);   // the table, where there is one, carries it
    f.htab = p->table_only ? p->htab : nullptr;
    // d = 3: the middle axis forward; axis 1 forward, filter, inverse for
    // every slot but the packed plane slot, in one column pass; that slot's
    // column (M = 1 restricts a column pass to it) forward, its filter with
    // the mirrored rows, inverse; the middle axis inverse
    push(grf::PASS_COL_LOAD_FWD, p->no, m);
    if (grf::col_length_supported(p->n1)) {
      Args cf = c;
      cf.scale = f.scale;
      cf.htab = f.htab;
      push(grf::PASS_COL_FILTER3, p->n1, cf);
      Args c0 = c;
      c0.M = 1;
      push(grf::PASS_COL_LOAD_FWD, p->n1, c0);
      push(grf::PASS_SPEC_FILTER0, 0, f);
      push(grf::PASS_COL_LOAD_INV, p->n1, c0);
    } else {
      // axis 1 on the runtime-radix kernels: forward, the filter on the whole
      // packed spectrum, inverse
      push(grf::PASS_COL_LOAD_FWD, p->n1, c);
      push(grf::PASS_SPEC_FILTER, 0, f);
      push(grf::PASS_COL_LOAD_INV, p->n1, c);
    }
    push(grf::PASS_COL_LOAD_INV, p->no, m);
  } else {
    Args r = a;
    r.tag = 0;
    r.tw2 = p->tw_row;
    r.rows = nb * (long long)p->n1;
    push(zsrc ? grf::PASS_ROW_R2C_LOAD : grf::PASS_ROW_R2C_GEN, p->M, r);
    Args c = a;
    c.src = nullptr;
    c.tw = p->tw_col1;
    c.stride_ax = p->M;
    c.stride_fixed = p->M;
    c.nfixed = 1;
    c.scale = 1.0 / std::sqrt((double)p->P);
    // this pass has VALU to spare: h on the fly beats a table load, except for the
    // families whose filter exists only as a table (built with the 1/sqrt(P) factor)
    c.htab = p->table_only ? p->htab : nullptr;
    if (grf::col_length_supported(p->n1)) {
      push(grf::PASS_COL_FILTER, p->n1, c);
    } else {
      // axis 1 on the runtime-radix kernels: forward, the filter on the packed
      // spectrum, inverse
      Args f = c;
      f.rows = nb * (long long)p->n1;
      push(grf::PASS_COL_LOAD_FWD, p->n1, c);
      push(grf::PASS_SPEC_FILTER, 0, f);
      push(grf::PASS_COL_LOAD_INV, p->n1, c);
    }
  }
  Args b = a;
  b.src = nullptr;
  b.tw2 = p->tw_row;
  b.rows = nb * (p->P / p->nd);
  push(grf::PASS_ROW_C2R, p->M, b);
}

// The launch sequence of the sampler (zsrc == nullptr generates the noise).
std::vector<PassLaunch> sample_passes(const grf_plan_s* p, uint64_t seed, const void* zsrc, long long batch,
                                      const FieldRec* recs, int rstride, void* out) {
  std::vector<PassLaunch> v;
  const long long C = chunk_fields(p, batch);
  const long long nch = (batch + C - 1) / C;
  for (long long k = 0; k < nch; ++k) chunk_passes(p, seed, zsrc, k * C, std::min(C, batch - k * C), recs, rstride, out, v);
  return v;
}

// Filter table of a family given by its density (PAPER, TABULATED), built on
// the host in float64: h[row][m] = scale sigma sqrt(S(p) / |D|) over the
// half-spectrum (rows = N_1 ... N_{d-1}, m = 0 .. N_d/2; row stride M + 2, the
// extra slot 0), then rounded once to the working precision.
grf_status build_density_table(grf_plan_s* p, const grf_plan_desc& d, double scale) {
  const int rows = p->n1 * p->no;
  const int M = p->M, HS = M + 2;
  std::vector<double> h((size_t)rows * HS, 0.0);
  auto kappa = [](int k, int n) { return 2 * k < n ? k : k - n; };
  const int last = p->d - 1;
  for (int row = 0; row < rows; ++row) {
    const int kk1 = row / p->no, o = row % p->no;
    double pc[3] = {0, 0, 0};
    int np = 0;
    if (p->d >= 2) pc[np++] = kappa(kk1, p->n1) / d.lengths[0];
    if (p->d == 3) pc[np++] = kappa(o, p->no) / d.lengths[1];
    for (int m = 0; m <= M; ++m) {
      const double pl = (m == M ? -M : m) / d.lengths[last];
      double S;
      if (d.cov_kind == GRF_COV_PAPER) {
        double q = std::pow(pl * pl, d.k);
        for (int i = 0; i < np; ++i) q += std::pow(pc[i] * pc[i], d.k);
        S = std::pow(std::pow(d.m, (double)d.k * d.l) + std::pow(q, d.l), -(double)d.n);
      } else {
        S = d.spectrum[(size_t)row * (M + 1) + m];
      }
      h[(size_t)row * HS + m] = scale * d.sigma * std::sqrt(S / p->vol);
    }
  }
  const size_t n = h.size();
  const size_t bytes = n * p->esz;
  hipError_t e = hipMalloc(&p->htab, bytes);
  if (e != hipSuccess) return fail(GRF_ENOMEM, "hipMalloc of the filter table failed");
  if (p->dtype == GRF_F32) {
    std::vector<float> f(h.begin(), h.end());
    e = hipMemcpy(p->htab, f.data(), bytes, hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(p->htab, h.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "filter table upload");
  return GRF_OK;
}

// Coefficient table a_n / z_n over the slot grid of a reflecting plan whose
// family is given by its density (PAPER, TABULATED), built on the host in
// float64: a_n = sigma sqrt(S(p_n) prod_i c(n_i) / |D|) at the frequencies
// p_i = k_i / (2 l_i), k_i = n_i (cosine axis) or N_i - n_i (sine axis), then
// rounded once to the working precision.
grf_status build_reflect_density_table(grf_plan_s* p, const grf_plan_desc& d) {
  const int rows = p->n1 * p->no, nd = p->nd;
  std::vector<double> h((size_t)rows * nd);
  // semantic axes: 0 = axis 1, 1 = middle, 2 = last; their lengths and l
  const int len[3] = {p->n1, p->no, p->nd};
  double l[3] = {1.0, 1.0, d.lengths[p->d - 1]};
  if (p->d >= 2) l[0] = d.lengths[0];
  if (p->d == 3) l[1] = d.lengths[1];
  const bool have[3] = {p->d >= 2, p->d == 3, true};
  for (int row = 0; row < rows; ++row) {
    const int n[2] = {row / p->no, row % p->no};
    for (int s = 0; s < nd; ++s) {
      const int slot[3] = {n[0], n[1], s};
      double pc[3];
      int np = 0;
      double c = 1.0;
      for (int ax = 0; ax < 3; ++ax) {
        if (!have[ax]) continue;
        const int k = ((p->sinemask >> ax) & 1) ? len[ax] - slot[ax] : slot[ax];
        pc[np++] = k / (2.0 * l[ax]);
        if (slot[ax] > 0) c *= 2.0;
      }
      double S;
      if (d.cov_kind == GRF_COV_PAPER) {
        double q = 0.0;
        for (int i = 0; i < np; ++i) q += std::pow(pc[i] * pc[i], d.k);
        S = std::pow(std::pow(d.m, (double)d.k * d.l) + std::pow(q, d.l), -(double)d.n);
      } else {
        S = d.spectrum[(size_t)row * nd + s];
      }
      h[(size_t)row * nd + s] = d.sigma * std::sqrt(S * c / p->vol);
    }
  }
  const size_t bytes = h.size() * p->esz;
  hipError_t e = hipMalloc(&p->htab, bytes);
  if (e != hipSuccess) return fail(GRF_ENOMEM, "hipMalloc of the coefficient table failed");
  if (p->dtype == GRF_F32) {
    std::vector<float> f(h.begin(), h.end());
    e = hipMemcpy(p->htab, f.data(), bytes, hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(p->htab, h.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "coefficient table upload");
  return GRF_OK;
}

// Checks of a tabulated density: finite, >= 0, and S(p) = S(-p) on the two
// planes k_d = 0 and N_d/2, where both entries are stored.
bool tabulated_ok(const grf_plan_desc& d, int n1, int no, int M) {
  const int rows = n1 * no;
  for (long long i = 0; i < (long long)rows * (M + 1); ++i)
    if (!(d.spectrum[i] >= 0) || !std::isfinite(d.spectrum[i])) return false;
  for (int row = 0; row < rows; ++row) {
    const int kk1 = row / no, o = row % no;
    const int mr = ((n1 - kk1) % n1) * no + (no - o) % no;
    for (int m : {0, M})
      if (d.spectrum[(size_t)row * (M + 1) + m] != d.spectrum[(size_t)mr * (M + 1) + m]) return false;
  }
  return true;
}

// Covariance estimator: workgroups of the one-dimensional epilogue (a fixed
// number, so that the result does not depend on the device) and the
// workspace layout: periodic d = 1 [partials: groups * P float64]; otherwise
// [acc: P float64][chunk of sampled fields].
constexpr long long COV_GROUPS = 2048;

struct CovLayout {
  long long groups, chunk;
  size_t acc, buf, total;
};

// The d = 1 one-FFT estimator is an epilogue of the one-launch sampler
// (listed lengths); every other plan estimates over sampled chunks.
bool cov_fused(const grf_plan_s* p) {
  return p->d == 1 && !p->reflect && p->desc.alg == GRF_ALG_ONE_FFT && p->listed;
}

CovLayout cov_layout(const grf_plan_s* p, long long n) {
  CovLayout c{};
  if (cov_fused(p)) {
    const grf::Geom g = grf::geom_gen1d(p->dtype, p->M);
    const long long rb = g.per_wg > 0 ? g.per_wg : 1;
    c.groups = std::min<long long>((n + rb - 1) / rb, COV_GROUPS);
    c.total = align256((size_t)c.groups * p->P * sizeof(double));
  } else {
    c.chunk = chunk_fields(p, n);
    c.acc = 0;
    c.buf = align256((size_t)p->P * sizeof(double));
    c.total = c.buf + align256((size_t)c.chunk * p->P * p->esz);
  }
  return c;
}

// stage < 0: run every pass; otherwise only that one.
grf_status sample_impl(grf_plan p, uint64_t seed, const void* zsrc, int64_t batch, const double* theta, void* out,
                       void* workspace, size_t ws_bytes, void* stream, int stage = -1) {
  if (p == nullptr) return fail(GRF_EINVAL, "null plan");
  if (batch < 0) return fail(GRF_EINVAL, "negative batch");
  if (batch == 0) return GRF_OK;
  if (out == nullptr) return fail(GRF_EINVAL, "null output");
  if (batch > 0x7fffffff) return fail(GRF_EINVAL, "batch too large");
  grf_status st = check_stream_device(p);
  if (st != GRF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const FieldRec* recs;
  int rstride;
  st = field_records(p, theta, batch, workspace, ws_bytes, s, &recs, &rstride);
  if (st != GRF_OK) return st;
  const std::vector<PassLaunch> v = sample_passes(p, seed, zsrc, batch, recs, rstride, out);
  if (stage >= (int)v.size()) return fail(GRF_EINVAL, "stage out of range");
  for (int i = 0; i < (int)v.size(); ++i) {
    if (stage >= 0 && i != stage) continue;
    st = run_launch(p, v[i], s);
    if (st != GRF_OK) return st;
  }
  return GRF_OK;
}

// ---- the adjoint's passes over one chunk of nb fields ----------------------
// c: the reduction pass's arguments (records, seed, noise, dL/dz, partial sums,
// c.data = the chunk's spectrum buffer); g: the chunk's upstream gradient.

// Last-axis real-to-complex transform of g into c.data (periodic plans).
grf_status adj_row_r2c(const grf_plan_s* p, const Args& c, const void* g, long long nb, hipStream_t s) {
  Args r = base_args(p, nb);
  r.data = c.data;
  r.src = g;
  r.tw2 = p->tw_row;
  r.rows = nb * (p->P / p->nd);
  return run_pass(p, grf::PASS_ROW_R2C_LOAD, p->M, r, 0, nb, s);
}

grf_status fwd_all_leading(const grf_plan_s* p, void* data, long long nb, hipStream_t s);

// One-FFT algorithm, periodic: G = F[g] by the last-axis R2C, (d = 3: the
// middle axis forward,) then axis 1 forward inside the reduction pass; d = 1:
// the reduction reads the last-axis spectrum.
grf_status adj_chunk_one_fft(const grf_plan_s* p, Args c, const void* g, const AdjTiles& at, void* plane,
                             long long nb, hipStream_t s) {
  grf_status st = adj_row_r2c(p, c, g, nb, s);
  if (st != GRF_OK) return st;
  const bool seq = p->desc.draw_order == GRF_DRAW_RECURSIVE;
  c.seq = seq;
  c.tag = seq ? 3 : 1;
  if (p->d == 1) {
    c.ntile = at.ntile;
    hipError_t e = grf::launch_grad1d(p->dtype, c, nb * at.ntile, s);
    return e == hipSuccess ? GRF_OK : hip_fail(e, "adjoint launch");
  }
  if (!p->listed) {
    // lengths without a compile-time adjoint column kernel: G transformed
    // along every leading axis in place, then the reduction reads it back
    st = fwd_all_leading(p, c.data, nb, s);
    if (st != GRF_OK) return st;
    c.ntile = at.ntile;
    if (nb * at.ntile > 0x7fffffffLL) return fail(GRF_EINVAL, "batch too large for one launch");
    hipError_t e = grf::launch_grad_gen(p->dtype, c, nb * at.ntile, s);
    return e == hipSuccess ? GRF_OK : hip_fail(e, "adjoint launch");
  }
  if (p->d == 3) {
    Args m = base_args(p, nb);
    m.data = c.data;
    m.tw = p->tw_col2;
    m.stride_ax = p->M;
    m.stride_fixed = (long long)p->no * p->M;
    m.nfixed = p->n1;
    st = run_pass(p, grf::PASS_COL_LOAD_FWD, p->no, m, 0, nb, s);
    if (st != GRF_OK) return st;
    c.plane = c.aux ? plane : nullptr;
  }
  c.tw = p->tw_col1;
  c.stride_ax = (long long)p->no * p->M;
  c.stride_fixed = p->M;
  c.nfixed = p->no;
  const int gp = p->d == 3 ? (seq ? grf::PASS_COL_GRAD3_SEQ : grf::PASS_COL_GRAD3)
                           : (seq ? grf::PASS_COL_GRAD_SEQ : grf::PASS_COL_GRAD);
  st = run_pass(p, gp, p->n1, c, 0, nb, s);
  if (st != GRF_OK) return st;
  if (p->d == 3 && c.aux) {
    hipError_t e = grf::launch_grad_plane(p->dtype, c, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  }
  return GRF_OK;
}

// Forward transforms along the leading axes of a packed spectrum (d = 3:
// middle axis, then axis 1), in place.
grf_status fwd_leading(const grf_plan_s* p, void* data, long long nb, hipStream_t s) {
  if (p->d != 3) return GRF_OK;
  Args m = base_args(p, nb);
  m.data = data;
  m.tw = p->tw_col2;
  m.stride_ax = p->M;
  m.stride_fixed = (long long)p->no * p->M;
  m.nfixed = p->n1;
  grf_status st = run_pass(p, grf::PASS_COL_LOAD_FWD, p->no, m, 0, nb, s);
  if (st != GRF_OK) return st;
  Args c = m;
  c.tw = p->tw_col1;
  c.stride_ax = (long long)p->no * p->M;
  c.stride_fixed = p->M;
  c.nfixed = p->no;
  return run_pass(p, grf::PASS_COL_LOAD_FWD, p->n1, c, 0, nb, s);
}

// Forward transforms along every leading axis of a packed spectrum, d = 2
// included (axis 1), in place.
grf_status fwd_all_leading(const grf_plan_s* p, void* data, long long nb, hipStream_t s) {
  if (p->d != 2) return fwd_leading(p, data, nb, s);
  Args c = base_args(p, nb);
  c.data = data;
  c.tw = p->tw_col1;
  c.stride_ax = p->M;
  c.stride_fixed = p->M;
  c.nfixed = 1;
  return run_pass(p, grf::PASS_COL_LOAD_FWD, p->n1, c, 0, nb, s);
}

// Two-FFT algorithm: xi = F[z] / sqrt(P), the white noise through the same
// transforms into spec2 (the table of a density-defined family already holds
// the 1/sqrt(P)); dL/dz is left to the caller (the sampler applied to g).
grf_status adj_chunk_two_fft(const grf_plan_s* p, Args c, const void* g, void* spec2, const AdjTiles& at,
                             long long nb, hipStream_t s) {
  grf_status st = adj_row_r2c(p, c, g, nb, s);
  if (st != GRF_OK) return st;
  if (p->d != 2 || !p->listed) {
    // d = 1, 3 (and d = 2 at lengths without a compile-time adjoint column
    // kernel): G = F[g] and F[z] transformed along every axis, then one
    // reduction pass over the two packed spectra
    st = fwd_all_leading(p, c.data, nb, s);
    if (st != GRF_OK) return st;
    Args rz = base_args(p, nb);
    rz.data = spec2;
    rz.src = c.src;
    rz.seed = c.seed;
    rz.tag = 0;
    rz.tw2 = p->tw_row;
    rz.rows = nb * (p->P / p->nd);
    st = run_pass(p, c.src ? grf::PASS_ROW_R2C_LOAD : grf::PASS_ROW_R2C_GEN, p->M, rz, 0, nb, s);
    if (st != GRF_OK) return st;
    st = fwd_all_leading(p, spec2, nb, s);
    if (st != GRF_OK) return st;
    c.src2 = spec2;
    c.scale = p->table_only ? 1.0 : 1.0 / std::sqrt((double)p->P);
    c.ntile = at.ntile;
    hipError_t e = grf::launch_grad_spec(p->dtype, c, nb * at.ntile, s);
    return e == hipSuccess ? GRF_OK : hip_fail(e, "adjoint launch");
  }
  Args rz = base_args(p, nb);
  rz.data = spec2;
  rz.src = c.src;
  rz.recs = c.recs;
  rz.rec_stride = c.rec_stride;
  rz.seed = c.seed;
  rz.tag = 0;
  rz.tw2 = p->tw_row;
  rz.rows = nb * (long long)p->n1;
  st = run_pass(p, c.src ? grf::PASS_ROW_R2C_LOAD : grf::PASS_ROW_R2C_GEN, p->M, rz, 0, nb, s);
  if (st != GRF_OK) return st;
  Args cz = base_args(p, nb);
  cz.data = spec2;
  cz.tw = p->tw_col1;
  cz.stride_ax = p->M;
  cz.stride_fixed = p->M;
  cz.nfixed = 1;
  st = run_pass(p, grf::PASS_COL_LOAD_FWD, p->n1, cz, 0, nb, s);
  if (st != GRF_OK) return st;
  c.tag = 0;
  c.aux = nullptr;
  c.src2 = spec2;
  c.scale = p->table_only ? 1.0 : 1.0 / std::sqrt((double)p->P);
  c.tw = p->tw_col1;
  c.stride_ax = p->M;
  c.stride_fixed = p->M;
  c.nfixed = 1;
  return run_pass(p, grf::PASS_COL_GRAD1, p->n1, c, 0, nb, s);
}

// Reflecting boundaries: B^T g by transposed cosine transforms (DCT-II), last
// axis first; the reduction runs with the last of them (axis 1, or the row
// for d = 1).
grf_status adj_chunk_reflect(const grf_plan_s* p, Args c, const void* g, long long nb, hipStream_t s) {
  c.tag = 2;
  c.bcmask = p->sinemask;
  c.src2 = c.src;   // a given noise (src carries g in the row pass)
  c.src = nullptr;
  Args rr = c;
  rr.src = g;
  rr.tw2 = p->tw_row;
  rr.tq = p->tq_row;
  rr.sine = (p->sinemask >> 2) & 1;
  rr.rows = nb * (p->P / p->nd);
  if (p->d == 1) return run_pass(p, grf::PASS_R2R_ROW_FWD_RED, p->M, rr, 0, nb, s);
  rr.aux = nullptr;
  grf_status st = run_pass(p, grf::PASS_R2R_ROW_FWD, p->M, rr, 0, nb, s);
  if (st != GRF_OK) return st;
  if (p->d == 3) {
    Args m = c;
    m.aux = nullptr;
    m.tw = p->tw_col2;
    m.tq = p->tq_col2;
    m.sine = (p->sinemask >> 1) & 1;
    m.stride_ax = p->M;
    m.stride_fixed = (long long)p->no * p->M;
    m.nfixed = p->n1;
    st = run_pass(p, grf::PASS_R2R_COL_FWD, p->no, m, 0, nb, s);
    if (st != GRF_OK) return st;
  }
  c.tw = p->tw_col1;
  c.tq = p->tq_col1;
  c.sine = p->sinemask & 1;
  c.stride_ax = (long long)p->no * p->M;
  c.stride_fixed = p->M;
  c.nfixed = p->no;
  return run_pass(p, grf::PASS_R2R_COL_FWD_RED, p->n1, c, 0, nb, s);
}

// ---- the plan autotuner -------------------------------------------------

// Passes whose kernel the tuner chooses, their names in the tuning cache and
// their direction.
const char* tune_pass_name(int pass) {
  switch (pass) {
    case grf::PASS_COL_GEN_INV: return "col-gen";
    case grf::PASS_COL_LOAD_INV: return "col-load";
    case grf::PASS_COL_LOAD_FWD: return "col-load";
    case grf::PASS_ROW_C2R: return "row-c2r";
    case grf::PASS_ROW_R2C_GEN: return "row-r2c-gen";
    case grf::PASS_ROW_R2C_LOAD: return "row-r2c-load";
    case grf::PASS_ROW_GEN_C2R: return "row-gen-c2r";
    default: return nullptr;
  }
}
const char* tune_dir(int pass) {
  return (pass == grf::PASS_COL_LOAD_FWD || pass == grf::PASS_ROW_R2C_GEN || pass == grf::PASS_ROW_R2C_LOAD) ? "fwd"
                                                                                                            : "inv";
}
int tune_pass_of(const std::string& name, const std::string& dir) {
  if (name == "col-gen" && dir == "inv") return grf::PASS_COL_GEN_INV;
  if (name == "col-load") return dir == "fwd" ? grf::PASS_COL_LOAD_FWD : grf::PASS_COL_LOAD_INV;
  if (name == "row-c2r" && dir == "inv") return grf::PASS_ROW_C2R;
  if (name == "row-r2c-gen" && dir == "fwd") return grf::PASS_ROW_R2C_GEN;
  if (name == "row-r2c-load" && dir == "fwd") return grf::PASS_ROW_R2C_LOAD;
  if (name == "row-gen-c2r" && dir == "inv") return grf::PASS_ROW_GEN_C2R;
  return -1;
}

// Can the runtime-radix kernel run this launch of this plan?  (The d = 1
// one-launch pass only for the one-FFT algorithm in the counter order.)
bool generic_capable(const grf_plan_s* p, int pass) {
  if (tune_pass_name(pass) == nullptr) return false;
  if (pass == grf::PASS_ROW_GEN_C2R)
    return p->desc.alg == GRF_ALG_ONE_FFT && p->desc.draw_order == GRF_DRAW_COUNTER;
  if (pass == grf::PASS_COL_GEN_INV) return p->desc.draw_order == GRF_DRAW_COUNTER;
  return true;
}

// Radix lists the tuner tries for L: every split of the power of two into
// radices 8, 4 and at most two 2s, with the 3s and 5s, each in up to four
// orders (large radices first, small first, odd radices first, the
// generator's order); duplicates removed, at most `cap` lists.
std::vector<std::vector<int>> radix_candidates(int L, size_t cap) {
  int n = L, e2 = 0, e3 = 0, e5 = 0;
  while (n % 2 == 0) { n /= 2; ++e2; }
  while (n % 3 == 0) { n /= 3; ++e3; }
  while (n % 5 == 0) { n /= 5; ++e5; }
  std::vector<std::vector<int>> out;
  if (n != 1) return out;
  auto add = [&](std::vector<int> r) {
    if (r.size() > 16 || out.size() >= cap) return;
    if (std::find(out.begin(), out.end(), r) == out.end()) out.push_back(r);
  };
  {
    int gen[16];
    const int ns = grf::radix_plan(L, gen);
    if (ns > 0) add(std::vector<int>(gen, gen + ns));
  }
  for (int a8 = e2 / 3; a8 >= 0; --a8) {
    for (int b4 = (e2 - 3 * a8) / 2; b4 >= 0; --b4) {
      const int c2 = e2 - 3 * a8 - 2 * b4;
      if (c2 > 2) continue;
      std::vector<int> ms;
      for (int i = 0; i < a8; ++i) ms.push_back(8);
      for (int i = 0; i < b4; ++i) ms.push_back(4);
      for (int i = 0; i < c2; ++i) ms.push_back(2);
      for (int i = 0; i < e5; ++i) ms.push_back(5);
      for (int i = 0; i < e3; ++i) ms.push_back(3);
      if (ms.empty()) continue;
      std::vector<int> desc = ms, asc = ms, odd;
      std::sort(desc.begin(), desc.end(), std::greater<int>());
      std::sort(asc.begin(), asc.end());
      for (int r : desc) if (r % 2) odd.push_back(r);
      for (int r : desc) if (r % 2 == 0) odd.push_back(r);
      add(desc);
      add(odd);
      add(asc);
    }
  }
  return out;
}

std::string choice_text(const TuneChoice& c) {
  if (!c.generic) return "fixed";
  std::string t = "generic " + std::to_string(c.vpt) + " ";
  for (int i = 0; i < c.ns; ++i) t += (i ? "," : "") + std::to_string(c.rad[i]);
  return t;
}

// A cache entry's choice, validated against the plan (a compile-time kernel
// must exist for "fixed"; the radices must be from {2, 3, 4, 5, 8} and
// multiply to L).
bool parse_choice(const grf_plan_s* p, int pass, long long L, const std::vector<std::string>& w, TuneChoice* c) {
  if (w[0] == "fixed") {
    if (!fixed_length(pass, (int)L)) return false;
    *c = TuneChoice{};
    return true;
  }
  if (w[0] != "generic" || w.size() != 3 || !generic_capable(p, pass)) return false;
  TuneChoice t;
  t.generic = true;
  t.vpt = std::atoi(w[1].c_str());
  if (t.vpt != 4 && t.vpt != 8) return false;
  if (grf::generic_geom(pass, p->dtype, (int)L, t.vpt).threads <= 0) return false;   // no such kernel shape
  long long prod = 1;
  size_t i = 0;
  const std::string& r = w[2];
  while (i < r.size()) {
    size_t j = r.find(',', i);
    if (j == std::string::npos) j = r.size();
    const int v = std::atoi(r.substr(i, j - i).c_str());
    if ((v != 2 && v != 3 && v != 4 && v != 5 && v != 8) || t.ns >= 16) return false;
    t.rad[t.ns++] = v;
    prod *= v;
    i = j + 1;
  }
  if (prod != L) return false;
  *c = t;
  return true;
}

// The (pass, length) pairs of the plan's sampler that the tuner can choose for.
std::vector<std::pair<int, int>> tunable_passes(const grf_plan_s* p, long long batch) {
  const UnsplitScope unsplit(p);
  std::vector<std::pair<int, int>> v;
  for (const PassLaunch& pl : sample_passes(p, 0, nullptr, batch, p->rec_dev, 0, nullptr)) {
    if (tune_pass_name(pl.pass) == nullptr) continue;
    const std::pair<int, int> k(pl.pass, pl.L);
    if (std::find(v.begin(), v.end(), k) == v.end()) v.push_back(k);
  }
  return v;
}

void load_plan_cache(grf_plan_s* p) {
  const std::vector<std::pair<int, int>> mine = tunable_passes(p, 1);
  const char* dt = p->dtype == GRF_F32 ? "f32" : "f64";
  for (const grf::tune::Line& l : grf::tune::read("plan", grf::tune::arch_name(p->device))) {
    if (l.dtype != dt) continue;
    const int pass = tune_pass_of(l.pass, l.dir);
    if (pass < 0) continue;
    if (std::find(mine.begin(), mine.end(), std::make_pair(pass, (int)l.length)) == mine.end()) continue;
    TuneChoice c;
    if (parse_choice(p, pass, l.length, l.choice, &c)) p->tune[tune_key(pass, (int)l.length)] = c;
  }
}

}  // namespace

namespace grf {

bool col_length_supported(int L) {
  switch (L) {
#define GRF_X(L_) case L_:
    GRF_COL_LENGTHS(GRF_X)
#undef GRF_X
    return true;
    default:
      return false;
  }
}

bool row_length_supported(int M) {
  switch (M) {
#define GRF_X(M_) case M_:
    GRF_ROW_LENGTHS(GRF_X)
#undef GRF_X
    return true;
    default:
      return false;
  }
}

Geom pass_geom(int pass, int dtype, int L) {
  if (pass == PASS_SPEC_FILTER || pass == PASS_SPEC_FILTER0) return Geom{256, 0};
  if (is_r2r_pass(pass)) return geom_r2r(pass, dtype, L);
  if (pass == PASS_ROW_GEN_C2R) return geom_gen1d(dtype, L);
  if (is_row_pass(pass)) return dtype == 0 ? geom_row_f32(pass, L) : geom_row_f64(pass, L);
  return dtype == 0 ? geom_col_f32(pass, L) : geom_col_f64(pass, L);
}

hipError_t launch_pass(int pass, int dtype, int L, const Args& a, long long nblocks, hipStream_t s) {
  if (pass == PASS_SPEC_FILTER || pass == PASS_SPEC_FILTER0)
    return launch_spec_filter(dtype, a, nblocks, pass == PASS_SPEC_FILTER0, s);
  if (is_r2r_pass(pass)) return launch_r2r(pass, dtype, L, a, nblocks, s);
  if (pass == PASS_ROW_GEN_C2R) return launch_gen1d(dtype, L, a, nblocks, nullptr, s);
  if (is_row_pass(pass))
    return dtype == 0 ? launch_row_f32(pass, L, a, nblocks, s) : launch_row_f64(pass, L, a, nblocks, s);
  return dtype == 0 ? launch_col_f32(pass, L, a, nblocks, s) : launch_col_f64(pass, L, a, nblocks, s);
}

}  // namespace grf

extern "C" {

const char* grf_last_error(void) { return g_err.c_str(); }

const char* grf_version(void) { return "grf-mi355x 0.1 (gfx950)"; }

grf_status grf_plan_create(const grf_plan_desc* desc, grf_plan* out) {
  if (desc == nullptr || out == nullptr) return fail(GRF_EINVAL, "null argument");
  *out = nullptr;
  const grf_plan_desc& d = *desc;
  if (d.ndim < 1 || d.ndim > 3) return fail(GRF_EINVAL, "ndim must be 1, 2 or 3");
  if (d.alg != GRF_ALG_TWO_FFT && d.alg != GRF_ALG_ONE_FFT) return fail(GRF_EINVAL, "unknown algorithm");
  if (d.dtype != GRF_F32 && d.dtype != GRF_F64) return fail(GRF_EINVAL, "unknown dtype");
  if (d.cov_kind < GRF_COV_GAUSSIAN || d.cov_kind > GRF_COV_TABULATED)
    return fail(GRF_EINVAL, "unknown covariance kind");
  const bool table_only = d.cov_kind == GRF_COV_PAPER || d.cov_kind == GRF_COV_TABULATED;
  if (d.cov_kind == GRF_COV_PAPER &&
      (!(d.m > 0) || !std::isfinite(d.m) || d.k < 1 || d.l < 1 || d.n < 1 || d.k > 64 || d.l > 64 || d.n > 64))
    return fail(GRF_EINVAL, "the family of Section 4 needs m > 0 and 1 <= k, l, n <= 64");
  if (d.cov_kind == GRF_COV_TABULATED && d.spectrum == nullptr) return fail(GRF_EINVAL, "null spectrum");
  for (int i = 0; i < d.ndim; ++i) {
    if (d.dims[i] <= 0 || (d.dims[i] % 2) != 0) return fail(GRF_EINVAL, "grid sizes must be positive and even");
    if (!smooth235(d.dims[i])) return fail(GRF_EINVAL, "grid sizes must factor into 2, 3 and 5");
    if (!(d.lengths[i] > 0) || !std::isfinite(d.lengths[i])) return fail(GRF_EINVAL, "edge lengths must be > 0");
  }
  if (!(d.sigma > 0) || !std::isfinite(d.sigma) ||
      (!table_only && (!(d.length_scale > 0) || !std::isfinite(d.length_scale))))
    return fail(GRF_EINVAL, "sigma and length_scale must be > 0");
  if (d.cov_kind == GRF_COV_MATERN && (!(d.nu > 0) || !std::isfinite(d.nu)))
    return fail(GRF_EINVAL, "nu must be > 0");
  int nreflect = 0;
  for (int i = 0; i < d.ndim; ++i) {
    if (d.bc[i] < GRF_BC_PERIODIC || d.bc[i] > GRF_BC_DIRICHLET) return fail(GRF_EINVAL, "unknown boundary condition");
    nreflect += d.bc[i] != GRF_BC_PERIODIC;
  }
  const bool reflect = nreflect > 0;
  if (reflect && nreflect != d.ndim)
    return fail(GRF_EUNSUPPORTED, "periodic and reflecting axes cannot be mixed");
  if (d.draw_order != GRF_DRAW_COUNTER && d.draw_order != GRF_DRAW_RECURSIVE)
    return fail(GRF_EINVAL, "unknown draw order");
  if (d.draw_order == GRF_DRAW_RECURSIVE && (reflect || d.alg != GRF_ALG_ONE_FFT))
    return fail(GRF_EUNSUPPORTED, "the recursive draw order is that of the periodic one-FFT algorithm");
  if (reflect && d.alg != GRF_ALG_ONE_FFT)
    return fail(GRF_EUNSUPPORTED, "reflecting boundaries use the one-transform method (GRF_ALG_ONE_FFT)");
  const int last = d.ndim - 1;
  // every even 2/3/5-smooth length: the listed ones (grf_configs.hpp) on the
  // compile-time kernels, the others on the runtime-radix kernels up to their
  // limits
  bool listed = d.dims[last] / 2 <= GRF_GENERIC_MAX_ROW && grf::row_length_supported((int)(d.dims[last] / 2));
  if (d.dims[last] / 2 > GRF_GENERIC_MAX_ROW)
    return fail(GRF_EUNSUPPORTED, "last-axis length above 2 * GRF_GENERIC_MAX_ROW");
  for (int i = 0; i < last; ++i) {
    if (d.dims[i] > GRF_GENERIC_MAX_COL) return fail(GRF_EUNSUPPORTED, "leading-axis length above GRF_GENERIC_MAX_COL");
    listed = listed && grf::col_length_supported((int)d.dims[i]);
  }
  if (!listed && (reflect || d.draw_order == GRF_DRAW_RECURSIVE))
    return fail(GRF_EUNSUPPORTED, "reflecting boundaries and the recursive draw order take the listed grid lengths only");

  grf_plan_s* p = new (std::nothrow) grf_plan_s();
  if (p == nullptr) return fail(GRF_ENOMEM, "host allocation failed");
  p->desc = d;
  p->d = d.ndim;
  p->n1 = d.ndim >= 2 ? (int)d.dims[0] : 1;   // d = 1: a field is one row
  p->no = d.ndim == 3 ? (int)d.dims[1] : 1;
  p->nd = (int)d.dims[last];
  p->M = p->nd / 2;
  p->P = (long long)p->n1 * p->no * p->nd;
  p->vol = 1.0;
  for (int i = 0; i < d.ndim; ++i) p->vol *= d.lengths[i];
  p->il2[0] = d.ndim >= 2 ? 1.0 / (d.lengths[0] * d.lengths[0]) : 0.0;
  p->il2[1] = d.ndim == 3 ? 1.0 / (d.lengths[1] * d.lengths[1]) : 0.0;
  p->il2[2] = 1.0 / (d.lengths[last] * d.lengths[last]);
  p->dtype = d.dtype;
  p->esz = d.dtype == GRF_F32 ? 4 : 8;
  p->reflect = reflect;
  p->listed = listed;
  if (reflect) {
    for (int i = 0; i < d.ndim; ++i) {
      // semantic axis of descriptor axis i: 0 = axis 1, 1 = middle, 2 = last
      const int ax = (i == d.ndim - 1) ? 2 : i;
      if (d.bc[i] == GRF_BC_DIRICHLET) p->sinemask |= 1 << ax;
    }
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  FieldRec rec;
  if (table_only) {
    if (d.cov_kind == GRF_COV_TABULATED && reflect) {
      for (long long i = 0; i < p->P; ++i)
        if (!(d.spectrum[i] >= 0) || !std::isfinite(d.spectrum[i])) {
          delete p;
          return fail(GRF_EINVAL, "tabulated density must be finite and >= 0");
        }
    } else if (d.cov_kind == GRF_COV_TABULATED && !tabulated_ok(d, p->n1, p->no, p->M)) {
      delete p;
      return fail(GRF_EINVAL, "tabulated density must be finite, >= 0 and symmetric on the planes k_d = 0, N_d/2");
    }
    grf::make_table_rec(d.sigma, &rec);
    p->table_only = true;
  } else if (grf::make_field_rec(d.cov_kind, d.ndim, p->vol, d.sigma, d.length_scale, d.nu, &rec) != 0) {
    delete p;
    return fail(GRF_EINVAL, "invalid covariance parameters");
  }
  grf_status st = d.ndim >= 2 ? make_table(p->n1, p->dtype, &p->tw_col1) : GRF_OK;
  if (st == GRF_OK && d.ndim == 3) st = make_table(p->no, p->dtype, &p->tw_col2);
  if (st == GRF_OK) st = make_table(p->nd, p->dtype, &p->tw_row);
  if (st == GRF_OK && reflect) {
    if (d.ndim >= 2) st = make_qtable(p->n1, p->n1, p->dtype, &p->tq_col1);
    if (st == GRF_OK && d.ndim == 3) st = make_qtable(p->no, p->no, p->dtype, &p->tq_col2);
    if (st == GRF_OK) st = make_row_rtable(p->nd, p->dtype, &p->tq_row);
  }
  if (st == GRF_OK) {
    e = hipMalloc((void**)&p->rec_dev, sizeof(FieldRec));
    if (e != hipSuccess) st = fail(GRF_ENOMEM, "hipMalloc of field record failed");
    else {
      e = hipMemcpy(p->rec_dev, &rec, sizeof(FieldRec), hipMemcpyHostToDevice);
      if (e != hipSuccess) st = hip_fail(e, "record upload");
    }
  }
  if (st == GRF_OK && reflect && table_only) {
    st = build_reflect_density_table(p, d);
  } else if (st == GRF_OK && reflect && d.ndim <= 2) {
    // a_n / z_n of every slot for the default parameters, by the kernels' own
    // float expressions (the generation passes read it)
    Args t = base_args(p, 1);
    t.recs = p->rec_dev;
    t.bcmask = p->sinemask;
    const size_t bytes = (size_t)p->P * p->esz;
    e = hipMalloc(&p->htab, bytes);
    if (e != hipSuccess) {
      st = fail(GRF_ENOMEM, "hipMalloc of the coefficient table failed");
    } else {
      e = grf::launch_r2r_table(p->dtype, t, p->htab, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
      if (e != hipSuccess) st = hip_fail(e, "coefficient table");
    }
  } else if (st == GRF_OK && reflect) {
    // d = 3: coefficients on the fly
  } else if (st == GRF_OK && table_only) {
    st = build_density_table(p, d, d.alg == GRF_ALG_TWO_FFT ? 1.0 / std::sqrt((double)p->P) : 1.0);
  } else if (st == GRF_OK && d.ndim == 2 && d.alg == GRF_ALG_ONE_FFT) {
    // filter table: h of every (row, m) for the default parameters, computed by
    // the kernels' own float expressions (read by the generation and adjoint passes)
    Args t = base_args(p, 1);
    t.recs = p->rec_dev;
    st = grf::build_filter_table(p->dtype, t, 1.0, &p->htab);
  }
  if (st != GRF_OK) {
    grf_plan_destroy(p);
    return st;
  }
  load_plan_cache(p);
  *out = p;
  return GRF_OK;
}

grf_status grf_plan_destroy(grf_plan p) {
  if (p == nullptr) return GRF_OK;
  if (p->tw_col1) (void)hipFree(p->tw_col1);
  if (p->tw_col2) (void)hipFree(p->tw_col2);
  if (p->tw_row) (void)hipFree(p->tw_row);
  if (p->rec_dev) (void)hipFree(p->rec_dev);
  if (p->htab) (void)hipFree(p->htab);
  if (p->tq_col1) (void)hipFree(p->tq_col1);
  if (p->tq_col2) (void)hipFree(p->tq_col2);
  if (p->tq_row) (void)hipFree(p->tq_row);
  delete p;
  return GRF_OK;
}

grf_status grf_workspace_size(grf_plan p, int64_t batch, int32_t op, size_t* bytes) {
  if (p == nullptr || bytes == nullptr) return fail(GRF_EINVAL, "null argument");
  if (batch < 0) return fail(GRF_EINVAL, "negative batch");
  if (op != GRF_OP_SAMPLE && op != GRF_OP_BACKWARD && op != GRF_OP_COVARIANCE) return fail(GRF_EINVAL, "unknown op");
  *bytes = op == GRF_OP_COVARIANCE ? (batch > 0 ? cov_layout(p, batch).total : 0) : ws_layout(p, batch, op).total;
  return GRF_OK;
}

grf_status grf_covariance(grf_plan p, uint64_t seed, int64_t nsamples, double* cov, void* workspace,
                          size_t workspace_bytes, void* stream) {
  if (p == nullptr || cov == nullptr) return fail(GRF_EINVAL, "null argument");
  if (nsamples < 1) return fail(GRF_EINVAL, "nsamples must be >= 1");
  grf_status st = check_stream_device(p);
  if (st != GRF_OK) return st;
  const CovLayout c = cov_layout(p, nsamples);
  if (workspace == nullptr || workspace_bytes < c.total) return fail(GRF_EINVAL, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const double scale = 1.0 / (double)nsamples;
  if (cov_fused(p)) {
    double* partial = (double*)workspace;
    Args a = base_args(p, nsamples);
    a.recs = p->rec_dev;
    a.rec_stride = 0;
    a.seed = seed;
    a.seq = p->desc.draw_order == GRF_DRAW_RECURSIVE;
    a.tag = a.seq ? 3 : 1;
    a.tw2 = p->tw_row;
    a.rows = nsamples;
    a.htab = p->table_only ? p->htab : nullptr;
    hipError_t e = grf::launch_gen1d(p->dtype, p->M, a, c.groups, partial, s);
    if (e == hipSuccess) e = grf::launch_cov_reduce(partial, (int)c.groups, p->P, scale, cov, s);
    if (e != hipSuccess) return hip_fail(e, "covariance launch");
    return GRF_OK;
  }
  double* acc = (double*)workspace;
  void* buf = (char*)workspace + c.buf;
  // acc = 0 (a reduction over no partial sums)
  hipError_t e = grf::launch_cov_reduce(nullptr, 0, p->P, 0.0, acc, s);
  if (e != hipSuccess) return hip_fail(e, "covariance launch");
  for (long long c0 = 0; c0 < nsamples; c0 += c.chunk) {
    const long long nb = std::min(c.chunk, nsamples - c0);
    st = sample_impl(p, seed + (uint64_t)c0, nullptr, nb, nullptr, buf, nullptr, 0, stream);
    if (st != GRF_OK) return st;
    e = grf::launch_cov_accum(p->dtype, buf, (int)nb, p->P, acc, s);
    if (e != hipSuccess) return hip_fail(e, "covariance launch");
  }
  e = grf::launch_cov_reduce(acc, 1, p->P, scale, cov, s);
  if (e != hipSuccess) return hip_fail(e, "covariance launch");
  return GRF_OK;
}

grf_status grf_sample(grf_plan p, uint64_t seed, int64_t batch, const double* theta, void* out, void* workspace,
                      size_t workspace_bytes, void* stream) {
  return sample_impl(p, seed, nullptr, batch, theta, out, workspace, workspace_bytes, stream);
}

grf_status grf_sample_from_noise(grf_plan p, const void* noise, int64_t batch, const double* theta, void* out,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  if (noise == nullptr && batch > 0) return fail(GRF_EINVAL, "null noise");
  if (noise != nullptr && noise == out) return fail(GRF_EINVAL, "noise and output must not alias");
  return sample_impl(p, 0, noise, batch, theta, out, workspace, workspace_bytes, stream);
}

grf_status grf_sample_stage_count(grf_plan p, int64_t batch, int32_t* count) {
  if (p == nullptr || count == nullptr) return fail(GRF_EINVAL, "null argument");
  if (batch < 1) return fail(GRF_EINVAL, "batch must be positive");
  *count = (int32_t)sample_passes(p, 0, nullptr, batch, p->rec_dev, 0, nullptr).size();
  return GRF_OK;
}

grf_status grf_sample_stage_info(grf_plan p, int64_t batch, int32_t stage, int32_t* kind, int64_t* first,
                                 int64_t* count) {
  if (p == nullptr) return fail(GRF_EINVAL, "null plan");
  if (batch < 1) return fail(GRF_EINVAL, "batch must be positive");
  const std::vector<PassLaunch> v = sample_passes(p, 0, nullptr, batch, p->rec_dev, 0, nullptr);
  if (stage < 0 || stage >= (int)v.size()) return fail(GRF_EINVAL, "stage out of range");
  const PassLaunch& pl = v[stage];
  if (kind) *kind = pl.pass;
  if (first) *first = pl.first;
  if (count) *count = pl.count;
  return GRF_OK;
}

grf_status grf_sample_stage(grf_plan p, int32_t stage, uint64_t seed, int64_t batch, const double* theta, void* out,
                            void* workspace, size_t workspace_bytes, void* stream) {
  if (stage < 0) return fail(GRF_EINVAL, "negative stage");
  return sample_impl(p, seed, nullptr, batch, theta, out, workspace, workspace_bytes, stream, stage);
}

grf_status grf_noise(grf_plan p, uint64_t seed, int64_t batch, void* noise_out, void* stream) {
  if (p == nullptr) return fail(GRF_EINVAL, "null plan");
  if (batch < 0) return fail(GRF_EINVAL, "negative batch");
  if (batch == 0) return GRF_OK;
  if (noise_out == nullptr) return fail(GRF_EINVAL, "null output");
  if (batch > 0x7fffffff) return fail(GRF_EINVAL, "batch too large");
  grf_status st = check_stream_device(p);
  if (st != GRF_OK) return st;
  const int tag = p->reflect ? 2 : p->desc.draw_order == GRF_DRAW_RECURSIVE ? 3 : (p->desc.alg == GRF_ALG_ONE_FFT ? 1 : 0);
  hipError_t e = grf::launch_noise(p->dtype, seed, tag, (int)(p->P / p->nd), p->nd, (int)batch, noise_out,
                                   (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "noise kernel");
  return GRF_OK;
}

grf_status grf_backward(grf_plan p, uint64_t seed, const void* noise, int64_t batch, const double* theta,
                        const void* grad_out, double* grad_theta, void* grad_noise, void* workspace,
                        size_t workspace_bytes, void* stream) {
  if (p == nullptr) return fail(GRF_EINVAL, "null plan");
  if (batch < 0) return fail(GRF_EINVAL, "negative batch");
  if (batch == 0) return GRF_OK;
  if (grad_out == nullptr || grad_theta == nullptr) return fail(GRF_EINVAL, "null gradient pointer");
  if (batch > 0x7fffffff) return fail(GRF_EINVAL, "batch too large");
  const WsLayout w = ws_layout(p, batch, GRF_OP_BACKWARD);
  if (workspace == nullptr || workspace_bytes < w.total) return fail(GRF_EINVAL, "workspace too small");
  grf_status st = check_stream_device(p);
  if (st != GRF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const FieldRec* recs;
  int rstride;
  st = field_records(p, theta, batch, ws + w.recs, w.partial, s, &recs, &rstride);
  if (st != GRF_OK) return st;
  // chunk by chunk (cache-sized, as the sampler), so that each pass reads the
  // previous one's output from the last-level cache
  const AdjTiles at = adj_tiles(p);
  const long long C = chunk_fields(p, batch);
  const size_t fbytes = (size_t)p->P * p->esz;
  for (long long c0 = 0; c0 < batch; c0 += C) {
    const long long nb = std::min(C, batch - c0);
    // the arguments of the reduction pass
    Args c = base_args(p, nb);
    c.recs = rstride ? recs + c0 : recs;
    c.rec_stride = rstride;
    c.seed = seed + (uint64_t)c0;
    c.htab = rstride == 0 ? p->htab : nullptr;
    c.data = ws + w.spec;
    c.src = noise ? (const char*)noise + c0 * fbytes : nullptr;
    c.aux = grad_noise ? (char*)grad_noise + c0 * fbytes : nullptr;
    c.partial = (double*)(ws + w.partial) + c0 * at.nper * 3;
    const void* g = (const char*)grad_out + c0 * fbytes;
    if (p->reflect)
      st = adj_chunk_reflect(p, c, g, nb, s);
    else if (p->desc.alg == GRF_ALG_TWO_FFT)
      st = adj_chunk_two_fft(p, c, g, ws + w.spec2, at, nb, s);
    else
      st = adj_chunk_one_fft(p, c, g, at, grad_noise ? ws + w.plane : nullptr, nb, s);
    if (st != GRF_OK) return st;
  }
  hipError_t e = grf::launch_reduce_partials((const double*)(ws + w.partial), (int)batch, at.nper, grad_theta, s);
  if (e != hipSuccess) return hip_fail(e, "reduction");
  if (p->desc.alg == GRF_ALG_TWO_FFT && grad_noise != nullptr) {
    // phi = F*[h F[z]] / sqrt(P) with h real and even is a symmetric operator
    // of z, so dL/dz is the same sampler applied to g
    for (const PassLaunch& pl : sample_passes(p, seed, grad_out, batch, recs, rstride, grad_noise)) {
      st = run_launch(p, pl, s);
      if (st != GRF_OK) return st;
    }
  }
  return GRF_OK;
}

grf_status grf_plan_tune(grf_plan p, int64_t batch, void* out, void* stream) {
  if (p == nullptr || out == nullptr) return fail(GRF_EINVAL, "null argument");
  if (batch < 1) return fail(GRF_EINVAL, "batch must be positive");
  grf_status st = check_stream_device(p);
  if (st != GRF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const long long nb = std::min<long long>(batch, chunk_fields(p, batch));
  const UnsplitScope unsplit(p);
  const std::vector<PassLaunch> v = sample_passes(p, 0, nullptr, nb, p->rec_dev, 0, out);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(GRF_EDEVICE, "event creation");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(GRF_EDEVICE, "event creation");
  }
  const std::string arch = grf::tune::arch_name(p->device);
  const char* dt = p->dtype == GRF_F32 ? "f32" : "f64";
  std::string lines;
  std::vector<long long> done;
  for (size_t i = 0; i < v.size() && st == GRF_OK; ++i) {
    const int pass = v[i].pass, L = v[i].L;
    const long long key = tune_key(pass, L);
    if (tune_pass_name(pass) == nullptr || std::find(done.begin(), done.end(), key) != done.end()) continue;
    done.push_back(key);
    std::vector<TuneChoice> cand;
    if (fixed_length(pass, L)) cand.push_back(TuneChoice{});
    if (generic_capable(p, pass)) {
      for (int vpt : {8, 4}) {
        for (const std::vector<int>& r : radix_candidates(L, 6)) {
          TuneChoice c;
          c.generic = true;
          c.vpt = vpt;
          c.ns = (int)r.size();
          for (int k = 0; k < c.ns; ++k) c.rad[k] = r[k];
          cand.push_back(c);
        }
      }
    }
    float best = 1e30f;
    TuneChoice bestc;
    bool any = false;
    for (const TuneChoice& c : cand) {
      p->tune[key] = c;
      if (run_launch(p, v[i], s) != GRF_OK) continue;   // a shape this kernel cannot take
      float tmin = 1e30f;
      for (int rep = 0; rep < 3 && st == GRF_OK; ++rep) {
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) st = run_launch(p, v[i], s);
        if (st != GRF_OK) break;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) st = hip_fail(e, "tuning run");
        tmin = std::min(tmin, t);
      }
      if (st != GRF_OK) break;
      if (tmin < best) {
        best = tmin;
        bestc = c;
        any = true;
      }
    }
    if (st != GRF_OK) break;
    if (!any) {
      p->tune.erase(key);
      continue;
    }
    p->tune[key] = bestc;
    lines += std::string("plan ") + arch + " " + dt + " " + tune_pass_name(pass) + " " + tune_dir(pass) + " " +
             std::to_string(L) + " " + choice_text(bestc) + "\n";
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GRF_OK) return st;
  grf::tune::append(lines);
  return GRF_OK;
}

grf_status grf_plan_tune_choice(grf_plan p, int32_t pass, int64_t length, char* buf, size_t len) {
  if (p == nullptr || buf == nullptr || len == 0) return fail(GRF_EINVAL, "null argument");
  const TuneChoice* c = tune_choice(p, pass, (int)length);
  const std::string t = c ? choice_text(*c) : std::string("default");
  std::snprintf(buf, len, "%s", t.c_str());
  return GRF_OK;
}

grf_status grf_debug_spectrum(grf_plan p, uint64_t seed, int64_t batch, void* spec_out, void* stream) {
  if (p == nullptr || (spec_out == nullptr && batch > 0)) return fail(GRF_EINVAL, "null argument");
  if (batch < 0) return fail(GRF_EINVAL, "negative batch");
  if (p->desc.alg != GRF_ALG_ONE_FFT || p->reflect || p->desc.draw_order != GRF_DRAW_COUNTER)
    return fail(GRF_EUNSUPPORTED, "spectrum defined for the one-FFT algorithm, periodic axes, counter draw order");
  if (batch == 0) return GRF_OK;
  grf_status st = check_stream_device(p);
  if (st != GRF_OK) return st;
  Args a = base_args(p, batch);
  a.data = spec_out;
  a.recs = p->rec_dev;
  a.rec_stride = 0;
  a.seed = seed;
  a.tag = 1;
  a.htab = p->htab;
  const long long slots = (long long)(p->P / p->nd) * ((p->M + 1) / 2);
  a.ntile = (int)((slots + 255) / 256);
  const long long nblocks = batch * a.ntile;
  if (nblocks > 0x7fffffffLL) return fail(GRF_EINVAL, "batch too large for one launch");
  hipError_t e = grf::launch_debug_spectrum(p->dtype, a, nblocks, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "spectrum kernel");
  return GRF_OK;
}

grf_status grf_debug_philox(uint64_t seed, const uint32_t* counters, int64_t n, uint32_t* out, void* stream) {
  if (n < 0) return fail(GRF_EINVAL, "negative count");
  if (n == 0) return GRF_OK;
  if (counters == nullptr || out == nullptr) return fail(GRF_EINVAL, "null pointer");
  hipError_t e = grf::launch_philox_raw(seed, counters, n, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "philox kernel");
  return GRF_OK;
}

}  // extern "C"
