// Host side of the batch entry points of include/grf.h: field records, work
// queues, the hipGraph of the two persistent launches, the one-field-per-launch
// baseline and the tile-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "grf.h"
#include "grf_batch.hpp"
#include "grf_dispatch.hpp"
#include "grf_host.hpp"
#include "grf_kernels.hpp"
#include "grf_tune_cache.hpp"

using grf::BatchField;
using grf::BatchItem;
using grf::host::fail;
using grf::host::hip_fail;

struct grf_batch_s {
  std::vector<grf_field_desc> desc;
  std::vector<long long> offsets;      // element offsets, nfields + 1
  std::vector<BatchField> fields;      // host copy of the device records
  std::map<int, int> cvar, rvar;       // tile-shape variant per column length / half-length
  std::map<int, int> twoff;            // twiddle pool offset per length
  BatchField* d_fields = nullptr;
  BatchItem* d_col = nullptr;
  BatchItem* d_row = nullptr;
  int* d_qoff = nullptr;               // column queue offsets, XCD_QUEUES + 1
  int ncol = 0, nrow = 0;
  void* d_tw = nullptr;
  int* d_counters = nullptr;
  int nwg_col = 0, nwg_row = 0;
  hipStream_t cap = nullptr;           // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_out = nullptr;           // output pointer baked into the graph
  int device = 0;
  // one-launch mode (the default where every XCD was seen at creation):
  // per-XCD queues of column and row items, per-field readiness counters
  bool one = false;
  long long group_bytes = 24ll << 20;  // fields per pipeline group of an XCD queue, in output bytes
  BatchItem* d_one_items = nullptr;
  int* d_one_qoff = nullptr;           // XCD_QUEUES + 1
  int* d_one_state = nullptr;          // [queue counters XCD_QUEUES][err][pad to 16][done, one per field]
  int nwg_one = 0;
};

namespace {

void free_graph(grf_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_out = nullptr;
}

// Cost weights for largest-first ordering of the work queues.
struct WItem {
  BatchItem it;
  long long cost;
};

// Column work items of the given fields (field, tiles, cost) in XCD_QUEUES
// queues: fields in decreasing order of cost go to the least-loaded queue,
// all tiles of a field together and in order, so that adjacent tiles run on
// one XCD.  qoff receives the XCD_QUEUES + 1 queue offsets.
void col_queues(std::vector<std::array<long long, 3>> fl, std::vector<BatchItem>& items, std::vector<int>& qoff) {
  std::stable_sort(fl.begin(), fl.end(), [](const std::array<long long, 3>& x, const std::array<long long, 3>& y) {
    return x[2] > y[2];
  });
  std::vector<std::vector<BatchItem>> q(grf::XCD_QUEUES);
  std::vector<long long> load(grf::XCD_QUEUES, 0);
  for (const auto& f : fl) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    for (long long t = 0; t < f[1]; ++t) q[x].push_back({(int)f[0], (int)t});
    load[x] += f[2];
  }
  items.clear();
  qoff.assign(grf::XCD_QUEUES + 1, 0);
  for (int x = 0; x < grf::XCD_QUEUES; ++x) {
    items.insert(items.end(), q[x].begin(), q[x].end());
    qoff[x + 1] = (int)items.size();
  }
}

constexpr int ONE_STATE_DONE = 16;     // offset of the readiness counters in d_one_state

// One-launch queues: fields go to the XCD queues largest first, each to the
// least-loaded queue; an XCD's fields are cut into groups of up to
// group_bytes of output, and its queue holds the column items of group 0,
// then for g = 1, 2, ... the column items of group g merged with the row items
// of group g - 1, and at the end the row items of the last group: a field's
// row items come one group after its column items, so they rarely wait and
// read a spectrum that is still in the caches, and every row item comes after
// all column items of its field (each of which a running workgroup took
// before), so every wait ends.
grf_status build_one_queues(grf_batch_s* b) {
  const int n = (int)b->desc.size();
  std::vector<int> order(n);
  for (int f = 0; f < n; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (long long)b->fields[x].n1 * b->fields[x].nd > (long long)b->fields[y].n1 * b->fields[y].nd;
  });
  std::vector<std::vector<int>> xf(grf::XCD_QUEUES);
  std::vector<long long> load(grf::XCD_QUEUES, 0);
  for (int f : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    xf[x].push_back(f);
    load[x] += (long long)b->fields[f].n1 * b->fields[f].nd;
  }
  std::vector<BatchItem> items;
  std::vector<int> qoff(grf::XCD_QUEUES + 1, 0);
  auto cols = [&](const std::vector<int>& g) {
    std::vector<BatchItem> v;
    for (int f : g)
      for (int t = 0; t < b->fields[f].ntile; ++t) v.push_back({f, t});
    return v;
  };
  auto rows = [&](const std::vector<int>& g) {
    std::vector<BatchItem> v;
    for (int f : g) {
      const int rb = grf::batch_row_rb(b->fields[f].M, b->fields[f].rvar);
      const int nrb = (b->fields[f].n1 + rb - 1) / rb;
      for (int k = 0; k < nrb; ++k) v.push_back({f, -k - 1});
    }
    return v;
  };
  // the column items of one group and the row items of the group before,
  // merged in proportion to their counts (each list keeps its order), so that
  // at any time some workgroups generate (VALU) while others transform rows
  // (memory)
  auto merge = [&](const std::vector<BatchItem>& c, const std::vector<BatchItem>& r) {
    const size_t nc = c.size(), nr = r.size();
    size_t i = 0, j = 0;
    while (i < nc || j < nr) {
      if (j >= nr || (i < nc && i * nr <= j * nc)) items.push_back(c[i++]);
      else items.push_back(r[j++]);
    }
  };
  for (int x = 0; x < grf::XCD_QUEUES; ++x) {
    std::vector<std::vector<int>> groups;
    long long acc = 0;
    for (int f : xf[x]) {
      const long long bytes = (long long)b->fields[f].n1 * b->fields[f].nd * 4;
      if (groups.empty() || (acc + bytes > b->group_bytes && acc > 0)) {
        groups.emplace_back();
        acc = 0;
      }
      groups.back().push_back(f);
      acc += bytes;
    }
    for (size_t g = 0; g < groups.size(); ++g) merge(cols(groups[g]), g >= 1 ? rows(groups[g - 1]) : std::vector<BatchItem>());
    if (!groups.empty()) merge(std::vector<BatchItem>(), rows(groups.back()));
    qoff[x + 1] = (int)items.size();
  }
  if (b->d_one_items) (void)hipFree(b->d_one_items);
  b->d_one_items = nullptr;
  hipError_t e = hipMalloc((void**)&b->d_one_items, std::max<size_t>(1, items.size()) * sizeof(BatchItem));
  if (e != hipSuccess) return fail(GRF_ENOMEM, "hipMalloc of work queues failed");
  e = hipMemcpy(b->d_one_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_one_qoff, qoff.data(), qoff.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch upload");
  return GRF_OK;
}

// (Re)build field records and work queues for the current variants; upload.
grf_status build_queues(grf_batch_s* b) {
  const int n = (int)b->desc.size();
  if (b->one) {
    for (int f = 0; f < n; ++f) {
      BatchField& r = b->fields[f];
      r.cvar = b->cvar[r.n1];
      r.rvar = b->rvar[r.M];
      const int cp = grf::batch_one_cp(r.n1, r.cvar);
      r.ntile = (r.M + 2 * cp - 1) / (2 * cp);
    }
    grf_status st = build_one_queues(b);
    if (st != GRF_OK) return st;
    hipError_t e =
        hipMemcpy(b->d_fields, b->fields.data(), b->fields.size() * sizeof(BatchField), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    free_graph(b);
    return GRF_OK;
  }
  std::vector<WItem> row;
  std::vector<std::array<long long, 3>> cf;
  for (int f = 0; f < n; ++f) {
    BatchField& r = b->fields[f];
    // the two kernels have the plan path's radix order only: the tile shape of
    // a one-launch variant
    r.cvar = b->cvar[r.n1] % grf::BATCH_VARIANTS;
    r.rvar = b->rvar[r.M] % grf::BATCH_VARIANTS;
    const int cp = grf::batch_col_cp(r.n1, r.cvar);
    const int rb = grf::batch_row_rb(r.M, r.rvar);
    r.ntile = (r.M + 2 * cp - 1) / (2 * cp);
    cf.push_back({f, r.ntile, (long long)r.ntile * r.n1 * 2 * cp});
    const int nrb = (r.n1 + rb - 1) / rb;
    for (int k = 0; k < nrb; ++k) row.push_back({{f, k}, (long long)r.M * 2 * rb});
  }
  auto by_cost = [](const WItem& x, const WItem& y) {
    if (x.cost != y.cost) return x.cost > y.cost;
    if (x.it.field != y.it.field) return x.it.field < y.it.field;
    return x.it.sub < y.it.sub;
  };
  std::stable_sort(row.begin(), row.end(), by_cost);
  std::vector<BatchItem> hc, hr(row.size());
  std::vector<int> qoff;
  col_queues(cf, hc, qoff);
  for (size_t i = 0; i < row.size(); ++i) hr[i] = row[i].it;
  if (b->d_col) (void)hipFree(b->d_col);
  if (b->d_row) (void)hipFree(b->d_row);
  b->d_col = nullptr;
  b->d_row = nullptr;
  b->ncol = (int)hc.size();
  b->nrow = (int)hr.size();
  hipError_t e = hipMalloc((void**)&b->d_col, std::max<size_t>(1, hc.size()) * sizeof(BatchItem));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_row, std::max<size_t>(1, hr.size()) * sizeof(BatchItem));
  if (e != hipSuccess) return fail(GRF_ENOMEM, "hipMalloc of work queues failed");
  e = hipMemcpy(b->d_col, hc.data(), hc.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_qoff, qoff.data(), qoff.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_row, hr.data(), hr.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_fields, b->fields.data(), b->fields.size() * sizeof(BatchField), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch upload");
  free_graph(b);
  return GRF_OK;
}

grf_status enqueue(grf_batch_s* b, void* out, hipStream_t s) {
  if (b->one) {
    hipError_t e = grf::launch_reset_counters(b->d_one_state, ONE_STATE_DONE + (int)b->fields.size(), s);
    if (e == hipSuccess)
      e = grf::launch_batch_one(b->d_fields, b->d_one_items, b->d_one_qoff, b->d_tw, (float*)out, b->d_one_state,
                                b->d_one_state + ONE_STATE_DONE, b->d_one_state + grf::XCD_QUEUES, b->nwg_one, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return GRF_OK;
  }
  hipError_t e = grf::launch_reset_counters(b->d_counters, grf::BATCH_COUNTERS, s);
  if (e == hipSuccess)
    e = grf::launch_batch_col(b->d_fields, b->d_col, b->d_qoff, b->d_tw, (float*)out, b->d_counters, b->nwg_col, s);
  if (e == hipSuccess)
    e = grf::launch_batch_row(b->d_fields, b->d_row, b->nrow, b->d_tw, (float*)out,
                              b->d_counters + grf::XCD_QUEUES, b->nwg_row, s);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  return GRF_OK;
}

// Tile-shape choices from the tuning cache (lines "batch <arch> f32 col|row
// inv <length> <variant>"); foreign, corrupt or out-of-range entries are
// ignored.
void load_cache(grf_batch_s* b) {
  for (const grf::tune::Line& l : grf::tune::read("batch", grf::tune::arch_name(b->device))) {
    if (l.dtype != "f32" || l.dir != "inv") continue;
    char* end = nullptr;
    const long v = std::strtol(l.choice[0].c_str(), &end, 10);
    if (end == l.choice[0].c_str() || *end != '\0' || v < 0 || v >= grf::BATCH_ONE_VARIANTS) continue;
    if (l.pass == "col" && b->cvar.count((int)l.length)) b->cvar[(int)l.length] = (int)v;
    if (l.pass == "row" && b->rvar.count((int)l.length)) b->rvar[(int)l.length] = (int)v;
  }
  for (const grf::tune::Line& l : grf::tune::read("batch", grf::tune::arch_name(b->device))) {
    if (l.dtype != "f32" || l.pass != "group" || l.dir != "inv" || l.length != 1) continue;
    char* end = nullptr;
    const long long v = std::strtoll(l.choice[0].c_str(), &end, 10);
    if (end != l.choice[0].c_str() && *end == '\0' && v >= (1 << 20)) b->group_bytes = v;
  }
}

}  // namespace

extern "C" {

grf_status grf_batch_create(const grf_field_desc* fields, int64_t nfields, grf_batch* out) {
  if (fields == nullptr || out == nullptr) return fail(GRF_EINVAL, "null argument");
  *out = nullptr;
  if (nfields <= 0 || nfields > (1 << 24)) return fail(GRF_EINVAL, "nfields out of range");
  for (int64_t f = 0; f < nfields; ++f) {
    const grf_field_desc& d = fields[f];
    for (int i = 0; i < 2; ++i) {
      if (d.dims[i] <= 0 || d.dims[i] % 2) return fail(GRF_EINVAL, "grid sizes must be positive and even");
      if (!grf::host::smooth235(d.dims[i])) return fail(GRF_EINVAL, "grid sizes must factor into 2, 3 and 5");
      if (!(d.lengths[i] > 0) || !std::isfinite(d.lengths[i])) return fail(GRF_EINVAL, "edge lengths must be > 0");
    }
    if (d.cov_kind < GRF_COV_GAUSSIAN || d.cov_kind > GRF_COV_EXPONENTIAL)
      return fail(GRF_EINVAL, "unknown covariance kind");
    grf::FieldRec rec;
    if (grf::make_field_rec(d.cov_kind, 2, d.lengths[0] * d.lengths[1], d.sigma, d.length_scale, d.nu, &rec) != 0)
      return fail(GRF_EINVAL, "invalid covariance parameters");
    if (!grf::batch_col_supported((int)d.dims[0]) || d.dims[1] > 1024 ||
        !grf::batch_row_supported((int)(d.dims[1] / 2)))
      return fail(GRF_EUNSUPPORTED, "grid length not in the batch lists");
  }
  grf_batch_s* b = new (std::nothrow) grf_batch_s();
  if (b == nullptr) return fail(GRF_ENOMEM, "host allocation failed");
  b->desc.assign(fields, fields + nfields);
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDevice");
  }
  // twiddle pool: every distinct length once
  std::vector<int> lens;
  for (const auto& d : b->desc) {
    lens.push_back((int)d.dims[0]);
    lens.push_back((int)d.dims[1]);
    b->cvar[(int)d.dims[0]] = 0;
    b->rvar[(int)(d.dims[1] / 2)] = 0;
  }
  std::sort(lens.begin(), lens.end());
  lens.erase(std::unique(lens.begin(), lens.end()), lens.end());
  std::vector<float> pool;
  for (int L : lens) {
    b->twoff[L] = (int)(pool.size() / 2);
    std::vector<double> w;
    grf::host::table_values(L, w);
    pool.insert(pool.end(), w.begin(), w.end());
  }
  b->offsets.resize(nfields + 1);
  b->offsets[0] = 0;
  b->fields.resize(nfields);
  for (int64_t f = 0; f < nfields; ++f) {
    const grf_field_desc& d = b->desc[f];
    BatchField& r = b->fields[f];
    std::memset(&r, 0, sizeof(r));
    r.out_off = b->offsets[f];
    r.seed = d.seed;
    r.n1 = (int)d.dims[0];
    r.nd = (int)d.dims[1];
    r.M = r.nd / 2;
    r.tw1 = b->twoff[r.n1];
    r.twd = b->twoff[r.nd];
    r.il2[0] = 1.0 / (d.lengths[0] * d.lengths[0]);
    r.il2[1] = 0.0;
    r.il2[2] = 1.0 / (d.lengths[1] * d.lengths[1]);
    grf::make_field_rec(d.cov_kind, 2, d.lengths[0] * d.lengths[1], d.sigma, d.length_scale, d.nu, &r.rec);
    b->offsets[f + 1] = b->offsets[f] + d.dims[0] * d.dims[1];
  }
  load_cache(b);
  grf_status st = GRF_OK;
  e = hipMalloc(&b->d_tw, pool.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(b->d_tw, pool.data(), pool.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_fields, b->fields.size() * sizeof(BatchField));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_counters, grf::BATCH_COUNTERS * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_qoff, (grf::XCD_QUEUES + 1) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_one_qoff, (grf::XCD_QUEUES + 1) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_one_state, (ONE_STATE_DONE + nfields) * sizeof(int));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) st = hip_fail(e, "batch allocation");
  if (st == GRF_OK) {
    // persistent grids: every workgroup slot of the device once
    int ncu = 0, occ_c = 0, occ_r = 0, occ_o = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_c, grf::k_batch_col_ptr(),
                                                       grf::BATCH_COL_THREADS, 0);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_r, grf::k_batch_row_ptr(),
                                                       grf::BATCH_ROW_THREADS, 0);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_o, grf::k_batch_one_ptr(),
                                                       grf::BATCH_ONE_THREADS, 0);
    if (e != hipSuccess) st = hip_fail(e, "occupancy query");
    b->nwg_col = std::max(1, ncu * std::max(1, occ_c));
    b->nwg_row = std::max(1, ncu * std::max(1, occ_r));
    b->nwg_one = std::max(1, ncu * std::max(1, occ_o));
    // The one-launch kernel takes each workgroup's queue from its XCD: use it
    // only when a launch of that grid meets all XCD_QUEUES XCDs (else, or with
    // GRF_BATCH_LAUNCHES=2, the column and row passes run as two launches).
    const char* lm = std::getenv("GRF_BATCH_LAUNCHES");
    if (st == GRF_OK && !(lm && lm[0] == '2')) {
      int mask = 0;
      e = grf::launch_xcc_seen(b->d_one_state, b->nwg_one, nullptr);
      if (e == hipSuccess) e = hipMemcpy(&mask, b->d_one_state, sizeof(int), hipMemcpyDeviceToHost);
      if (e != hipSuccess) st = hip_fail(e, "XCD probe");
      b->one = mask == (1 << grf::XCD_QUEUES) - 1;
    }
  }
  if (st == GRF_OK) st = build_queues(b);
  if (st != GRF_OK) {
    grf_batch_destroy(b);
    return st;
  }
  *out = b;
  return GRF_OK;
}

grf_status grf_batch_offsets(grf_batch b, int64_t* offsets) {
  if (b == nullptr || offsets == nullptr) return fail(GRF_EINVAL, "null argument");
  for (size_t i = 0; i < b->offsets.size(); ++i) offsets[i] = b->offsets[i];
  return GRF_OK;
}

grf_status grf_batch_sample(grf_batch b, void* out, void* stream) {
  if (b == nullptr || out == nullptr) return fail(GRF_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  if (b->exec == nullptr || b->graph_out != out) {
    free_graph(b);
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    grf_status st = enqueue(b, out, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (st != GRF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      free_graph(b);
      return hip_fail(e, "graph instantiation");
    }
    b->graph_out = out;
  }
  hipError_t e = hipGraphLaunch(b->exec, s);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return GRF_OK;
}

grf_status grf_batch_sample_plain(grf_batch b, void* out, void* stream) {
  if (b == nullptr || out == nullptr) return fail(GRF_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  for (size_t f = 0; f < b->fields.size(); ++f) {
    const BatchField& r = b->fields[f];
    grf::Args a;
    std::memset(&a, 0, sizeof(a));
    a.data = (float*)out + r.out_off;
    a.recs = &b->d_fields[f].rec;
    a.tw = (const float*)b->d_tw + 2 * (size_t)r.tw1;
    a.tw2 = (const float*)b->d_tw + 2 * (size_t)r.twd;
    a.seed = r.seed;
    a.field_stride = (long long)r.n1 * r.M;
    a.stride_ax = r.M;
    a.stride_fixed = r.M;
    a.rows = r.n1;
    a.il2[0] = r.il2[0];
    a.il2[2] = r.il2[2];
    a.scale = 1.0;
    a.batch = 1;
    a.n1 = r.n1;
    a.no = 1;
    a.nd = r.nd;
    a.M = r.M;
    a.nfixed = 1;
    a.rows_per_field = r.n1;
    a.tag = 1;
    const grf::Geom gc = grf::pass_geom(grf::PASS_COL_GEN_INV, 0, r.n1);
    const grf::Geom gr = grf::pass_geom(grf::PASS_ROW_C2R, 0, r.M);
    a.ntile = (r.M + 2 * gc.per_wg - 1) / (2 * gc.per_wg);
    hipError_t e = grf::launch_pass(grf::PASS_COL_GEN_INV, 0, r.n1, a, a.ntile, s);
    if (e == hipSuccess) e = grf::launch_pass(grf::PASS_ROW_C2R, 0, r.M, a, (r.n1 + gr.per_wg - 1) / gr.per_wg, s);
    if (e != hipSuccess) return hip_fail(e, "plain batch launch");
  }
  return GRF_OK;
}

}  // extern "C"

namespace {

// Tuner of the one-launch mode: coordinate descent over the variant (radix
// order, i.e. threads per transform, and tile shape) of each column length
// and of each row length and over the pipeline group size, each setting timed
// on the whole batch (best of three after a warm-up).
grf_status tune_one(grf_batch_s* b, void* out, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  auto time_all = [&](float* ms) -> grf_status {
    grf_status st = build_queues(b);
    if (st != GRF_OK) return st;
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      hipError_t e = hipEventRecord(e0, s);
      if (e != hipSuccess) return hip_fail(e, "tuning run");
      st = enqueue(b, out, s);
      if (st != GRF_OK) return st;
      e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e != hipSuccess) return hip_fail(e, "tuning run");
      if (rep > 0) best = std::min(best, t);
    }
    *ms = best;
    return GRF_OK;
  };
  const std::string arch = grf::tune::arch_name(b->device);
  std::string lines;
  for (int pass = 0; pass < 2; ++pass) {
    auto& vm = pass == 0 ? b->cvar : b->rvar;
    for (auto& kv : std::map<int, int>(vm)) {
      float tv[grf::BATCH_ONE_VARIANTS];
      for (int v = 0; v < grf::BATCH_ONE_VARIANTS; ++v) {
        vm[kv.first] = v;
        grf_status st = time_all(&tv[v]);
        if (st != GRF_OK) return st;
      }
      int bv = 0;
      for (int v = 1; v < grf::BATCH_ONE_VARIANTS; ++v)
        if (tv[v] < tv[bv]) bv = v;
      vm[kv.first] = bv;
      char buf[128];
      std::snprintf(buf, sizeof(buf), "batch %s f32 %s inv %d %d\n", arch.c_str(), pass == 0 ? "col" : "row",
                    kv.first, bv);
      lines += buf;
    }
  }
  const long long groups[] = {8ll << 20, 16ll << 20, 24ll << 20, 48ll << 20, 1ll << 40};
  float bt = 1e30f;
  long long bg = b->group_bytes;
  for (long long g : groups) {
    b->group_bytes = g;
    float t = 0.0f;
    grf_status st = time_all(&t);
    if (st != GRF_OK) return st;
    if (t < bt) {
      bt = t;
      bg = g;
    }
  }
  b->group_bytes = bg;
  lines += "batch " + arch + " f32 group inv 1 " + std::to_string(bg) + "\n";
  grf_status st = build_queues(b);
  if (st != GRF_OK) return st;
  grf::tune::append(lines);
  return GRF_OK;
}

}  // namespace

extern "C" {

grf_status grf_batch_tune(grf_batch b, void* out, void* stream) {
  if (b == nullptr || out == nullptr) return fail(GRF_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(GRF_EDEVICE, "event creation");
  if (b->one) {
    const grf_status st = tune_one(b, out, s, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
  }
  // time one pass of the batch restricted to the fields of one length, per variant
  auto time_pass = [&](bool colpass, int len, int var, float* ms) -> grf_status {
    auto& vm = colpass ? b->cvar : b->rvar;
    const std::map<int, int> saved = vm;
    vm[len] = var;
    grf_status st = build_queues(b);
    if (st != GRF_OK) return st;
    // work items of this length only (column items in their XCD queues)
    std::vector<BatchItem> items;
    std::vector<std::array<long long, 3>> cf;
    for (size_t f = 0; f < b->fields.size(); ++f) {
      const BatchField& r = b->fields[f];
      if ((colpass ? r.n1 : r.M) != len) continue;
      const int per = colpass ? grf::batch_col_cp(len, var) : grf::batch_row_rb(len, var);
      const int nsub = colpass ? (r.M + 2 * per - 1) / (2 * per) : (r.n1 + per - 1) / per;
      if (colpass)
        cf.push_back({(long long)f, nsub, (long long)nsub * r.n1 * 2 * per});
      else
        for (int k = 0; k < nsub; ++k) items.push_back({(int)f, k});
    }
    std::vector<int> qoff;
    if (colpass) col_queues(cf, items, qoff);
    BatchItem* d_items = nullptr;
    int* d_q = nullptr;
    hipError_t e = hipMalloc((void**)&d_items, std::max<size_t>(1, items.size()) * sizeof(BatchItem));
    if (e == hipSuccess) e = hipMalloc((void**)&d_q, (grf::XCD_QUEUES + 1) * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
    if (e == hipSuccess && colpass) e = hipMemcpy(d_q, qoff.data(), qoff.size() * sizeof(int), hipMemcpyHostToDevice);
    float best = 1e30f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      e = grf::launch_reset_counters(b->d_counters, grf::BATCH_COUNTERS, s);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        e = colpass ? grf::launch_batch_col(b->d_fields, d_items, d_q, b->d_tw, (float*)out, b->d_counters,
                                            b->nwg_col, s)
                    : grf::launch_batch_row(b->d_fields, d_items, (int)items.size(), b->d_tw, (float*)out,
                                            b->d_counters + grf::XCD_QUEUES, b->nwg_row, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (rep > 0) best = std::min(best, t);   // first run warms up
    }
    if (d_items) (void)hipFree(d_items);
    if (d_q) (void)hipFree(d_q);
    vm = saved;
    if (e != hipSuccess) return hip_fail(e, "tuning run");
    *ms = best;
    return GRF_OK;
  };
  grf_status st = GRF_OK;
  std::string lines;
  const std::string arch = grf::tune::arch_name(b->device);
  for (int pass = 0; pass < 2 && st == GRF_OK; ++pass) {
    auto& vm = pass == 0 ? b->cvar : b->rvar;
    for (auto& kv : std::map<int, int>(vm)) {
      float tv[grf::BATCH_VARIANTS];
      for (int v = 0; v < grf::BATCH_VARIANTS && st == GRF_OK; ++v) st = time_pass(pass == 0, kv.first, v, &tv[v]);
      if (st != GRF_OK) break;
      int bv = 0;
      for (int v = 1; v < grf::BATCH_VARIANTS; ++v)
        if (tv[v] < tv[bv]) bv = v;
      vm[kv.first] = bv;
      char buf[128];
      std::snprintf(buf, sizeof(buf), "batch %s f32 %s inv %d %d\n", arch.c_str(), pass == 0 ? "col" : "row",
                    kv.first, bv);
      lines += buf;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GRF_OK) return st;
  st = build_queues(b);
  if (st != GRF_OK) return st;
  grf::tune::append(lines);
  return GRF_OK;
}

grf_status grf_batch_info(grf_batch b, int32_t* launches, int32_t* wait_errors) {
  if (b == nullptr) return fail(GRF_EINVAL, "null argument");
  if (launches) *launches = b->one ? 1 : 2;
  if (wait_errors) {
    int v = 0;
    if (b->one) {
      hipError_t e = hipMemcpy(&v, b->d_one_state + grf::XCD_QUEUES, sizeof(int), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "batch state read");
    }
    *wait_errors = v;
  }
  return GRF_OK;
}

grf_status grf_batch_destroy(grf_batch b) {
  if (b == nullptr) return GRF_OK;
  free_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_fields) (void)hipFree(b->d_fields);
  if (b->d_col) (void)hipFree(b->d_col);
  if (b->d_row) (void)hipFree(b->d_row);
  if (b->d_qoff) (void)hipFree(b->d_qoff);
  if (b->d_tw) (void)hipFree(b->d_tw);
  if (b->d_counters) (void)hipFree(b->d_counters);
  if (b->d_one_items) (void)hipFree(b->d_one_items);
  if (b->d_one_qoff) (void)hipFree(b->d_one_qoff);
  if (b->d_one_state) (void)hipFree(b->d_one_state);
  delete b;
  return GRF_OK;
}

}  // extern "C"
