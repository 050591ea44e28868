// Batches of fields with different grid sizes and parameters (d = 2, one-FFT
// algorithm, float32), sampled by two persistent launches: every workgroup
// takes work items -- (field, column tile) for the column generation pass,
// (field, row block) for the last-axis pass -- from an atomic queue in
// decreasing order of cost and runs the kernel body of the field's length.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grf_common.hpp"

namespace grf {

// Device record of one field of a batch.
struct BatchField {
  long long out_off;          // offset of the field in the output (real elements)
  unsigned long long seed;    // Philox key of the field
  int n1, nd, M;              // N_1, N_2, N_2 / 2
  int cvar, rvar;             // tile-shape variants of the two passes
  int ntile;                  // column tiles of the field (for its variant)
  int tw1, twd;               // offsets of W_{N_1} and W_{N_2} in the twiddle pool (complex)
  int pad;
  double il2[3];
  FieldRec rec;
};

struct BatchItem {
  int field;
  int sub;                    // column tile, or row block; in the one-launch queues a row block b is -b - 1
};

constexpr int BATCH_COL_THREADS = 256;
constexpr int BATCH_ROW_THREADS = 512;
constexpr int BATCH_VARIANTS = 2;       // tile shapes of the two-launch kernels' bodies
// the one-launch kernel's bodies: variants 0, 1 as BATCH_VARIANTS; 2, 3 another
// radix order (threads per transform) with two tile shapes
constexpr int BATCH_ONE_VARIANTS = 4;
constexpr int XCD_QUEUES = 8;         // column work queues, one per XCD
constexpr int BATCH_COUNTERS = XCD_QUEUES + 1;   // column queues, then the row queue

// One persistent launch (k_batch_one): 512-thread workgroups run column and
// row items alike; each XCD has its own queue (producer and consumer of a
// field share one L2), and a row item waits for the field's column items by
// its readiness counter (a bounded wait: past BATCH_ONE_SPIN_LIMIT polls the
// item is skipped and the error word set, so every workgroup exits).
constexpr int BATCH_ONE_THREADS = 512;
constexpr int BATCH_ONE_SPIN_LIMIT = 1 << 22;

// Geometry of a variant: column pairs per column workgroup / rows per row
// workgroup (var < BATCH_VARIANTS; batch_row_rb and batch_one_cp also take
// the one-launch kernel's variants < BATCH_ONE_VARIANTS).
int batch_col_cp(int L, int var);
int batch_one_cp(int L, int var);   // column pairs per workgroup in the one-launch kernel
int batch_row_rb(int M, int var);
bool batch_col_supported(int L);
bool batch_row_supported(int M);

// One persistent launch (grid = nwg workgroups, a multiple of XCD_QUEUES for
// the XCD grouping to hold) over the column items in XCD_QUEUES queues
// (device offsets qoff[0..XCD_QUEUES], counters[0..XCD_QUEUES-1]) or over
// `nitems` row items.
hipError_t launch_batch_col(const BatchField* fields, const BatchItem* items, const int* qoff, const void* twpool,
                            float* out, int* counters, int nwg, hipStream_t s);
hipError_t launch_batch_row(const BatchField* fields, const BatchItem* items, int nitems, const void* twpool,
                            float* out, int* counter, int nwg, hipStream_t s);
hipError_t launch_reset_counters(int* counters, int n, hipStream_t s);
// The one-launch kernel over XCD_QUEUES queues (queue q: items[qoff[q] ..
// qoff[q+1]), counter counters[q]); done[f] counts the finished column items
// of field f; err is set if a wait gave up.  counters, done and err must be
// zero at launch (launch_reset_counters).
hipError_t launch_batch_one(const BatchField* fields, const BatchItem* items, const int* qoff, const void* twpool,
                            float* out, int* counters, int* done, int* err, int nwg, hipStream_t s);
const void* k_batch_one_ptr();
// Bit x of *mask set for every XCD x that a grid of nwg workgroups runs on
// (synchronous).
hipError_t launch_xcc_seen(int* mask, int nwg, hipStream_t s);
// The two persistent kernels (for occupancy queries).
const void* k_batch_col_ptr();
const void* k_batch_row_ptr();

}  // namespace grf
