/*
 * grf.h -- C ABI of the MI355X (gfx950) Gaussian random field sampler.
 *
 * Implements the FFT-based sampling of centred stationary Gaussian random
 * fields on a periodic rectangular grid of Lang & Potthoff, "Fast simulation
 * of Gaussian random fields" (arXiv 1105.2737), Section 3:
 *   - the two-FFT algorithm (white noise, forward FFT, multiplication by
 *     gamma^{1/2} |D|^{-1}, inverse FFT), from eq. (1);
 *   - the one-FFT algorithm (Hermitian-symmetric complex noise drawn directly
 *     in Fourier space through the paper's data arrangement, rules a-e of
 *     Section 2 and eq. (3), then one inverse FFT), from eq. (2) and Lemma 1;
 * plus the adjoint of the one-FFT sampler (gradients of a loss with respect to
 * the covariance parameters and the noise).
 *
 * Problem statement (the algorithms' Input/Output lists): a region D with edge
 * lengths l_i, grid sizes N_i (all even), the square root of a symmetric
 * positive spectral density gamma, and a generator of independent normals;
 * output a real field B on the grid whose covariance is the Fourier transform
 * of gamma.
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - spectral density S in cycles: C(x) = int S(p) exp(-2 pi i p.x) dp
 *     (Section 2); frequency of index k along axis i: p = kappa(k)/l_i with
 *     kappa(k) = k for k < N_i/2 and k - N_i otherwise;
 *   - output phi_j = sum_k A_k exp(+2 pi i k.j/N) with A_k = h_k xi_k,
 *     h_k = sqrt(S(p_k)/|D|), so Cov(phi_0, phi_j) = (1/|D|) sum_k S(p_k)
 *     exp(2 pi i k.j/N), the Riemann sum of the covariance integral;
 *   - noise: Philox-4x32-10 (Salmon et al., SC'11), key = seed + b for field b,
 *     counter (s div 4, row, tag, 0) for slot s of a row, Box-Muller normals;
 *     tag 0 = two-FFT white noise, tag 1 = one-FFT Fourier noise.  The noise
 *     z of a field is a real array with the field's shape; the one-FFT
 *     algorithm maps it bijectively onto the independent real and imaginary
 *     parts of the Hermitian half-spectrum.
 *
 * Memory: all data pointers are DEVICE pointers unless stated otherwise; the
 * caller owns them.  Fields are stored row-major [batch][N_1]...[N_d].  A plan
 * owns only small device tables (twiddles, default per-field constants).
 * Streams are hipStream_t passed as void* (NULL = default stream).  All work
 * is asynchronous on that stream; a device error surfaces as GRF_EDEVICE at
 * the launch or at a later call.  Every call validates its arguments on the
 * host before launching anything: on GRF_EINVAL nothing has been written.
 * Results are deterministic: the same plan, parameters and seed give the same
 * bits whatever the batch size or the field's position in the batch.
 * A plan may be used by one stream at a time.
 */
#ifndef GRF_H
#define GRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct grf_plan_s* grf_plan;

typedef enum {
  GRF_OK = 0,
  GRF_EINVAL = -1,       /* invalid argument (nothing written) */
  GRF_ENOMEM = -2,       /* device or host allocation failed */
  GRF_EDEVICE = -3,      /* HIP runtime error */
  GRF_EUNSUPPORTED = -4  /* valid request outside what the library implements */
} grf_status;

enum { GRF_ALG_TWO_FFT = 1, GRF_ALG_ONE_FFT = 2 };
enum { GRF_F32 = 0, GRF_F64 = 1 };
enum { GRF_COV_GAUSSIAN = 0, GRF_COV_MATERN = 1, GRF_COV_EXPONENTIAL = 2, GRF_COV_PAPER = 3, GRF_COV_TABULATED = 4 };
enum { GRF_OP_SAMPLE = 0, GRF_OP_BACKWARD = 1, GRF_OP_COVARIANCE = 2 };
enum { GRF_BC_PERIODIC = 0, GRF_BC_NEUMANN = 1, GRF_BC_DIRICHLET = 2 };
enum { GRF_DRAW_COUNTER = 0, GRF_DRAW_RECURSIVE = 1 };

/*
 * Plan description.
 *   ndim      1, 2 or 3 (the grid's dimension d).
 *   dims      N_1..N_d: each even and a product of 2, 3 and 5 (Section 2
 *             requires even N_i; the FFT factorisation needs the rest), leading
 *             lengths N_1 (and N_2 for d = 3) up to 4096, the last length N_d
 *             up to 16384 (GRF_EUNSUPPORTED above).  The listed lengths run on
 *             compile-time kernels tuned per length: leading lengths {4, 8, 12,
 *             16, 24, 32, 48, 64, 96, 128, 180, 256, 360, 384, 500, 512, 768,
 *             1000, 1024}, N_d/2 from {2, 4, 8, 12, 16, 24, 32, 48, 64, 96, 128,
 *             180, 192, 256, 360, 384, 500, 512, 1024, 2048}; every other length
 *             runs on runtime-radix kernels
 *             (sampling and grf_backward with either algorithm, d = 1, 2, 3).
 *             Reflecting boundaries and the recursive draw order take the
 *             listed lengths only (GRF_EUNSUPPORTED otherwise).
 *   lengths   l_1..l_d > 0 (edge lengths of D; the unit torus is all 1).
 *   alg       GRF_ALG_ONE_FFT or GRF_ALG_TWO_FFT (periodic boundaries, counter draw order).
 *   dtype     GRF_F32 (complex64 arithmetic, twiddles from float64) or GRF_F64.
 *   cov_kind  covariance family (S = the spectral density in cycles,
 *             C(x) = integral of S(p) exp(-2 pi i p.x) dp, Section 2):
 *               GAUSSIAN    C(r) = sigma^2 exp(-r^2 / (2 ell^2))
 *               MATERN      C(r) = sigma^2 2^{1-nu}/Gamma(nu) (sqrt(2nu) r/ell)^nu K_nu(sqrt(2nu) r/ell)
 *               EXPONENTIAL C(r) = sigma^2 exp(-r/ell)   (nu ignored)
 *               PAPER       S(p) = sigma^2 (m^{kl} + (sum_i p_i^{2k})^l)^{-n}, the family
 *                           of Section 4, eq. (5) (k, l, n >= 1, m > 0; any d)
 *               TABULATED   S given at the grid frequencies of the half-spectrum:
 *                           `spectrum` is a host float64 array [N_1]..[N_{d-1}][N_d/2 + 1]
 *                           (row-major; frequency index k_i stands for p_i = kappa(k_i)/l_i
 *                           with kappa(k) = k for k < N_i/2 and k - N_i otherwise), S >= 0,
 *                           equal on mirrored entries of the planes k_d = 0 and N_d/2
 *                           (S(p) = S(-p)); copied at plan creation; scaled by sigma^2.
 *             PAPER and TABULATED have no length scale or nu: their filter is a
 *             table built at plan creation, per-field theta is not accepted
 *             (GRF_EUNSUPPORTED), and the adjoint's d/d(ell, nu) are 0.
 *   sigma, length_scale, nu   default parameters (> 0).
 *   m, k, l, n   parameters of GRF_COV_PAPER (ignored otherwise).
 *   spectrum  GRF_COV_TABULATED only (NULL otherwise).
 *   bc        boundary condition of each axis i < ndim: GRF_BC_PERIODIC (0,
 *             the FFT algorithms of Section 3), or GRF_BC_NEUMANN (1) /
 *             GRF_BC_DIRICHLET (2), the cosine / sine transform variant that
 *             the introduction and Section 3 name for these boundaries.  Either
 *             every axis is periodic or none is (else GRF_EUNSUPPORTED); the
 *             reflecting variant needs alg = GRF_ALG_ONE_FFT (it has a single
 *             transform; GRF_EUNSUPPORTED otherwise).  Reflecting fields live
 *             on the cell centres x_j = (j + 1/2) l_i / N_i of [0, l_i] and are
 *             sums over slots n (same shape as the field) of a_n z_n times
 *             prod_i cos(pi n_i (j_i + 1/2) / N_i) on Neumann axes and
 *             sin(pi (N_i - n_i)(j_i + 1/2) / N_i) on Dirichlet axes, with
 *             frequency p_i = n_i / (2 l_i) resp. (N_i - n_i) / (2 l_i),
 *             a_n = sigma sqrt(S(p) prod_i c(n_i) / |D|), c(0) = 1, c(n >= 1) = 2,
 *             and z the Philox normals of tag 2 indexed by slot (the
 *             covariance is the method-of-images sum of the periodic one on
 *             the doubled grid).  TABULATED then gives S on the slot grid,
 *             [N_1]..[N_d] (field layout).
 *   draw_order GRF_DRAW_COUNTER (0): each normal of the one-FFT algorithm is
 *             addressed by its entry (tag 1), any order of work; or
 *             GRF_DRAW_RECURSIVE (1): the normals are the sequence R() of the
 *             recursive algorithm of Section 3 (exactly P draws per field),
 *             draw j being the value of the field-shaped tag-3 noise at
 *             row-major index j (grf_noise writes it; grf_sample_from_noise
 *             takes it), so a sequential implementation of that algorithm fed
 *             the same sequence gives the same field.  Order of the draws:
 *             the entries with 1 <= k_d < N_d/2 (row-major, k_d fastest; real
 *             then imaginary part), then the plane k_d = 0, then k_d = N_d/2,
 *             each by the same rule over the axes before d; on axis 1 the
 *             real entries k_1 = 0 and N_1/2 come last.  GRF_ALG_ONE_FFT with
 *             periodic axes only (else GRF_EUNSUPPORTED).
 */
typedef struct {
  int32_t ndim;
  int32_t alg;
  int32_t dtype;
  int32_t cov_kind;
  int64_t dims[3];
  double lengths[3];
  double sigma;
  double length_scale;
  double nu;
  double m;
  int32_t k, l, n;
  int32_t reserved;
  const double* spectrum;
  int32_t bc[3];
  int32_t draw_order;
} grf_plan_desc;

/* Create a plan: validates the description, builds float64 twiddle tables
 * (rounded once to the working precision) and the default per-field
 * constants.  *out receives a library-owned handle.  Errors: GRF_EINVAL (bad
 * description, null pointer), GRF_EUNSUPPORTED (a length above its limit,
 * reflecting boundaries or the recursive draw order with a length not in the
 * lists, two-FFT with reflecting boundaries or the recursive draw order),
 * GRF_ENOMEM, GRF_EDEVICE. */
grf_status grf_plan_create(const grf_plan_desc* desc, grf_plan* out);

/* Release a plan and its device tables (NULL is accepted). */
grf_status grf_plan_destroy(grf_plan plan);

/* Autotuner of a plan: for every pass of the sampler (the launch sequence
 * of a batch of `batch` fields), times the candidate kernels on one chunk
 * of fields in `out` (device, batch fields of the plan's shape; its contents
 * are overwritten) and keeps the fastest for later calls: the compile-time
 * kernel of a listed length, and the runtime-radix kernel with every radix
 * order the tuner generates for the length (the splits of its power of two
 * into radices 8, 4, 2 with its 3s and 5s, in several orders) at 4 and 8
 * values per thread.  Appends one line per pass to the file named by
 * GRF_TUNE_CACHE, if set:
 *   plan <arch> <f32|f64> <pass> <inv|fwd> <length> fixed | generic <vpt> <r1,r2,...>
 * and grf_plan_create reads that file: the last line for a key (arch, dtype,
 * pass, direction, length) that the plan uses and that names a kernel it can
 * run wins; other lines (other architectures, corrupt ones) are ignored.
 * Synchronises the stream.  Results stay within the tolerance of the oracle
 * whatever the choice (a different radix order rounds differently). */
grf_status grf_plan_tune(grf_plan plan, int64_t batch, void* out, void* stream);
/* The plan's current choice for pass `pass` (a GRF_PASS_* value) of transform
 * length `length` ("default", "fixed" or "generic <vpt> <radices>"), into the
 * host buffer buf of len bytes. */
grf_status grf_plan_tune_choice(grf_plan plan, int32_t pass, int64_t length, char* buf, size_t len);

/* Bytes of device workspace that grf_sample / grf_sample_from_noise
 * (op = GRF_OP_SAMPLE), grf_backward (op = GRF_OP_BACKWARD) or
 * grf_covariance (op = GRF_OP_COVARIANCE, batch = number of samples) need for
 * `batch` fields (host pointer `bytes`).  The sampler runs in place in the
 * output buffer; its workspace only holds per-field constants. */
grf_status grf_workspace_size(grf_plan plan, int64_t batch, int32_t op, size_t* bytes);

/* Sample fields seed, seed+1, ..., seed+batch-1 (Section 3: the plan's
 * algorithm).  out: device, batch * N_1 * ... * N_d elements of the plan's
 * dtype.  theta: NULL (use the plan's parameters) or a device array
 * [batch][3] of float64 (sigma, length_scale, nu) per field.  workspace: device,
 * at least grf_workspace_size(..., GRF_OP_SAMPLE) bytes (may be NULL if that
 * size is 0).  batch = 0 is a no-op. */
grf_status grf_sample(grf_plan plan, uint64_t seed, int64_t batch, const double* theta, void* out,
                      void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory during a call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * grf_sample without a workspace argument.  Per-field parameters (theta,
 * as in grf_sample) are turned into per-field constants in a library-owned
 * device array of GRF_NOALLOC_MAX_FIELDS records (6.5 MiB per device, held
 * from the first call on a device until the process ends); the call itself
 * allocates nothing.  theta != NULL with batch > GRF_NOALLOC_MAX_FIELDS is
 * rejected with GRF_EINVAL before any launch; theta == NULL uses no scratch
 * and has no limit.  Every call on a device shares that device's array and
 * rewrites the records it uses before reading them: calls that overlap on one
 * device (concurrent streams or host threads) race; serialise them.  Output
 * is bitwise that of grf_sample with the same arguments. */
#define GRF_NOALLOC_MAX_FIELDS 65536
grf_status grf_sample_noalloc(grf_plan plan, uint64_t seed, int64_t batch, const double* theta, void* out,
                              void* stream);

/* As grf_sample, but the normals z are read from `noise` (device, same
 * shape and dtype as the output) instead of being generated. */
grf_status grf_sample_from_noise(grf_plan plan, const void* noise, int64_t batch, const double* theta,
                                 void* out, void* workspace, size_t workspace_bytes, void* stream);

/* Measurement support.  grf_sample runs its passes chunk by chunk: the batch
 * is cut into chunks of fields sized to the device's 256 MB last-level cache
 * (the environment variable GRF_CHUNK_BYTES sets another size), and every
 * pass of a chunk runs before the next chunk, so that a pass reads what the
 * previous one wrote from that cache.  Passes of a chunk: one-FFT d = 2:
 * column generation + inverse transform, then last-axis complex-to-real;
 * d = 3 adds the middle-axis inverse transform; two-FFT, d = 2: last-axis
 * noise + real-to-complex, column forward/filter/inverse, last-axis
 * complex-to-real; d = 1 (both algorithms): one launch over whole fields
 * (GRF_PASS_ROW_GEN_C2R); two-FFT, d = 3: last-axis noise +
 * real-to-complex, forward transform along the middle axis, the column pass
 * of axis 1 (forward, filter, inverse) for every slot but the packed plane
 * slot, then for that slot alone forward along axis 1, its filter and the
 * inverse (three small launches), the middle-axis inverse transform and the
 * last-axis complex-to-real; the axis-1 column pass and the plane-slot filter
 * report the internal kinds 109 and 110.  One-FFT, d = 2, on the 512 x 512
 * grid: the column pass stops before the last radix stage of
 * its transform (internal kind 111; 113 in the recursive draw order) and the
 * last-axis pass runs that stage before the complex-to-real (112), with the
 * same bits as the two passes above (the environment variable GRF_SPLIT=0
 * selects those instead).
 * grf_sample_stage_count returns the number of launches for a batch of
 * `batch` fields (host pointer); grf_sample_stage runs only launch `stage`
 * (0-based) with the arguments of grf_sample, so that each kernel can be
 * timed on its own.  Run alone, a later stage transforms whatever `out`
 * holds.  grf_sample_stage_info reports, for launch `stage` of a batch of
 * `batch` fields, the pass it runs (*kind, one of GRF_PASS_*) and the fields
 * first .. first + count - 1 it covers; host pointers, any may be NULL. */
enum {
  GRF_PASS_COL_GEN_INV = 0,   /* noise + filter + inverse transform along axis 1 (one-FFT) */
  GRF_PASS_COL_LOAD_INV = 1,  /* inverse transform along the middle axis (d = 3) */
  GRF_PASS_COL_LOAD_FWD = 2,  /* forward transform along the middle axis */
  GRF_PASS_COL_FILTER = 3,    /* forward transform, filter, inverse transform along axis 1 (two-FFT) */
  GRF_PASS_COL_GRAD = 4,      /* forward transform and adjoint reduction along axis 1 */
  GRF_PASS_ROW_C2R = 5,       /* last-axis complex-to-real inverse transform */
  GRF_PASS_ROW_R2C_GEN = 6,   /* last-axis white noise + real-to-complex forward transform (two-FFT) */
  GRF_PASS_ROW_R2C_LOAD = 7,  /* last-axis real-to-complex forward transform of stored rows */
  GRF_PASS_ROW_GEN_C2R = 8,   /* d = 1: noise (+ forward transform, two-FFT) + filter + complex-to-real, whole fields */
  GRF_PASS_R2R_COL_GEN = 9,   /* reflecting boundaries: coefficients + cosine transform along axis 1 */
  GRF_PASS_R2R_COL_LOAD = 10, /* reflecting boundaries: cosine transform along the middle axis (d = 3) */
  GRF_PASS_R2R_ROW_LOAD = 11, /* reflecting boundaries: cosine transform along the last axis */
  GRF_PASS_R2R_ROW_GEN = 12,  /* reflecting boundaries, d = 1: coefficients + cosine transform of whole fields */
  GRF_PASS_COL_SEQ_INV = 13,  /* as GRF_PASS_COL_GEN_INV, normals in the recursive algorithm's draw order */
  GRF_PASS_SPEC_FILTER = 14   /* two-FFT: filter on the packed spectrum after the forward transforms (not in the sampler's sequences) */
};
grf_status grf_sample_stage_count(grf_plan plan, int64_t batch, int32_t* count);
grf_status grf_sample_stage(grf_plan plan, int32_t stage, uint64_t seed, int64_t batch, const double* theta,
                            void* out, void* workspace, size_t workspace_bytes, void* stream);
grf_status grf_sample_stage_info(grf_plan plan, int64_t batch, int32_t stage, int32_t* kind, int64_t* first,
                                 int64_t* count);

/* Statistical covariance of the sampler, the estimator of Section 4:
 *   cov[j] = (1/nsamples) sum_{b < nsamples} phi_b(x_0) phi_b(x_j)
 * for every grid point x_j, where phi_b is field seed+b exactly as grf_sample
 * returns it with the plan's parameters (x_0 is the grid's first point).  cov:
 * device, float64, one value per grid point (the field's shape).  d = 1
 * accumulates in the sampler's last pass (the fields are never written); d = 2
 * and 3 sample cache-sized chunks of fields into the workspace and
 * accumulate them.  The sums are taken in a fixed order (float64), so the
 * result does not depend on scheduling.  workspace: device, at least
 * grf_workspace_size(plan, nsamples, GRF_OP_COVARIANCE) bytes.  Errors:
 * GRF_EINVAL (null pointer, nsamples < 1, workspace too small). */
grf_status grf_covariance(grf_plan plan, uint64_t seed, int64_t nsamples, double* cov, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Write the noise z of the contract for fields seed..seed+batch-1 (device,
 * same shape and dtype as the output; tag 0 two-FFT, 1 one-FFT, 2 reflecting
 * boundaries, where z is indexed by slot, 3 the recursive draw order, where
 * z in row-major order is the sequence of draws). */
grf_status grf_noise(grf_plan plan, uint64_t seed, int64_t batch, void* noise_out, void* stream);

/* Adjoint of the one-FFT sampler.  Given the upstream gradient
 * grad_out = dL/dphi (device, field-shaped, plan dtype), computes
 *   grad_theta[b] = dL/d(sigma, length_scale, nu) of field b (device float64
 *                   [batch][3]; the derivative for a parameter the family does
 *                   not have is 0), and
 *   grad_noise    = dL/dz (device, field-shaped; NULL to skip).
 * The noise is regenerated from `seed` (noise == NULL) or read from `noise`.
 * The Fourier transform of grad_out is recomputed; no spectrum is stored by
 * the forward call.  Both algorithms, the
 * reflecting boundaries (B^T g by the transposed cosine transforms) and both
 * draw orders (in the recursive one dL/dz is indexed like the sequence of
 * draws); ndim = 1, 2 or 3.
 * For the two-FFT algorithm xi = F[z] / sqrt(P) enters in place of the
 * Hermitian noise, and dL/dz = F*[h F[grad_out]] / sqrt(P), the sampler
 * applied to grad_out.  At a grid length outside the compiled lists the
 * one-FFT reduction reads G = F[grad_out], transformed along every axis by the
 * runtime-radix passes, back from the workspace (one more pass over the
 * spectrum than the fused column kernel of a listed length). */
grf_status grf_backward(grf_plan plan, uint64_t seed, const void* noise, int64_t batch, const double* theta,
                        const void* grad_out, double* grad_theta, void* grad_noise, void* workspace,
                        size_t workspace_bytes, void* stream);

/* ---- Batches of fields with different sizes and parameters --------------
 * d = 2, one-FFT algorithm, float32.  Every field has its own grid, edge
 * lengths, covariance parameters and seed.  grf_batch_sample runs the whole
 * batch as one persistent launch (per-XCD queues of column-generation items
 * and last-axis items, a last-axis item waiting on its field's readiness
 * counter) or, where one launch cannot reach all 8 XCDs, as two (column
 * generation of every field, then the last-axis pass of every field), each
 * workgroup taking work items from an atomic queue in decreasing order of
 * cost; the launches are captured once in a hipGraph and replayed
 * (grf_batch_info tells which).  Results are bit-identical to sampling each field
 * with its own plan.  N_1 must be one of {64, 96, 128, 180, 256, 360, 500, 512,
 * 1000, 1024} and N_2/2 one of {32, 48, 64, 96, 128, 180, 256, 360, 500, 512}. */
typedef struct grf_batch_s* grf_batch;

typedef struct {
  int64_t dims[2];      /* N_1, N_2 (even) */
  double lengths[2];    /* l_1, l_2 > 0 */
  int32_t cov_kind;     /* GRF_COV_* */
  int32_t reserved;
  double sigma, length_scale, nu;
  uint64_t seed;        /* Philox key of this field */
} grf_field_desc;

/* fields: host array of nfields descriptors (copied).  Allocates the device
 * tables of the batch (field records, work queues, twiddles).  Tile shapes come
 * from the autotune cache file named by GRF_TUNE_CACHE when it exists. */
grf_status grf_batch_create(const grf_field_desc* fields, int64_t nfields, grf_batch* out);
/* Output layout: field f occupies elements [offsets[f], offsets[f+1]) of the
 * output, row-major N_1 x N_2; offsets is a host array of nfields + 1. */
grf_status grf_batch_offsets(grf_batch b, int64_t* offsets);
/* Sample every field into out (device, offsets[nfields] float32 elements). */
grf_status grf_batch_sample(grf_batch b, void* out, void* stream);
/* The same fields, one plan-style launch pair per field (the baseline the
 * persistent launch is compared with). */
grf_status grf_batch_sample_plain(grf_batch b, void* out, void* stream);
/* Autotuner: for each column length and each row half-length present in the
 * batch, its variants (one-launch mode: two radix orders, i.e. two numbers of
 * threads per transform, times two tile shapes, variants 0-3; two-launch
 * mode: the two tile shapes of the plan path's radix order, variants 0-1),
 * and (one-launch mode) the pipeline group size of the XCD queues, each timed
 * on the whole batch (writing into out, which must hold the batch), keeping
 * the fastest; appends the choices to the GRF_TUNE_CACHE file if set (lines
 * "batch <arch> f32 col|row inv <length> <variant>" and "batch <arch> f32
 * group inv 1 <bytes>"; see grf_plan_tune for the cache rules).  A tile shape
 * leaves a field's bits unchanged; the other radix order changes them within
 * the oracle's float32 tolerance.  Synchronises the stream. */
grf_status grf_batch_tune(grf_batch b, void* out, void* stream);
/* How the batch runs: *launches = 1 (one persistent launch: per-XCD queues of
 * column and row items, each row item waiting for its field's column items
 * by a readiness counter; chosen at creation when a launch reaches all 8
 * XCDs) or 2 (a column and a row launch; GRF_BATCH_LAUNCHES=2 forces it);
 * *wait_errors = the number of row items of the last sample whose wait gave
 * up (0 unless the device misbehaves; their fields are then incomplete).
 * Synchronous; either pointer may be NULL. */
grf_status grf_batch_info(grf_batch b, int32_t* launches, int32_t* wait_errors);
grf_status grf_batch_destroy(grf_batch b);

/* Raw Philox-4x32-10 blocks: counters (device, n x 4 uint32) -> out (device,
 * n x 4 uint32) under key = seed.  For bit-exact checks of the generator. */
grf_status grf_debug_philox(uint64_t seed, const uint32_t* counters, int64_t n, uint32_t* out, void* stream);

/* The half-spectrum A_k = h_k xi_k that the one-FFT sampler hands to its
 * inverse transforms (Section 3, the second algorithm: the Hermitian
 * arrangement of the noise of fields seed .. seed+batch-1 times the filter
 * h_k = sqrt(S(p_k)/|D|) at the plan's parameters), computed by the
 * generating pass's own device code.  spec_out: device, batch * (P / N_d) *
 * (N_d / 2) complex values of the plan's dtype (interleaved re, im), laid out
 * [field][N_1 ... N_{d-1} row][m], m = 0 .. N_d/2 - 1, where slot m = 0 holds
 * A(k, 0) + i A(k, N_d/2) (both planes are Hermitian, so each is determined
 * by its real and imaginary parts over the rows k).  The entries with
 * 0 < m < N_d/2 are A(k, m) as they are.  For inspection and tests; the
 * sampler never stores this array.  Errors: GRF_EINVAL, GRF_EUNSUPPORTED (the
 * two-FFT algorithm, reflecting boundaries or the recursive draw order),
 * GRF_EDEVICE. */
grf_status grf_debug_spectrum(grf_plan plan, uint64_t seed, int64_t batch, void* spec_out, void* stream);

/* Human-readable message of the last error on the calling thread. */
const char* grf_last_error(void);

/* Library version string. */
const char* grf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRF_H */
