/*
 * dedisp.h -- C-ABI of an MI355X (gfx950) library for brute-force incoherent
 * dedispersion.
 *
 * Method: Sclocco, van Leeuwen, Bal, van Nieuwpoort, "Real-Time Dedispersion
 * for Fast Radio Transient Surveys, using Auto Tuning on Many-Core
 * Accelerators" (arXiv 1601.01165).
 *
 *   out[b][dm][t] = sum over channels c, ascending, of w[c] * in[b][c][t + delta[dm][c]]
 *
 * (Section 2.1, Algorithm 1; the per-channel weight w is an extension, w == NULL
 * means all ones), with integer delays delta from the dispersion law of
 * Section 2, Equation 1:
 *
 *   k = 4150 * DM * (1/f_c^2 - 1/f_h^2) seconds  (f in MHz, f_h = highest channel)
 *   delta[dm][c] = floor(k / tsamp + 1/2)          (FP64, round half up)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns a dedisp_status and never aborts or throws.  On
 *    failure dedisp_last_error() returns a thread-local text with the detail.
 *  - Pointers named d_* are device pointers on the device that was current
 *    when the plan was created; pointers without the prefix are host pointers.
 *  - The caller owns every data buffer.  A plan owns its delay tables (host
 *    and device); a batch owns its work table and its graph.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  The
 *    execute, batched-execute and adjoint calls only enqueue work on that
 *    stream: they never allocate, never synchronise and return before the
 *    kernels finish.
 *  - Layouts (row-major, time contiguous):
 *      input      in  [nbeam][nchan][in_stride]
 *      output     out [nbeam][ndm][out_stride]
 *    with in_stride >= nsamp + max_delay and out_stride >= nsamp.  The byte
 *    size of a row (stride * element size) and every device base pointer
 *    must be multiples of 16 bytes (DEDISP_E_ALIGN otherwise).
 *  - Data types: float32 input -> float32 output (optional float32 weights),
 *    uint8 input -> int32 output (exact; weights must be NULL).
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dedisp_plan_s* dedisp_plan;
typedef struct dedisp_batch_s* dedisp_batch;

typedef enum dedisp_status {
  DEDISP_OK = 0,
  DEDISP_E_INVALID = 1, /* bad argument value (count < 1, tsamp <= 0, bad frequency or DM, NULL pointer) */
  DEDISP_E_SHAPE = 2,   /* stride too small for nsamp + max_delay, or a delay that overflows int32 */
  DEDISP_E_DTYPE = 3,   /* unsupported dtype pair, or weights given with uint8 input */
  DEDISP_E_ALIGN = 4,   /* pointer or row byte size not a multiple of 16 */
  DEDISP_E_NOMEM = 5,   /* host or device allocation failed */
  DEDISP_E_HIP = 6,     /* a HIP runtime call failed; detail in dedisp_last_error() */
  DEDISP_E_UNTUNED = 7, /* no compiled kernel variant fits this plan (never returned by execute: it falls back) */
  DEDISP_E_WORKSPACE = 8 /* workspace too small */
} dedisp_status;

typedef enum dedisp_dtype { DEDISP_F32 = 0, DEDISP_U8 = 1, DEDISP_I32 = 2 } dedisp_dtype;

/* ------------------------------------------------------------------------ */
/* Plans                                                                     */
/* ------------------------------------------------------------------------ */

/* Build a plan: the delay table of Section 2, Equation 1 (computed ahead of
 * time, Section 2.1), in FP64 and rounded half up to int32, for channel
 * centre frequencies freq_mhz[nchan] (any order, all > 0 and finite), sample
 * time tsamp_s > 0 and trial DMs dm[ndm] (any order, duplicates allowed,
 * each >= 0 and finite).  Uploads the table and the tile tables of the
 * default kernels to the current device.
 * Errors: DEDISP_E_INVALID for a bad count, frequency, DM, tsamp or NULL
 * pointer; DEDISP_E_SHAPE if a delay does not fit in int32; DEDISP_E_NOMEM /
 * DEDISP_E_HIP on allocation failure.  *plan is NULL on failure. */
dedisp_status dedisp_plan_create(dedisp_plan* plan, int32_t nchan, const double* freq_mhz, double tsamp_s,
                                 int32_t ndm, const double* dm);

/* Host-only: the same delay table a plan would hold, written to
 * host_delays[ndm][nchan], without touching any device.  Same argument rules
 * and errors as dedisp_plan_create. */
dedisp_status dedisp_compute_delays(int32_t nchan, const double* freq_mhz, double tsamp_s, int32_t ndm,
                                    const double* dm, int32_t* host_delays, int32_t* max_delay);

/* Release a plan and its device memory (waits for nothing: do not destroy a
 * plan while work that uses it is still queued). NULL is accepted. */
dedisp_status dedisp_plan_destroy(dedisp_plan plan);

/* Sizes of a plan; any output pointer may be NULL. */
dedisp_status dedisp_plan_info(dedisp_plan plan, int32_t* nchan, int32_t* ndm, int32_t* max_delay);

/* Copy the integer delay table delta[ndm][nchan] to host memory. */
dedisp_status dedisp_plan_delays(dedisp_plan plan, int32_t* host_delays);

/* Choose the kernel of one path (in_type F32 or U8 forward, or the F32
 * adjoint when adjoint != 0) and upload the tile tables it needs.  The
 * float32 forward path is prepared by dedisp_plan_create; the others are
 * prepared on their first call, which then allocates.  Call this before
 * capturing such a first call into a graph. */
dedisp_status dedisp_plan_prepare(dedisp_plan plan, dedisp_dtype in_type, int32_t adjoint);

/* ------------------------------------------------------------------------ */
/* Forward dedispersion (Section 2.1, Algorithm 1)                           */
/* ------------------------------------------------------------------------ */

/* out[b][dm][t] = sum_c w[c] * in[b][c][t + delta[dm][c]] for b < nbeam,
 * dm < ndm, t < nsamp; channels are summed in ascending order, one rounding
 * per term (fused multiply-add; a plain add when d_w == NULL), in an FP32
 * accumulator (int32 for uint8 input).
 *   d_in      [nbeam][nchan][in_stride] of in_type (F32 or U8)
 *   d_w       [nchan] float32 weights, or NULL for all ones (must be NULL for U8)
 *   d_out     [nbeam][ndm][out_stride] of out_type (F32 for F32 input, I32 for U8)
 * Beams share the plan's delays and weights.  Uses the plan's tuned kernel
 * variant for this dtype when one was chosen by dedisp_autotune, otherwise
 * the default; falls back to a direct (untiled) kernel when no tiled variant
 * fits the plan's delay spans.  Asynchronous on `stream`.
 * Errors: DEDISP_E_INVALID (NULL plan or pointer, nbeam < 1, nsamp < 1),
 * DEDISP_E_DTYPE, DEDISP_E_SHAPE (in_stride < nsamp + max_delay,
 * out_stride < nsamp, rows longer than 2^29 samples, or more than 65535
 * beams), DEDISP_E_ALIGN, DEDISP_E_HIP (launch failure). */
dedisp_status dedisp_execute(dedisp_plan plan, int32_t nbeam, int32_t nsamp, const void* d_in, dedisp_dtype in_type,
                             int64_t in_stride, const float* d_w, void* d_out, dedisp_dtype out_type,
                             int64_t out_stride, void* stream);

/* ------------------------------------------------------------------------ */
/* Adjoint (transpose of the Algorithm 1 map) and the weight gradient        */
/* ------------------------------------------------------------------------ */

/* Gather-form adjoint, no atomics, deterministic:
 *   G[b][c][t]        = sum over dm ascending with 0 <= t - delta[dm][c] < nsamp
 *                       of g[b][dm][t - delta[dm][c]]            (FP32)
 *   d_grad_in[b][c][t] = w[c] * G[b][c][t]   for t < nin  (w = 1 if d_w == NULL)
 *   d_grad_w[c]        = sum_b sum_t in[b][c][t] * G[b][c][t]   (FP64 partial sums
 *                       reduced in a fixed order, stored as float32)
 *   d_g       [nbeam][ndm][g_stride] float32 (g_stride >= nsamp)
 *   d_in      [nbeam][nchan][in_stride] float32 forward input, or NULL to skip grad_w
 *   d_grad_in [nbeam][nchan][gi_stride] float32 (gi_stride >= nin), or NULL to skip
 *   d_grad_w  [nchan] float32 or NULL; needs d_in
 *   nin       input samples per channel row to produce (nsamp + max_delay <= nin
 *             <= in_stride when d_in is given)
 *   d_workspace / workspace_bytes: device scratch of at least
 *             dedisp_adjoint_workspace_bytes(plan, nbeam, nin) bytes when
 *             d_grad_w != NULL (may be NULL/0 otherwise).
 * Errors as for dedisp_execute, plus DEDISP_E_WORKSPACE. */
dedisp_status dedisp_adjoint(dedisp_plan plan, int32_t nbeam, int32_t nsamp, int32_t nin, const float* d_g,
                             int64_t g_stride, const float* d_w, const float* d_in, int64_t in_stride,
                             float* d_grad_in, int64_t gi_stride, float* d_grad_w, void* d_workspace,
                             size_t workspace_bytes, void* stream);

/* Bytes of workspace dedisp_adjoint needs for the weight gradient. */
size_t dedisp_adjoint_workspace_bytes(dedisp_plan plan, int32_t nbeam, int32_t nin);

/* Allocation-free form of dedisp_adjoint, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and results as dedisp_adjoint (the
 * same kernels, so grad_in and grad_w are bit-identical to it) without the
 * workspace: the weight gradient's FP64 partial sums go to a fixed scratch
 * array of DEDISP_ADJOINT_NOALLOC_SCRATCH_BYTES (8 MiB) that the library
 * holds on every GPU it runs on until the process ends.  Nothing is
 * allocated or freed by the call: the plan's adjoint kernel and its tile
 * tables must exist already (dedisp_plan_prepare(plan, ..., 1), or an
 * earlier dedisp_adjoint call).  Every call writes each partial sum it later
 * reads, so the scratch needs no clearing, but calls on one GPU share the
 * array: calls that overlap (on different streams, or in different threads)
 * race and give wrong weight gradients.  Calls without d_grad_w do not touch
 * the scratch.
 * Errors as for dedisp_adjoint, plus DEDISP_E_WORKSPACE when the partial sums
 * (dedisp_adjoint_noalloc_bytes) exceed the scratch (use dedisp_adjoint
 * then), DEDISP_E_INVALID when the adjoint kernel or its tables are not
 * prepared or the current device is not the plan's. */
#define DEDISP_ADJOINT_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
dedisp_status dedisp_adjoint_noalloc(dedisp_plan plan, int32_t nbeam, int32_t nsamp, int32_t nin, const float* d_g,
                                     int64_t g_stride, const float* d_w, const float* d_in, int64_t in_stride,
                                     float* d_grad_in, int64_t gi_stride, float* d_grad_w, void* stream);

/* Scratch bytes dedisp_adjoint_noalloc needs for the weight gradient with
 * the plan's chosen adjoint kernel (nbeam x time parts x nchan FP64 values);
 * 0 if that kernel is not chosen yet. */
size_t dedisp_adjoint_noalloc_bytes(dedisp_plan plan, int32_t nbeam, int32_t nin);

/* ------------------------------------------------------------------------ */
/* Batched execution of many uneven beams (multi-beam use, Section 5.1)      */
/* ------------------------------------------------------------------------ */

/* Describe nbeam independent beams, each with its own plan (channel count,
 * DM list), output length nsamp[i], input d_in[i] of type in_t (stride
 * in_stride[i] elements), weights d_w[i] (or NULL) and float32 output
 * d_out[i] (stride out_stride[i]); the same validity rules as dedisp_execute
 * apply to every beam.  Only in_t = DEDISP_F32 is supported (DEDISP_E_DTYPE
 * otherwise): the persistent kernel is the FP32 tile engine.
 *
 * Chooses the tiled kernel variant(s) and builds a device work table of all
 * tiles ordered by decreasing cost for one persistent kernel.  With tune != 0
 * every candidate is timed on the batch's own buffers (their contents are
 * overwritten) and the fastest kept (Section 2.2 and Section 4.1: the best
 * configuration depends on the platform and the set-up); with tune_cache
 * non-NULL the choice is looked up in, and stored to, that JSON file, keyed
 * by the device, the weights flag and the multiset of beam set-ups (channel
 * count, DM count, output length rounded up to a power of two, hash of the
 * delay table), so a later batch of the same shapes skips the search.
 * tune == 0 takes the first default variant that fits every beam.  The
 * arrays are copied; plans and buffers must outlive the batch (the captured
 * graph keeps their addresses).  Allocates; not for use under graph capture. */
dedisp_status dedisp_batch_create(dedisp_batch* batch, int32_t nbeam, const dedisp_plan* plans,
                                  const int32_t* nsamp, const void* const* d_in, dedisp_dtype in_t,
                                  const int64_t* in_stride, const float* const* d_w, void* const* d_out,
                                  const int64_t* out_stride, int32_t tune, const char* tune_cache);

/* 1 if the batch's variant came from its tune cache, 0 if it was searched
 * or defaulted, -1 for a NULL batch. */
int32_t dedisp_batch_cache_hit(dedisp_batch batch);

/* Run every beam of the batch: one persistent launch that walks the work
 * table.  The first call captures the launch into a HIP graph; later calls
 * replay the graph on `stream`.  Calls on one batch must not overlap. */
dedisp_status dedisp_execute_batched(dedisp_batch batch, void* stream);

/* The same work as one dedisp_execute call per beam, in order, on `stream`
 * (the plain per-beam launch loop the batched launch is compared with). */
dedisp_status dedisp_execute_per_beam(dedisp_batch batch, void* stream);

/* Switch the batch to tiled variant `variant` (an index of
 * dedisp_variant_name(DEDISP_F32, .)): rebuilds the work table and drops the
 * captured graph (the next dedisp_execute_batched captures again).  Waits
 * for the device first.  DEDISP_E_INVALID for an index out of range,
 * DEDISP_E_UNTUNED if the variant does not fit some beam (the batch keeps its
 * variant then).  Allocates; not for use under graph capture. */
dedisp_status dedisp_batch_set_variant(dedisp_batch batch, int32_t variant);

/* The tiled variant the batch runs (-1 for a NULL batch). */
int32_t dedisp_batch_variant(dedisp_batch batch);

/* Work queues of the batch's persistent launch: 1 (one global order) or 8
 * (one per XCD, each (beam, time tile) group in one queue, so the blocks
 * that share an input window share that XCD's L2); the tuner keeps the
 * faster (0 for a NULL batch). */
int32_t dedisp_batch_queues(dedisp_batch batch);

/* Rebuild the batch's work table with nqueue (1 or 8) queues, keeping its
 * variant; drops the captured graph.  Waits for the device first.
 * DEDISP_E_INVALID for another count.  Allocates; not for use under graph
 * capture. */
dedisp_status dedisp_batch_set_queues(dedisp_batch batch, int32_t nqueue);

/* Wait for any replay of the batch still in flight, then free it. */
dedisp_status dedisp_batch_destroy(dedisp_batch batch);

/* ------------------------------------------------------------------------ */
/* Single-pulse search (the detection step that dedispersion feeds in the    */
/* real-time pipeline of Section 1; the paper does not define it, so this is */
/* the textbook boxcar matched filter)                                       */
/* ------------------------------------------------------------------------ */

/* For every dedispersed series y = out[b][dm][0 .. nsamp) of dedisp_execute:
 *   widths    w = 1, 2, 4, ..., 2^(nwidth-1) (1 <= nwidth <= 6), skipping
 *             widths longer than nsamp
 *   B_w(t)    = y[t] + ... + y[t + w - 1] for 0 <= t <= nsamp - w
 *   mean, std of y over its nsamp samples (population std, ddof = 0)
 *   S/N_w     = (max_t B_w(t) - w * mean) / (std * sqrt(w)), 0 when std == 0
 * and the result is the width with the largest S/N (ties: the narrower), the
 * first t where that width's boxcar reaches its maximum, the S/N, mean and
 * std.  The series themselves are never written to memory: the search runs
 * in the epilogue of the dedispersion tile kernel (time tiles overlap by the
 * widest window, so each window lies inside one tile), which leaves one
 * 64-byte record per (series, tile) in the workspace; a second kernel merges
 * them.  uint8 input is searched in exact integers (float32 input: boxcar
 * sums in FP32 by pairwise doubling); moments and S/N are FP64.
 *   d_in, in_type, in_stride, d_w: as for dedisp_execute
 *   d_snr    [nbeam][ndm] double        d_width [nbeam][ndm] int32
 *   d_start  [nbeam][ndm] int32         d_mean, d_std [nbeam][ndm] double, or NULL
 *   d_workspace: device scratch of at least dedisp_detect_workspace_bytes(...)
 *            bytes, 16-byte aligned (contents on return: undefined).
 * Uses a kernel variant with the search in its epilogue: the one set with
 * dedisp_plan_set_detect_variant or kept by dedisp_detect_autotune, else the
 * first that fits from an order of preference measured on MI355X (see
 * dedisp_detect_variant); when that is -1 or none fits it dedisperses into
 * the workspace and searches the stored rows (dedisp_detect_rows).  The
 * forward variant (dedisp_plan_set_variant, dedisp_autotune) only serves the
 * unfused path.  Asynchronous on
 * `stream`; the first call of a plan and dtype may build tile tables
 * (allocates).
 * Errors: as dedisp_execute, plus DEDISP_E_INVALID (nwidth out of range,
 * NULL snr/width/start) and DEDISP_E_WORKSPACE (NULL or too small). */
dedisp_status dedisp_detect(dedisp_plan plan, int32_t nbeam, int32_t nsamp, const void* d_in, dedisp_dtype in_type,
                            int64_t in_stride, const float* d_w, int32_t nwidth, double* d_snr, int32_t* d_width,
                            int32_t* d_start, double* d_mean, double* d_std, void* d_workspace,
                            size_t workspace_bytes, void* stream);

/* Workspace bytes dedisp_detect needs for these sizes with the variant it
 * would use now (0 for invalid arguments).  May build tile tables. */
size_t dedisp_detect_workspace_bytes(dedisp_plan plan, dedisp_dtype in_type, int32_t nbeam, int32_t nsamp);

/* The variant dedisp_detect would use for in_type (an index of
 * dedisp_variant_name(in_type, .)), or -1 for the unfused path. */
int32_t dedisp_detect_variant(dedisp_plan plan, dedisp_dtype in_type);

/* Force the search path for in_type: a variant with the search in its
 * epilogue, -1 for the unfused path (dedisp_execute, then the row search),
 * or -2 to go back to the automatic choice.  DEDISP_E_UNTUNED if the variant
 * has no search epilogue or does not fit the plan; may build tile tables. */
dedisp_status dedisp_plan_set_detect_variant(dedisp_plan plan, dedisp_dtype in_type, int32_t variant);

/* Time every fused variant that fits and the unfused path (which uses the
 * plan's current forward variant: tune that first) on nbeam x nsamp
 * scratch samples of in_type, and keep the fastest for dedisp_detect.
 * ms (may be NULL) receives up to n times: ms[i] for variant i (-1 if it
 * does not fit), ms[dedisp_variant_count(in_type)] for the unfused path.
 * Synchronous; allocates scratch memory. */
dedisp_status dedisp_detect_autotune(dedisp_plan plan, int32_t nbeam, int32_t nsamp, dedisp_dtype in_type,
                                     int32_t nwidth, float* ms, int32_t n);

/* The same search over nrows stored series d_rows[nrows][stride] (F32, or
 * I32 searched in float32: exact while every boxcar sum is below 2^24 in
 * magnitude), with a workspace of dedisp_detect_rows_workspace_bytes(nrows,
 * nsamp) bytes.  Output arrays are [nrows].  Errors: DEDISP_E_INVALID,
 * DEDISP_E_DTYPE, DEDISP_E_SHAPE (stride < nsamp), DEDISP_E_ALIGN (row
 * pointer or row bytes not multiples of 16), DEDISP_E_WORKSPACE. */
dedisp_status dedisp_detect_rows(int32_t nrows, int32_t nsamp, const void* d_rows, dedisp_dtype type, int64_t stride,
                                 int32_t nwidth, double* d_snr, int32_t* d_width, int32_t* d_start, double* d_mean,
                                 double* d_std, void* d_workspace, size_t workspace_bytes, void* stream);
size_t dedisp_detect_rows_workspace_bytes(int32_t nrows, int32_t nsamp);

/* ------------------------------------------------------------------------ */
/* Auto-tuning (Section 2.2: tunable work-group and per-thread work sizes,   */
/* chosen by exhaustive search, Sections 3 and 4.1)                          */
/* ------------------------------------------------------------------------ */

/* Time every compiled kernel variant that fits the plan on scratch buffers of
 * nbeam x nsamp samples of in_type, keep the fastest for later execute calls
 * of that dtype, and record the result in the JSON file cache_path (keyed by
 * device, dtype, nchan, ndm, nsamp bucket and a hash of the delay table; a
 * hit skips the search).  cache_path may be NULL (no file).  Synchronous;
 * allocates scratch memory. */
dedisp_status dedisp_autotune(dedisp_plan plan, int32_t nbeam, int32_t nsamp, dedisp_dtype in_type,
                              const char* cache_path);

/* Median times (ms) of the last dedisp_autotune search of this plan and
 * dtype on the calling thread: ms[i] for variant i (-1 if it did not fit or
 * was not timed), ms[dedisp_variant_count(in_type)] for the direct kernel.
 * Copies at most n values; returns the number copied (0 if none). */
int32_t dedisp_autotune_times(dedisp_plan plan, dedisp_dtype in_type, float* ms, int32_t n);

/* Number of kernel variants compiled for in_type, and the name of variant i
 * (static storage; NULL if out of range). */
int32_t dedisp_variant_count(dedisp_dtype in_type);
const char* dedisp_variant_name(dedisp_dtype in_type, int32_t i);

/* Force the variant execute uses for in_type: an index from
 * dedisp_variant_count, or -1 for the direct (untiled) kernel, which is the
 * paper's "generically tuned" form (Section 5: one-dimensional work-groups,
 * one DM per work-item, no data reuse).  Builds the tile tables it needs
 * (allocates).  DEDISP_E_UNTUNED if the variant does not fit the plan. */
dedisp_status dedisp_plan_set_variant(dedisp_plan plan, dedisp_dtype in_type, int32_t variant);

/* Variant execute will use for in_type (-1 = direct kernel). */
int32_t dedisp_plan_variant(dedisp_plan plan, dedisp_dtype in_type);

/* The same for the adjoint (float32 variants; -1 = direct adjoint kernel). */
dedisp_status dedisp_plan_set_adjoint_variant(dedisp_plan plan, int32_t variant);
int32_t dedisp_plan_adjoint_variant(dedisp_plan plan);

/* Auto-tuning of the adjoint (an extension of the paper's tuning, §2.2):
 * time every variant that fits, and the direct adjoint kernel, on nbeam
 * beams of nsamp output samples of scratch data (grad_in and grad_w both
 * computed, as in training), and keep the fastest for dedisp_adjoint.
 * ms (may be NULL) receives up to n times: ms[i] for variant i (-1 if it
 * did not fit), ms[dedisp_variant_count(DEDISP_F32)] for the direct kernel.
 * Synchronous; allocates scratch memory. */
dedisp_status dedisp_autotune_adjoint(dedisp_plan plan, int32_t nbeam, int32_t nsamp, float* ms, int32_t n);

/* ------------------------------------------------------------------------ */
/* Errors                                                                    */
/* ------------------------------------------------------------------------ */

const char* dedisp_status_string(dedisp_status status);
const char* dedisp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DEDISP_H */
