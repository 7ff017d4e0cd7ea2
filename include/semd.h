/*
 * semd.h -- C ABI of the MI355X (gfx950) Serial-EMD library, libsemd.so.
 *
 * Serial-EMD (Zhang et al., arXiv 2106.15319) decomposes a set of N equally
 * long signals -- the columns of an M x N matrix X (Sec. 3.2) -- by
 * serializing them into one 1D signal of length L = M*N + D*N - D with linear
 * cross-fade transitions of length D between neighbouring columns (Sec. 3.2),
 * running 1D EMD on it (Sec. 2.1; EEMD, Sec. 2.2) and slicing the IMFs back to
 * M x N by dropping the transition samples (Sec. 3.3).
 *
 * Conventions shared by every call:
 *  - Arrays are FP64.  Device pointers point to HIP device memory of the
 *    current device; [host] marks host memory.
 *  - X is column-major: element (m, i) at m + M*i, column i = signal i.  With
 *    ndim > 2, dims[1..ndim-1] are flattened column-major into N.
 *  - Output slots: imfs_out holds (max_imfs + 1) slots of M*N doubles each.
 *    Slot k < n_imfs is IMF k (k = 0 is the highest-frequency mode), slots
 *    n_imfs .. max_imfs-1 are zero (the zero-fill convention of Sec. 4.3) and
 *    slot max_imfs is the residue r of eq. (1), so sum of all slots = X.
 *  - Sifting: sift_iters (S) sifts per IMF; an IMF ends early when its
 *    candidate has no maximum, no minimum or fewer than 3 extrema; the
 *    decomposition stops when the residue is in that state or max_imfs IMFs
 *    exist (the paper leaves the stopping rule open, Sec. 2.1 Step 5).
 *  - Envelopes: natural cubic splines through the extrema (one per equal-valued
 *    run, at its floor-middle; end samples excluded) plus min(2, n) knots
 *    mirrored about each end sample (boundary_rule SEMD_BOUNDARY_MIRROR).
 *  - Every call validates its arguments on the host first; on an invalid
 *    argument it returns SEMD_EINVAL, records a message for semd_last_error()
 *    and enqueues nothing.  Work is enqueued on `stream` and the call returns
 *    without waiting for it; a launch failure returns SEMD_EDEVICE.
 *  - Input containing NaN or Inf is not decomposed: its n_imfs entry is set to
 *    -SEMD_ENONFINITE and all of its slots to zero.
 *  - The library never writes to the input and never frees caller memory.
 *    Outputs must not overlap inputs.  Calls that overlap on one stream are
 *    ordered; on different streams they are independent.
 */
#ifndef SEMD_H
#define SEMD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SEMD_ABI_VERSION 3

typedef enum {
  SEMD_OK = 0,
  SEMD_EINVAL = 1,       /* invalid argument; nothing enqueued             */
  SEMD_ENOMEM = 2,       /* a device or pinned allocation failed           */
  SEMD_EDEVICE = 3,      /* a HIP call or kernel launch failed             */
  SEMD_EBUSY = 4,        /* serving engine: request exceeds free budget    */
  SEMD_ENONFINITE = 5,   /* input holds NaN/Inf (reported via n_imfs)      */
  SEMD_EUNSUPPORTED = 6  /* valid request the library cannot run          */
} semd_status;

typedef enum { SEMD_BOUNDARY_MIRROR = 0 } semd_boundary;

/* Execution path.  AUTO: one workgroup decomposes a signal on chip when its
 * serialized length is at most semd_resident_max_length(), the streaming
 * path (many workgroups per signal, state in device memory) otherwise.  The
 * two paths compute the same decomposition within rounding. */
typedef enum { SEMD_PATH_AUTO = 0, SEMD_PATH_ONCHIP = 1, SEMD_PATH_STREAM = 2 } semd_path;

/* When an IMF's sifting stops (Sec. 2.1 Step 5 leaves the criterion open).
 * FIXED: after sift_iters sifts.  SD: also after the first sift whose mean
 * envelope m satisfies sum m^2 < sd_threshold * sum h^2, h the candidate
 * before that sift, still at most sift_iters sifts.  This is the
 * ratio-of-sums (Cauchy-type) form of the standard-deviation test between
 * consecutive candidates (h - (h - m) = m), not the sum of per-sample ratios.
 * Either way an IMF ends early when its candidate has too few extrema to
 * sift. */
typedef enum { SEMD_STOP_FIXED = 0, SEMD_STOP_SD = 1 } semd_stop;

/* Method parameters.  transition_len is D of Sec. 3.2 (0 <= D <= M);
 * max_imfs is K >= 1; sift_iters is S >= 1; ensemble is the number NR >= 1 of
 * EEMD realizations (Sec. 2.2, used by semd_eemd_batch only); path is a
 * semd_path; seed keys the EEMD noise; stop_rule is a semd_stop and
 * sd_threshold (> 0, finite) its threshold under SEMD_STOP_SD. */
typedef struct {
  int32_t transition_len;
  int32_t max_imfs;
  int32_t sift_iters;
  int32_t boundary_rule;
  int32_t ensemble;
  int32_t path;
  uint64_t seed;
  int32_t stop_rule;
  int32_t reserved; /* must be 0 */
  double sd_threshold;
} semd_params;

/* One signal of a batch.  signal: device, M*N doubles (M = dims[0], N =
 * product of dims[1..ndim-1]); imfs_out: device, (K+1)*M*N doubles;
 * n_imfs_out: device, one int32, or NULL.  stats_out: device, 3 int64, or
 * NULL: receives the number of sifts performed, the number of envelope knots
 * used (mirrored knots included) and the number of sample-sifts (sum over
 * sifts of L); semd_decompose_batch, and semd_eemd_batch (summed over the
 * item's realizations).  noise_sigma is the absolute EEMD
 * noise amplitude beta of Sec. 2.2 for semd_eemd_batch, and the relative
 * amplitude eps for semd_ceemdan_batch; item_id selects the item's noise
 * streams. */
typedef struct {
  const double* signal;
  double* imfs_out;
  int32_t* n_imfs_out;
  int64_t* stats_out;
  int64_t dims[4];
  int32_t ndim;
  int32_t reserved; /* must be 0 */
  double noise_sigma;
  uint64_t item_id;
} semd_item;

/* ---- information ------------------------------------------------------- */

/* ABI version (SEMD_ABI_VERSION). */
int semd_abi_version(void);

/* Message of the last failed call on this host thread ("" if none). */
const char* semd_last_error(void);

/* Sec. 3.2: serialized length M*N + D*N - D, or -1 if M < 1, N < 1 or D is
 * outside [0, M]. */
int64_t semd_serial_length(int64_t M, int64_t N, int64_t D);

/* Longest serialized signal the single-workgroup on-chip path takes (longer
 * signals go to the multi-workgroup streaming path).  Any path accepts
 * serialized lengths up to 2^28; longer ones return SEMD_EUNSUPPORTED. */
int64_t semd_resident_max_length(void);

/* ---- launch-shape tuning (on-chip path) -------------------------------- */

/* The on-chip kernel runs one workgroup per signal in one of several compiled
 * launch shapes (threads per workgroup x samples per thread); the shape
 * changes speed only, never results.  A process-wide table chooses the shape
 * per signal-length bucket (upper bounds 1024, 2048, 3072, 4096, 6144, 8192,
 * 12288, 16384) and per regime: "latency" for launches with fewer signals
 * than the device has compute units, "throughput" otherwise.  Buckets absent
 * from the table use built-in defaults.  These calls are not meant to run
 * concurrently with decompositions on other host threads. */

/* Times every eligible shape for each bucket up to max_length (in [3,
 * 16384]) on synthetic signals -- one signal for the latency regime, `batch`
 * (at least the compute-unit count) for the throughput regime, 6 IMFs x 10
 * sifts -- and records the fastest in the table.  Blocks until done; uses
 * `stream` and temporary device memory. */
int semd_autotune(int64_t max_length, int batch, hipStream_t stream);

/* The table as text ([host] buf of cap bytes, NUL-terminated; *needed [host]
 * receives the size it needs).  First line "semd-tune <abi> <gfx arch>", then
 * one line "latency|throughput <bucket bound> <threads> <samples>" per entry.
 * Returns SEMD_EINVAL (with *needed set) when cap is too small. */
int semd_tune_get(char* buf, size_t cap, size_t* needed);

/* Replaces the table with one in the text form above ([host] NUL-terminated).
 * SEMD_EINVAL if it was made for another ABI version or GPU architecture, or
 * names a shape that is not compiled or too small for its bucket; the table
 * is then unchanged. */
int semd_tune_set(const char* text);

/* Empties the table (built-in defaults everywhere). */
int semd_tune_reset(void);

/* ---- the method --------------------------------------------------------- */

/* Serial-EMD of one signal (Sec. 3): serialize, EMD, deserialize.  D is the
 * paper's recommended 20% of the signal length, round(0.2*M) (Sec. 4.1); no
 * ensemble.  dims: [host], ndim >= 1 entries. */
int semd_decompose(const double* signal, const int64_t* dims, int ndim, int max_imfs,
                   int sift_iters, int boundary_rule, double* imfs_out, hipStream_t stream);

/* Device bytes of the workspace semd_decompose_ex needs for a signal of
 * these dims under these parameters (dims: [host]; p: [host]): the signal's
 * descriptor, on the streaming path its tile tables, and the path's state --
 * the residue r and candidate h of Sec. 2.1 Steps 1-5 over the L = M*N +
 * D*N - D serialized samples of Sec. 3.2, and the envelope knots.  Returns 0
 * (message in semd_last_error()) when semd_decompose_ex would reject the
 * arguments with SEMD_EINVAL or SEMD_EUNSUPPORTED. */
size_t semd_workspace_bytes(const int64_t* dims, int ndim, const semd_params* p);

/* Serial-EMD of one signal (Sec. 3: serialize with transition length D of
 * Sec. 3.2, 1D EMD of Sec. 2.1, deserialize as in Sec. 3.3) with explicit
 * parameters (p->ensemble is ignored), launched on its own: the plain
 * one-signal-per-launch path.  signal: device, M*N doubles; imfs_out:
 * device, (K+1)*M*N doubles; n_imfs_out: device int32 or NULL; dims, p:
 * [host].
 * workspace: device memory owned by the caller, at least
 * semd_workspace_bytes(dims, ndim, p) bytes (ws_bytes), 256-byte aligned,
 * not touched by anything else until the work enqueued on `stream` has
 * finished; its contents need no initialization and are undefined after.
 * With workspace == NULL (ws_bytes ignored) the library allocates and frees
 * the workspace itself, stream-ordered, from its memory pool.  An
 * undersized or misaligned workspace returns SEMD_EINVAL with nothing
 * enqueued.  With a workspace the call enqueues kernels only (no allocation,
 * no copy, no memset), so it may be captured into a HIP graph. */
int semd_decompose_ex(const double* signal, const int64_t* dims, int ndim,
                      const semd_params* p, double* imfs_out, int32_t* n_imfs_out,
                      void* workspace, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the same
 * decomposition as semd_decompose_ex, bit for bit, with its workspace in a
 * static device array of semd_noalloc_scratch_bytes() bytes (64 MiB) that
 * each GPU the library runs on holds until the process ends.  It calls no
 * allocator; it enqueues kernels only.  Signals whose
 * semd_workspace_bytes(dims, ndim, p) exceeds the array (serialized lengths
 * above about 1.36 million samples on the streaming path) return SEMD_EINVAL
 * with nothing enqueued.  Every call on one GPU uses that GPU's one array:
 * calls that overlap in time on one GPU (different streams, or host threads
 * without ordering between their streams) race and corrupt each other's
 * results; calls ordered on one stream are safe.  The array's contents need
 * no initialization and are undefined between calls. */
int semd_decompose_ex_noalloc(const double* signal, const int64_t* dims, int ndim,
                              const semd_params* p, double* imfs_out, int32_t* n_imfs_out,
                              hipStream_t stream);

/* Size of the static array semd_decompose_ex_noalloc works in. */
size_t semd_noalloc_scratch_bytes(void);

/* Parity instrumentation for the extremum decisions of Sec. 2.1 Step 1:
 * semd_decompose_ex (library-allocated workspace) that also records every
 * extremum detection the decomposition makes.  trace: device, trace_cap
 * int32 (4 <= trace_cap < 2^31); afterwards trace[0] = entries used (the 4
 * header entries included), trace[1] = 1 if every record fitted (0 once one
 * did not; recording stops there), then one record per detection, in order:
 *   imf, sift, nmax, nmin, maxima (nmax positions), minima (nmin positions)
 * -- positions in the serialized signal of Sec. 3.2, increasing; sift 0 is
 * the detection on the residue before IMF imf, sift s > 0 the one on the
 * candidate before its sift s.  On the on-chip path the decomposition runs
 * in its 1024-thread x 16-sample launch shape; outputs equal
 * semd_decompose_ex's bit for bit on the streaming path and whenever
 * semd_decompose_ex also takes a 1024-thread shape, within rounding
 * otherwise. */
int semd_decompose_trace(const double* signal, const int64_t* dims, int ndim,
                         const semd_params* p, double* imfs_out, int32_t* n_imfs_out,
                         int32_t* trace, int64_t trace_cap, hipStream_t stream);

/* Standard (slice-wise) EMD, the baseline Serial-EMD is compared with (Sec. 4):
 * each of the N columns of X (length M each, dims as above) is decomposed by
 * the 1D EMD of Sec. 2.1 on its own, with no serialization.  p->transition_len
 * must be 0; p->ensemble is ignored.  imfs_out: (K+1)*M*N doubles in the same
 * slot-major layout as semd_decompose_ex (column i of every slot is column
 * i's mode); n_imfs_out: N int32 (IMFs of each column) or NULL.  Signals longer
 * than semd_resident_max_length() take the streaming path. */
int semd_decompose_slices(const double* signal, const int64_t* dims, int ndim,
                          const semd_params* p, double* imfs_out, int32_t* n_imfs_out,
                          hipStream_t stream);

/* Serial-EMD of n independent signals of any shapes in one batched launch
 * (p->ensemble ignored).  items, p: [host]; the items array may be reused as
 * soon as the call returns. */
int semd_decompose_batch(const semd_item* items, int n, const semd_params* p,
                         hipStream_t stream);

/* Serial-EEMD (Sec. 2.2 applied to the serialized signal, Sec. 3.3): for each
 * item, NR = p->ensemble realizations x + beta*w_m (beta = item noise_sigma,
 * w_m white noise with zero mean and unit variance drawn from SplitMix64
 * streams keyed by (p->seed, item_id, m)), each decomposed by EMD, and the
 * slot-wise mean over m written to imfs_out (zero-filled slots included).
 * n_imfs_out receives the largest IMF count over the realizations. */
int semd_eemd_batch(const semd_item* items, int n, const semd_params* p, hipStream_t stream);

/* Serial-CEEMDAN (Sec. 2.2, Torres et al. 2011, on the serialized signal x of
 * Sec. 3.2).  With w_m (m < NR = p->ensemble) the noise realizations of
 * semd_eemd_batch, E_i(w) the i-th mode of the EMD of w (zero if it has
 * fewer), F1(v) the first EMD mode of v, std the population standard
 * deviation over the L serialized samples and eps = the item's noise_sigma:
 *   mode 1:      c_1 = mean_m F1(x + eps std(x) w_m),
 *   mode i > 1:  c_i = mean_m F1(r_{i-1} + eps std(r_{i-1}) E_{i-1}(w_m)),
 *   r_i = r_{i-1} - c_i, r_0 = x.
 * A mode is extracted while the residue can still be sifted (>= 1 maximum,
 * >= 1 minimum, >= 3 extrema) and i <= K = p->max_imfs.  Every EMD uses
 * p->sift_iters sifts per mode and p->stop_rule.  imfs_out receives the
 * deserialized modes, zero slots, and the residue in slot K; n_imfs_out the
 * number of modes (-5 for NaN/Inf input, all outputs zero).  Cost: about
 * 2 * NR times an EMD of the item.  items, p: [host]; eps finite and >= 0. */
int semd_ceemdan_batch(const semd_item* items, int n, const semd_params* p,
                       hipStream_t stream);

/* ---- single steps (each runs the kernels of the full path) -------------- */

/* Sec. 3.2: x (device, L doubles) = serialization of X with transition D. */
int semd_serialize(const double* X, const int64_t* dims, int ndim, int D, double* x,
                   hipStream_t stream);

/* Sec. 3.3: out (device, M*N doubles) = y (device, L doubles) with the
 * transition samples removed. */
int semd_deserialize(const double* y, const int64_t* dims, int ndim, int D, double* out,
                     hipStream_t stream);

/* Sec. 2.1 Step 1 on a 1D signal h (device, L doubles, 3 <= L <=
 * semd_resident_max_length()): imax / imin (device, each L/2+1 int32) receive
 * the maxima / minima indices in increasing order, counts (device, 2 int32)
 * their numbers. */
int semd_extrema(const double* h, int64_t L, int32_t* imax, int32_t* imin, int32_t* counts,
                 hipStream_t stream);

/* Sec. 2.2 Step 1 noise: w (device, L doubles) = the white-noise stream of
 * realization m of item `item` under `seed`, as used by semd_eemd_batch. */
int semd_noise(uint64_t seed, uint64_t item, uint64_t m, int64_t L, double* w,
               hipStream_t stream);

/* ---- memory --------------------------------------------------------------- */

/* Workspaces the library allocates (every call but semd_decompose_ex with a
 * caller's workspace and semd_decompose_ex_noalloc) come stream-ordered from
 * a memory pool of the library's own per device, which keeps freed memory
 * for the next call instead of returning it to the device.  This call
 * returns every cached, unused byte of those pools to the device (for
 * callers that need the memory elsewhere); later calls allocate anew. */
int semd_release_cached_memory(void);

/* ---- kernel timing (measurement) ---------------------------------------- */

/* While enabled (on != 0), the batch calls (semd_decompose_batch,
 * semd_eemd_batch, semd_decompose_slices, semd_ceemdan_batch) record HIP
 * events on the launch stream around every on-chip launch and around each
 * kernel of every streaming step; the streaming steps are then launched
 * directly instead of replayed from a captured graph (same kernels, same
 * order, same results).  semd_profile_read waits for the recorded events and
 * returns, for one kernel ("st_load_kernel", "st_scan_kernel",
 * "st_compact_kernel", "st_solve_kernel", "st_eval_kernel" or
 * "resident_emd_kernel"), the launches timed since the last reset and
 * their summed duration in milliseconds, or for one host phase of the batch
 * calls ("host_alloc", "host_tables", "host_upload", "host_launch",
 * "host_batch_call") the calls and their summed wall time ([host]
 * results).  Not meant to run concurrently with decompositions on other
 * host threads. */
int semd_profile_enable(int on);
int semd_profile_reset(void);
int semd_profile_read(const char* kernel, int64_t* launches, double* total_ms);

/* ---- serving: continuous batching -------------------------------------- */

/* An engine keeps decompositions of independent requests resident on the
 * device and advances all of them at every semd_engine_step.  Requests join
 * between steps when their device footprint fits the engine's memory
 * budget.  Each request is routed as semd_decompose_ex routes its path:
 * on chip (path AUTO up to semd_resident_max_length() samples, or ONCHIP),
 * the whole decomposition of every request admitted since the last step
 * runs in one launch at the next step and completes with it; streaming
 * (longer ones, or path STREAM), each step performs one sift (Sec. 2.1),
 * whatever IMF or sift the request is at, or the IMF end / final output
 * work it reaches.  Every request is decomposed exactly as
 * semd_decompose_ex with the same parameters would (bit-identical outputs):
 * its arithmetic does not depend on the others.
 * All engine calls on one engine must come from one host thread at a time
 * and all steps must use one stream.  The engine owns its device memory
 * (hbm_budget_bytes, allocated at creation); the caller owns every
 * request's input and output buffers, which must stay valid until the
 * request is reported done. */
typedef struct semd_engine semd_engine;

/* max_requests >= 1 resident requests at a time. */
int semd_engine_create(size_t hbm_budget_bytes, int max_requests, semd_engine** out);

/* Device bytes a request needs inside an engine. */
int semd_engine_footprint(const semd_item* item, const semd_params* p, size_t* bytes);

/* Admit one request (item: [host]; its signal, imfs_out and n_imfs_out as in
 * semd_decompose_batch; noise fields ignored).  *ticket identifies it.
 * SEMD_EBUSY: the footprint does not fit the free budget or all request
 * slots are taken; retry after finished requests are polled.  SEMD_ENOMEM:
 * the footprint exceeds the engine's whole budget, so the request can never
 * be admitted. */
int semd_engine_admit(semd_engine* e, const semd_item* item, const semd_params* p,
                      int64_t* ticket);

/* One step of every resident request, enqueued on `stream`. */
int semd_engine_step(semd_engine* e, hipStream_t stream);

/* n_steps consecutive steps in one call, enqueued on `stream`: the requests
 * admitted since the last call (on chip: whole) start with the first, and
 * every streaming request advances by n_steps sifts (Sec. 2.1), or less
 * when it finishes on the way; outputs are the same as from n_steps calls
 * of semd_engine_step.  Completions are gathered once, after the last step,
 * so a caller with no request waiting for admission saves the per-step host
 * round trip.  n_steps outside [1, SEMD_ENGINE_MAX_STEPS] is SEMD_EINVAL. */
#define SEMD_ENGINE_MAX_STEPS 64
int semd_engine_step_n(semd_engine* e, int n_steps, hipStream_t stream);

/* Up to cap tickets ([host] done) of requests whose outputs are complete in
 * stream order; n_done receives their number.  Does not wait for the device
 * except for the step before the last one issued. */
int semd_engine_poll(semd_engine* e, int64_t* done, int cap, int* n_done);

/* Number of resident (admitted, not yet reported done) requests. */
int semd_engine_resident(semd_engine* e, int* n);

/* Waits for the engine's work and frees its device memory. */
int semd_engine_destroy(semd_engine* e);

#ifdef __cplusplus
}
#endif
#endif /* SEMD_H */
