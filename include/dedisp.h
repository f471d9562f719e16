/*
 * dedisp.h -- C ABI of libdedisp, brute-force incoherent dedispersion on
 * AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Sclocco et al., "Auto-Tuning Dedispersion for
 * Many-Core Accelerators" (arXiv:1601.05052):
 *
 *   delay[i][ch] = rint( 4150 * DM_i * (1/f_ch^2 - 1/f_h^2) / t_samp )
 *                                  (Sec. II, Eq. (1), f in MHz, result in samples)
 *   out[i][t]    = sum_ch in[ch][t + delay[i][ch]]        (Sec. III-A, Algorithm 1)
 *
 * for trial DMs DM_i = dm_first + i*dm_step (i < n_dm; Sec. IV sets the grid by
 * its first value and step), channels f_ch = f_min + ch*df (ch < n_channels,
 * channel 0 the lowest frequency) and f_h the top channel's frequency, so the
 * top channel's delay is 0.  The delay table is evaluated on the host in IEEE
 * binary64 (one rounding per operation, no contraction) and rounded half to
 * even.  Sums run in binary32 on the GPU; the order over channels is not
 * specified.
 *
 * Conventions shared by every entry point
 *   - Every function returns DD_OK (0) or a negative dd_status.  On failure
 *     dd_last_error() describes the cause (thread-local; valid until the
 *     calling thread's next dd_* call).
 *   - Argument, shape, stride and alignment errors are detected before any
 *     GPU work is enqueued; nothing is written in that case.
 *   - Device pointers are HIP device allocations on the current device.  The
 *     caller owns every buffer; the library never frees or synchronises
 *     caller memory or streams.  Work is enqueued asynchronously on `stream`
 *     (a hipStream_t; NULL means the default stream).  Faults inside a kernel
 *     surface at the caller's next synchronisation.
 *   - Arrays are row-major; strides are in elements, not bytes.
 *   - A plan is immutable after creation except for its tile choices and its
 *     lazily built device tables (both guarded by a mutex), so one plan may be
 *     used from several host threads and streams at once.
 *   - The first call that uses a plan on a device uploads its tables with a
 *     synchronous copy; make that first call outside HIP graph capture (or
 *     call dd_plan_prepare first).
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_plan dd_plan;
typedef struct dd_batch dd_batch;

/* Input sample storage.  Accumulation is binary32 for every type.
 * DD_F32: IEEE binary32.  DD_F16: IEEE binary16, widened exactly.
 * DD_U8: unsigned 8-bit integers summed as their values (no zero point). */
typedef enum dd_dtype { DD_F32 = 0, DD_F16 = 1, DD_U8 = 2 } dd_dtype;

/* Which linear map a tile choice or a tuning run refers to. */
typedef enum dd_direction { DD_FORWARD = 0, DD_ADJOINT = 1 } dd_direction;

typedef enum dd_status {
    DD_OK = 0,
    DD_EINVAL = -1,       /* bad scalar argument or NULL pointer */
    DD_ESHAPE = -2,       /* stride / size / alignment inconsistent with the plan */
    DD_ENOMEM = -3,       /* host or device allocation failed */
    DD_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
    DD_EUNSUPPORTED = -5  /* valid request the compiled tile variants cannot serve */
} dd_status;

/* ---------------------------------------------------------------- plans */

/* Create a plan: validates the setup and computes the delay table on the
 * host (Sec. II, Eq. (1); Sec. III-A notes it is computed in advance).
 *   n_channels  >= 1          channels; channel ch at f_min_mhz + ch*df_mhz
 *   f_min_mhz   > 0, finite   frequency of channel 0 (the lowest), MHz
 *   df_mhz      > 0, finite   channel spacing, MHz
 *   t_samp_s    > 0, finite   sampling time, seconds
 *   dm_first    >= 0, finite  first trial DM, pc/cm^3
 *   dm_step     >= 0, finite  DM increment, pc/cm^3
 *   n_dm        >= 1          number of trial DMs
 *   n_samples   >= 1          output samples per DM
 * Fails with DD_EINVAL if a delay does not fit int32 or if n_samples plus
 * the largest delay is 2^29 or more.  Touches no GPU.  *out receives the plan
 * (caller destroys it with dd_plan_destroy). */
int dd_plan_create(dd_plan **out, int32_t n_channels, double f_min_mhz, double df_mhz,
                   double t_samp_s, double dm_first, double dm_step, int32_t n_dm,
                   int64_t n_samples);

/* Release a plan and its device tables on every device it used.  NULL is a
 * no-op.  No call may be using the plan concurrently. */
int dd_plan_destroy(dd_plan *plan);

/* Plan dimensions (any output pointer may be NULL). */
int dd_plan_dims(const dd_plan *plan, int32_t *n_channels, int32_t *n_dm, int64_t *n_samples);

/* Largest delay in samples (delay[n_dm-1][0] for the monotone law). */
int dd_plan_max_delay(const dd_plan *plan, int32_t *out);

/* Input samples each channel row must hold: n_samples + max delay. */
int dd_plan_input_samples(const dd_plan *plan, int64_t *out);

/* Copy the delay table, n_dm*n_channels int32, row-major [dm][ch], into host
 * memory owned by the caller. */
int dd_plan_delay_table(const dd_plan *plan, int32_t *host_dst);

/* Build and upload the device tables that `direction` with `in_type` needs on
 * the current device, with a synchronous copy.  Optional: the compute calls
 * do it on first use. */
int dd_plan_prepare(dd_plan *plan, dd_direction direction, dd_dtype in_type);

/* ---------------------------------------------------------------- compute */

/* Forward dedispersion, Sec. III-A, Algorithm 1:
 *   d_out[i*out_stride + t] = sum_ch d_in[ch*in_stride + t + delay[i][ch]]
 * for i < n_dm, t < n_samples.
 *   d_in       device, n_channels rows of in_stride elements of in_type;
 *              in_stride >= n_samples + max_delay; aligned to the element size
 *   d_out      device float, n_dm rows of out_stride >= n_samples; columns
 *              [0, n_samples) are overwritten, padding is never touched
 *   stream     hipStream_t or NULL
 * d_in and d_out must not overlap. */
int dd_dedisperse(const dd_plan *plan, const void *d_in, dd_dtype in_type, int64_t in_stride,
                  float *d_out, int64_t out_stride, void *stream);

/* Allocation-free dd_dedisperse, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and checks as dd_dedisperse, and
 * the same kernels; the plan's tile tables come from the plan's host copy
 * and are staged, by asynchronous copies on `stream`, into one fixed device
 * array of the library (16 MiB, held by each device the library runs on until
 * the process ends), not into memory the plan allocates.  It calls no
 * hipMalloc, hipFree or other allocating routine.
 *   - The plan's forward tables for (in_type's tile variant) must exist: call
 *     dd_plan_prepare(plan, DD_FORWARD, in_type) (or dd_dedisperse once)
 *     beforehand, where allocation is allowed; otherwise DD_EINVAL.
 *   - DD_EUNSUPPORTED if the tables need more than 16 MiB (e.g. a plan of
 *     more than about four million delay-table entries on an LDS-form tile).
 *   - Every call on one device shares the array and overwrites it: calls that
 *     overlap on a device (several host threads, or streams with no ordering
 *     between them) race and must be serialised by the caller. */
int dd_dedisperse_noalloc(const dd_plan *plan, const void *d_in, dd_dtype in_type, int64_t in_stride,
                          float *d_out, int64_t out_stride, void *stream);

/* Adjoint (transpose) of dd_dedisperse for binary32 data:
 *   d_grad_in[ch*in_stride + tau] = sum over i with 0 <= tau - delay[i][ch] < n_samples
 *                                   of d_grad_out[i*out_stride + tau - delay[i][ch]]
 * for ch < n_channels and tau < n_samples + max_delay.  Written as a gather
 * per channel over DMs (no atomics), so results are deterministic.  The
 * direct tile variants with row blocks (dd_tile_info kind 2) enqueue one
 * kernel per block of DMs, d_grad_in holding the partial sums in between.
 *   d_grad_out  device float, n_dm rows of out_stride >= n_samples
 *   d_grad_in   device float, n_channels rows of in_stride >= n_samples + max_delay;
 *               columns [0, n_samples + max_delay) are overwritten (zeros where
 *               no output reads a sample), padding is never touched
 * The two buffers must not overlap. */
int dd_dedisperse_adjoint(const dd_plan *plan, const float *d_grad_out, int64_t out_stride,
                          float *d_grad_in, int64_t in_stride, void *stream);

/* ---------------------------------------------------------------- tiles */

/* Number of compiled tile variants, and the shape of one: each work-group
 * is `waves` wavefronts of 64 lanes; a lane owns `items_t` output samples of
 * `items_acc` output rows (DMs forward, channels adjoint), so a work-group
 * covers (64*items_t) samples x (waves*items_acc) rows -- the four parameters
 * of the paper's Sec. III-B (work-items and elements per work-item, in time
 * and in DM). */
int dd_tile_count(int32_t *n_variants);
int dd_tile_info(int32_t variant, int32_t *items_t, int32_t *items_acc, int32_t *waves,
                 int32_t *kind);

/* Force a tile variant for (direction, in_type) on this plan, or -1 to
 * return to the automatic choice.  DD_EUNSUPPORTED if the variant cannot
 * serve this plan (its staging window would not fit in LDS).  The adjoint
 * works on float32 rows: with DD_ADJOINT, in_type must be DD_F32 (DD_EINVAL
 * otherwise), here and in dd_plan_set_blocks and dd_autotune. */
int dd_plan_set_tile(dd_plan *plan, dd_direction direction, dd_dtype in_type, int32_t variant);

/* Tile variant the next call would use (with a row split, see below, the
 * variant of its largest block). */
int dd_plan_get_tile(const dd_plan *plan, dd_direction direction, dd_dtype in_type,
                     int32_t *variant);

/* Row splits.  Every output is a sum over input rows (channels forward, trial
 * DMs adjoint; Sec. III-A, Algorithm 1).  A plan may split those rows into
 * consecutive blocks, each summed by its own tile variant in its own launch,
 * every block after the first continuing the partial sums the previous one
 * left in the output.  Each output still receives its rows in ascending
 * order, so the results equal those of one variant for all rows, bit for bit.
 * Rows whose delay spread across a tile is small can then use a tile that
 * only fits them (e.g. the adjoint's low trial DMs), the rest a wider one.
 *   row_starts  n_blocks increasing row indices, the first 0; block b holds
 *               rows [row_starts[b], row_starts[b+1]) (the last: to the end);
 *               each start a multiple of its variant's rows per staged chunk
 *   variants    n_blocks tile variants of the LDS or register-window kinds
 * Within a block, each accumulator row's tiles are skewed along time by the
 * average offset of that row over the block's first and last rows, so that a
 * tile's rows line up with the delay curve; a shorter block thus needs a
 * narrower staged window.  dd_plan_set_blocks forces a split for
 * (direction, in_type) (a later dd_plan_set_tile replaces it); dd_autotune may
 * choose one (Sec. IV-A: 2-, 3- and 4-block splits, and 8, 16 and 32 blocks where
 * only the direct kind serves the whole plan, each timed against the best
 * single variant).  Batches always use one variant per beam.  dd_plan_get_blocks reports the launches the next call
 * makes (one block when there is no split); arrays hold up to DD_MAX_BLOCKS.
 *   DD_EINVAL  bad counts, starts or ids;  DD_EUNSUPPORTED  a variant cannot
 *              serve its block */
#define DD_MAX_BLOCKS 32
int dd_plan_set_blocks(dd_plan *plan, dd_direction direction, dd_dtype in_type, int32_t n_blocks,
                       const int32_t *row_starts, const int32_t *variants);
int dd_plan_get_blocks(const dd_plan *plan, dd_direction direction, dd_dtype in_type, int32_t *n_blocks,
                       int32_t *row_starts, int32_t *variants);

/* Auto-tuning, Sec. IV-A: time every tile variant that can serve this plan
 * on the current device (mean of `reps` runs after one warm-up, on private
 * scratch buffers allocated and freed here), keep the fastest for
 * (direction, in_type) and report it.  Variants are timed in the cost model's
 * order; one whose warm-up run takes over 3x the best mean so far is not run
 * again (its warm-up time stands); the three fastest are timed twice and
 * ranked by the mean of both.  If cache_path is non-NULL, the result
 * is looked up in / appended to that text file, keyed by device architecture,
 * direction, dtype and plan shape.  Synchronises `stream`.
 *   best_variant  out, may be NULL
 *   best_ms       out, mean milliseconds of the best variant, may be NULL */
int dd_autotune(dd_plan *plan, dd_direction direction, dd_dtype in_type, int32_t reps,
                const char *cache_path, void *stream, int32_t *best_variant, float *best_ms);

/* ---------------------------------------------------------------- batches */

/* Many independent beams (Sec. III-A describes one beam; the method applies
 * unchanged to each of many) dedispersed by ONE HIP graph launch.
 * Each beam uses the forward tile variant its plan would use alone (forced
 * by dd_plan_set_tile, tuned by dd_autotune / dd_batch_autotune, else the
 * cost model's choice); beams sharing a variant are served by one launch of
 * that variant's multi-beam kernel, whose work list deals every beam's tiles
 * evenly over the XCDs.  The batch keeps pointers to the plans, which must
 * outlive it; every beam uses in_type.  Variant choices are read here: later
 * tuning of the plans does not change an existing batch.  At most 96 beams,
 * each under 2^24 tiles.
 *   DD_EINVAL        NULL argument, n_beams out of range, unknown dtype
 *   DD_EUNSUPPORTED  a beam has no fitting variant or too many tiles
 *   DD_ENOMEM / DD_EHIP  device allocation or graph construction failed */
int dd_batch_create(dd_batch **out, const dd_plan *const *plans, int32_t n_beams,
                    dd_dtype in_type);

/* Auto-tune each plan's forward tile (Sec. IV-A) for in_type over every
 * variant, as dd_autotune does (no row splits); plans of identical shape are
 * timed once per call.  If one variant serves every beam at most 1% slower
 * than each beam's own best (times summed over the beams, each timed alone),
 * every plan gets that variant and the batch becomes a single multi-beam
 * launch.  The choice is stored in each plan (so single-beam calls use it too)
 * and read by the next dd_batch_create; cache_path as in dd_autotune (the
 * common-variant choice is cached under a key of all beams' shapes; it is
 * made only when that key is cached or every beam was timed in this call).
 * Scratch buffers are allocated and freed here.  Synchronises `stream`. */
int dd_batch_autotune(dd_plan *const *plans, int32_t n_beams, dd_dtype in_type, int32_t reps,
                      const char *cache_path, void *stream);

/* Run every beam: for beam b, the forward of plans[b] on d_in[b] (row stride
 * in_strides[b] elements) into d_out[b] (row stride out_strides[b]).  The
 * pointer arrays are host arrays of n_beams device pointers; they are copied
 * into the graph's kernel arguments before the launch, so the host arrays
 * may be reused when the call returns.  Same per-beam requirements as
 * dd_dedisperse; must be called with the batch's device current.  Runs that
 * overlap on one batch from several host threads race on its arguments. */
int dd_batch_run(dd_batch *batch, const void *const *d_in, const int64_t *in_strides,
                 float *const *d_out, const int64_t *out_strides, void *stream);

/* Total additions (sum over beams of n_dm*n_samples*n_channels). */
int dd_batch_adds(const dd_batch *batch, double *adds);

/* The tile variant each beam runs with (variants: n_beams entries). */
int dd_batch_variants(const dd_batch *batch, int32_t *variants);

int dd_batch_destroy(dd_batch *batch);

/* ---------------------------------------------------------------- real time */

/* Streaming dedispersion of one beam, one chunk of n_samples at a time.  The
 * method's step dedisperses one second of data, reading the samples its
 * largest delay reaches past that second (Sec. III-A); real time means each
 * second is dedispersed in under a second (Sec. V, Sec. V-D).  The object keeps
 * the last T_in = n_samples + max_delay input samples of every channel on the
 * device (zeros before the first push).  Push k (k = 0, 1, ...) appends
 * samples [k*S, (k+1)*S) of the stream (S = n_samples) and writes
 *     out[i][t] = sum_ch x[ch][k*S - max_delay + t + delay[i][ch]],  t < S,
 * where x is the pushed stream with x = 0 before time 0: consecutive pushes
 * produce consecutive, non-overlapping output times, max_delay samples behind
 * the newest input.
 *
 * dd_realtime_create binds the plan (which must outlive the object), the
 * input type and the compute stream; it allocates two device windows of
 * n_channels x T_in samples (host chunks are copied straight into them),
 * creates its own non-blocking copy stream, and builds the plan's forward
 * tables.
 *   DD_EINVAL  NULL argument, unknown dtype
 *   DD_ENOMEM / DD_EHIP  allocation or stream set-up failed */
typedef struct dd_realtime dd_realtime;
int dd_realtime_create(dd_realtime **out, const dd_plan *plan, dd_dtype in_type, void *stream);

/* Append one chunk and dedisperse the window.
 *   h_chunk     host memory, n_channels rows of n_samples samples of the bound
 *               in_type, row stride h_stride >= n_samples elements.  The copy to
 *               the device runs asynchronously on the object's copy stream
 *               (overlapping the previous chunk's kernels when h_chunk is pinned,
 *               e.g. from hipHostMalloc); h_chunk must stay unchanged until the
 *               next push on this object returns or the bound stream has been
 *               synchronised.
 *   d_out       device, [n_dm][out_stride] float32, out_stride >= n_samples;
 *               written on the bound stream (columns [0, n_samples) only).
 * The call blocks only until the previous chunk's host copy has completed.
 * Must be called with the object's device current; pushes on one object from
 * several host threads must be serialised by the caller.
 *   DD_EINVAL  NULL argument or wrong device;  DD_ESHAPE  stride or alignment */
int dd_realtime_push(dd_realtime *rt, const void *h_chunk, int64_t h_stride, float *d_out, int64_t out_stride);

/* Number of chunks pushed so far (the next push is chunk *n_pushed). */
int dd_realtime_pushed(const dd_realtime *rt, int64_t *n_pushed);

/* Waits for the object's outstanding copies and for the last kernels that
 * read its windows, then frees it.  NULL is accepted. */
int dd_realtime_destroy(dd_realtime *rt);

/* ---------------------------------------------------------------- candidate search */

/* Boxcar single-pulse search over dedispersed rows.  The dedispersed
 * time-series are searched for pulses afterwards (Sec. I); the paper does not
 * define that step, so this is the plain definition: for each row y[0:S]
 * (S = n_samples), with mu and sigma its mean and population standard
 * deviation,
 *     snr_w(t) = sum_{i < w} (y[t + i] - mu) / (sigma * sqrt(w))
 * for w = 1, 2, 4, ..., 2^(n_widths - 1) (widths <= S) and 0 <= t <= S - w.
 * Per row it writes the largest snr and one (t, w) reaching it (ties: smaller
 * w, then smaller t); a row with sigma == 0 gives (0, 0, 1).  mu and sigma are
 * accumulated in binary64, boxcar sums in binary32.
 *   d_rows      device, [n_rows][row_stride] float32 (e.g. dd_dedisperse's
 *               output), row_stride >= n_samples
 *   n_widths    1 .. 12 (widths up to 2048 samples)
 *   d_snr       device, n_rows float32;  d_t, d_width: device, n_rows int32
 * Runs asynchronously on `stream` (one work-group per row).
 *   DD_EINVAL  NULL pointer, n_rows < 1, n_samples outside [1, 2^31), n_widths
 *   DD_ESHAPE  row_stride < n_samples, misaligned pointer */
int dd_search_boxcar(const float *d_rows, int64_t row_stride, int32_t n_rows, int64_t n_samples, int32_t n_widths,
                     float *d_snr, int32_t *d_t, int32_t *d_width, void *stream);

/* ---------------------------------------------------------------- errors */

/* Message for the calling thread's last failure ("" if none). */
const char *dd_last_error(void);

/* Library version string. */
const char *dd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DEDISP_H */
