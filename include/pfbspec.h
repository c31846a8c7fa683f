/*
 * pfbspec -- polyphase-filter-bank spectrometer on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  Plain pointers and sizes only; no C++ or framework
 * types cross this boundary.  Device pointers are HIP device addresses on
 * the plan's device; host pointers are ordinary process memory.
 *
 * What one plan computes (A GPU-Based Wide-Band Radio Spectrometer, Section 4,
 * with the initialisation / per-block loop of its high-level algorithm):
 *
 *   input   : a stream of 8-bit complex samples, one or two polarisations,
 *             int8 x[t][pol][2] (time-major; re then im; two's complement);
 *   filter  : spectrum j is the N-point DFT of
 *               y_j[n] = sum_{p<P} h[p*N + n] * x[(j+p)*N + n]
 *             (P-tap polyphase filter bank, hop N); in direct mode y_j is
 *             frame j itself (no filter);
 *   FFT     : X_j[k] = sum_n y_j[n] exp(-2 pi i k n / N), natural order;
 *   products: |X|^2 for one polarisation; |X|^2, |Y|^2, Re(X Y*), Im(X Y*)
 *             for two (Section 4);
 *   dumps   : the products summed over n_int consecutive valid spectra
 *             ("accumulate spectra for desired duration").
 *
 * Spectrum j = 0 is the first one whose P frames have all arrived; earlier
 * partial windows are not emitted.  The last P-1 frames of every block are
 * kept by the plan (the "tap history") so that the stream may be cut into
 * blocks of any whole number of frames.
 *
 * Threading: a plan is not thread-safe; calls on one plan must be ordered on
 * one stream.  Distinct plans are independent.  Every call is asynchronous
 * with respect to the host unless stated otherwise.
 *
 * Errors: every call returns a status; no exception crosses the ABI.
 * Arguments are validated before any state changes, so a rejected call leaves
 * the plan as it was.  A failure reported by the HIP runtime marks the plan
 * poisoned: later calls return PFBS_ERR_STATE until pfbs_plan_reset().
 * pfbs_last_error() describes the most recent failure of the calling thread.
 */
#ifndef PFBSPEC_H
#define PFBSPEC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfbs_plan pfbs_plan;    /* opaque; owns all device state of one stream */
typedef struct pfbs_batch pfbs_batch;  /* opaque; several plans run by one launch sequence */
typedef struct pfbs_hstream pfbs_hstream;  /* opaque; a plan fed from host memory */

typedef enum {
    PFBS_OK = 0,
    PFBS_ERR_INVALID = 1,     /* an argument is out of range or inconsistent   */
    PFBS_ERR_UNSUPPORTED = 2, /* valid request the library does not support   */
    PFBS_ERR_NOMEM = 3,       /* device or host allocation failed              */
    PFBS_ERR_DEVICE = 4,      /* the HIP runtime reported an error             */
    PFBS_ERR_STATE = 5        /* plan destroyed, poisoned, or used wrongly     */
} pfbs_status;

/* Prototype filter of the polyphase filter bank (Section 4 names an 8-tap PFB
 * but not its coefficients):
 *   HANN_SINC: h[m] = sinc((m - P*N/2)/N) * (1/2 - 1/2 cos(2 pi m/(P*N))),
 *              sinc(u) = sin(pi u)/(pi u), no gain normalisation;
 *   RECT     : h[m] = 1 (with P = 1 this reproduces direct mode);
 *   CUSTOM   : P*N double coefficients supplied by the caller.            */
typedef enum {
    PFBS_WINDOW_HANN_SINC = 0,
    PFBS_WINDOW_RECT = 1,
    PFBS_WINDOW_CUSTOM = 2
} pfbs_window;

/* PFB: pre-filter then FFT.  DIRECT: FFT of each frame (P must be 1). */
typedef enum { PFBS_MODE_PFB = 0, PFBS_MODE_DIRECT = 1 } pfbs_mode;

/* Arithmetic of the FFT.  FP32: every stage on the vector ALUs in float,
 * except that from 2^18 channels the row pass of the two-pass FFT (its second
 * set of sub-transforms, Section 4 "parallel FFTs") runs in double on the
 * same ALUs: a strong tone's energy sits in one intermediate row and
 * single-precision rounding of that row, spread over all of its channels,
 * exceeds 1e-5 of the integrated power there; the intermediate between the
 * passes, the products' accumulation and the dumps stay FP32.
 * MFMA_FP16: each radix-16 stage as a product with the 16x16 DFT matrix on
 * the FP16 matrix cores (v_mfma_f32_16x16x32_f16, FP32 accumulation), matrix
 * and data rounded to single FP16 values after a per-butterfly power-of-two
 * scaling; about 3 significant decimal digits.  MFMA_FP16X2: matrix and data
 * split into FP16 hi + lo pairs, three products per stage (Wlo*hi + Whi*lo +
 * Whi*hi); accuracy of the FP32 path.  The first radix-2/4/8 stage, the
 * inter-stage and four-step twiddles, the pre-filter, the products and the
 * accumulation stay FP32 in every precision.  MIXED: the single pass and the
 * column pass of the two-pass FFT in FP32, the row pass as MFMA_FP16X2; the
 * row pass is where a strong tone's rounding error concentrates (its energy
 * sits in one intermediate row), so MIXED meets the FP32 path's accuracy with
 * the faster 256-point column split at every N.  Batches (pfbs_batch_create)
 * take FP32 and MIXED plans. */
typedef enum {
    PFBS_PREC_FP32 = 0,
    PFBS_PREC_MFMA_FP16 = 1,
    PFBS_PREC_MFMA_FP16X2 = 2,
    PFBS_PREC_MIXED = 3
} pfbs_precision;

/* Form of the dumps (and of pfbs_flush's partial sum).  PRODUCTS: the four
 * integrated products |X|^2, |Y|^2, Re XY*, Im XY* (Section 4).  STOKES
 * (two polarisations only): I = |X|^2 + |Y|^2, Q = |X|^2 - |Y|^2,
 * U = 2 Re XY*, V = -2 Im XY*, the Stokes parameters of linear feeds, which
 * the paper notes follow from the four products (Section 4); computed in
 * FP32 from the integrated products. */
typedef enum { PFBS_OUT_PRODUCTS = 0, PFBS_OUT_STOKES = 1 } pfbs_output;

/* Full plan description.  Fields beyond the six of pfbs_plan_create:
 *   precision   : see pfbs_precision;
 *   custom_taps : host array of P*N doubles, read during the call only,
 *                 required iff window == PFBS_WINDOW_CUSTOM, else ignored;
 *   device      : HIP device ordinal, -1 = the calling thread's current one;
 *   tune        : 0 = built-in heuristics, 1 = consult / fill the autotune
 *                 cache (file named by PFBS_TUNE_CACHE, when set);
 *   chunk       : spectra per partial integration (0 = automatic);
 *   split_n2    : column length of the two-pass FFT (0 = automatic);
 *   group_bytes : bound on the intermediate buffer of the two-pass FFT
 *                 (0 = automatic);
 *   col_run     : spectra per workgroup of the column pass (0 = automatic);
 *   output      : see pfbs_output (batched plans: PRODUCTS only);
 *   fftshift    : 1 = each dump row in shifted channel order (channel k at
 *                 position (k + N/2) mod N, negative frequencies first);
 *                 batched plans: 0 only;
 *   stream_z    : 1 = streaming (non-temporal) stores and loads of the
 *                 two-pass intermediate, 0 = ordinary ones;
 *   tap_unroll, col_pair: see the fields (speed only; the same arithmetic in
 *                 the same order either way, so the same bits).
 * chunk, split_n2, group_bytes, col_run, stream_z, tap_unroll, col_pair and
 * row_tile only change speed, never results beyond FP32 rounding order
 * (tap_unroll, col_pair and row_tile not even that: same bits).
 * With tune = 1 they are taken from the autotune cache when it holds an
 * entry for this device and shape (see pfbs_autotune); with tune = 2 a
 * missing entry is measured first.                                          */
typedef struct {
    int64_t N;
    int32_t P;
    int32_t window;     /* pfbs_window    */
    int32_t mode;       /* pfbs_mode      */
    int32_t n_pol;
    int64_t n_int;
    int32_t precision;  /* pfbs_precision */
    int32_t device;
    const double *custom_taps;
    int32_t tune;
    int32_t chunk;
    int64_t split_n2;
    int64_t group_bytes;
    int32_t col_run;
    int32_t stream_z;
    int32_t output;     /* pfbs_output */
    int32_t fftshift;   /* 1: channels in shifted order, k' = (k + N/2) mod N */
    int32_t tap_unroll; /* pre-filter tap loop: 0 automatic, 1 unrolled at compile
                           time (P = 4 or 8), 2 a loop over P at run time */
    int32_t col_pair;   /* column pass on two spectra per workgroup step (pre-filter
                           with 4-point columns of at most 256, PFB mode): 0
                           automatic, 1 where it applies, 2 never */
    int32_t row_tile;   /* row pass of the two-pass FFT: points per polarisation per
                           workgroup step (TP/N1 rows of N1 points, TP/16 threads
                           per polarisation): 0 = max(1024, N1), else 1024, 2048
                           or 4096, at least N1 (PFBS_ERR_INVALID otherwise);
                           ignored for N <= 4096 */
} pfbs_plan_desc;

/* Create a plan (FP32 arithmetic; Section 4, initialisation: coefficients are
 * generated and loaded to the device, the FFT is planned).
 *   N     : channels = FFT length, a power of two in [16, 2^20];
 *   P     : taps (frames per spectrum), 1..16; must be 1 in DIRECT mode;
 *   n_pol : 1 or 2 polarisations;
 *   n_int : spectra per dump, >= 1.
 * On success *out owns device memory for the taps, FFT tables, tap history
 * and accumulators on the calling thread's current device.
 * Returns PFBS_ERR_INVALID for bad arguments (checked before any HIP call). */
pfbs_status pfbs_plan_create(pfbs_plan **out, int64_t N, int32_t P, int32_t window,
                             int32_t mode, int32_t n_pol, int64_t n_int);

/* Create a plan from a full description (see pfbs_plan_desc). */
pfbs_status pfbs_plan_create_ex(pfbs_plan **out, const pfbs_plan_desc *desc);

/* Release every resource of the plan.  Waits for the plan's queued work.
 * NULL is accepted (no-op). */
pfbs_status pfbs_plan_destroy(pfbs_plan *plan);

/* Number of complete dumps that pfbs_execute would emit for the next block of
 * n_time_samples samples (host arithmetic from the plan's counters; no device
 * call).  Returns -1 if n_time_samples is not a positive multiple of N. */
int64_t pfbs_dumps_in(const pfbs_plan *plan, int64_t n_time_samples);

/* Process one block of the stream (Section 4, loop: pre-filter, parallel FFTs,
 * accumulate).
 *   d_block        : device, int8 [n_time_samples][n_pol][2], 16-byte aligned,
 *                    read only, must stay valid until the stream reaches the
 *                    work;
 *   n_time_samples : a positive multiple of N;
 *   d_dumps        : device, float [dump_capacity][n_prod][N] with n_prod = 1
 *                    (one polarisation) or 4 (|X|^2, |Y|^2, Re XY*, Im XY*),
 *                    product-major, channels in natural order; may be NULL
 *                    when no dump completes;
 *   dump_capacity  : dumps the buffer can hold; must be >= pfbs_dumps_in();
 *   n_dumps_written: host, set to the number of dumps this call writes
 *                    (known at return, no synchronisation);
 *   stream         : hipStream_t (NULL = default stream).
 * Dumps not yet complete stay in the plan's accumulators and continue with
 * the next block. */
pfbs_status pfbs_execute(pfbs_plan *plan, const void *d_block, int64_t n_time_samples,
                         float *d_dumps, int64_t dump_capacity, int64_t *n_dumps_written,
                         void *stream);

/* pfbs_execute for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results (bit for bit) and errors as pfbs_execute, but the plan's
 * own intermediate and partial-sum buffers are not used or grown: the work
 * goes through one fixed scratch array of 128 MiB per device (a file-scope
 * device array of the library, held by every device the library runs on
 * until the process ends), and the call makes no hipMalloc, hipFree or other
 * allocating call (kernel timing is skipped).  A block whose partial sums
 * (4 * n_prod * N bytes per chunk of spectra it touches) plus one chunk of
 * the two-pass intermediate (8 * n_pol * N bytes per spectrum of a chunk) do
 * not fit in 128 MiB is rejected with PFBS_ERR_INVALID before anything is
 * queued (use smaller blocks, or a smaller chunk in the plan).  The scratch
 * array is shared by every such call on one device and keeps the last
 * call's contents; each call writes what it reads, so nothing needs clearing,
 * but calls that overlap on one device (other streams, other plans or
 * threads) race on it and must be serialised by the caller. */
pfbs_status pfbs_execute_noalloc(pfbs_plan *plan, const void *d_block, int64_t n_time_samples,
                                 float *d_dumps, int64_t dump_capacity, int64_t *n_dumps_written,
                                 void *stream);

/* Write the partial integration (spectra accumulated since the last dump) to
 * d_partial (device, float [n_prod][N]) and its spectrum count to *n_spectra
 * (host).  The plan's state is unchanged. */
pfbs_status pfbs_flush(pfbs_plan *plan, float *d_partial, int64_t *n_spectra, void *stream);

/* Forget the stream: clear the tap history, accumulators and counters, and
 * clear the poisoned flag.  Synchronises with the plan's device. */
pfbs_status pfbs_plan_reset(pfbs_plan *plan);

/* Test hook: the FP32 pre-filter output y_j[n] of the spectra that the next
 * block would complete, without changing the plan.  d_y: device,
 * float [n_spectra][n_pol][N][2]; *n_spectra (host) receives the count.
 * A kernel of its own: it shares the frame addressing (block or tap history)
 * and the per-tap multiply-add with the kernels of pfbs_execute, in the same
 * tap order, but not their tile addressing; the production kernels' indexing
 * is checked through pfbs_execute itself (one-hot taps against direct mode). */
pfbs_status pfbs_debug_pfb(pfbs_plan *plan, const void *d_block, int64_t n_time_samples,
                           float *d_y, int64_t y_capacity_spectra, int64_t *n_spectra,
                           void *stream);

/* Test hook: copy the plan's FP32 filter taps h[P*N] to d_out (device). */
pfbs_status pfbs_debug_taps(pfbs_plan *plan, float *d_out, void *stream);

/* Test hook: copy one of the plan's device tables (all generated on the
 * device in FP64 and rounded once, Section 4 initialisation) to d_out
 * (device, capacity_bytes long); *bytes (host) receives its size, 0 when the
 * plan has no such table (then nothing is copied).  With d_out NULL only the
 * size is returned.  Tables:
 *   TAPS        : float h[P*N];
 *   TW_FIRST    : float2 radix-16 pass twiddles of the single pass or column
 *                 pass, W_(16 Ns)^(k r) for k < Ns, r = 1..15, passes
 *                 Ns = r0, 16 r0, ... concatenated (r0 = L / 16^floor(log16 L));
 *   TW_ROWS     : the same for the row pass of the two-pass FFT;
 *   TW_ROWS_F64 : double2, the same in FP64 (FP64 row pass only);
 *   TW_STEP     : float2 four-step twiddles, [n1][k2] = W_N^(n1 k2);
 *   MFMA        : the matrix-core DFT-16 operands, 64 lanes x 4 x 16 bytes. */
#define PFBS_TABLE_TAPS 0
#define PFBS_TABLE_TW_FIRST 1
#define PFBS_TABLE_TW_ROWS 2
#define PFBS_TABLE_TW_ROWS_F64 3
#define PFBS_TABLE_TW_STEP 4
#define PFBS_TABLE_MFMA 5
pfbs_status pfbs_debug_table(pfbs_plan *plan, int32_t which, void *d_out, int64_t capacity_bytes,
                             int64_t *bytes, void *stream);

/* Read-only plan facts for callers and tests (host, no device call). */
typedef struct {
    int64_t N;
    int32_t P, n_pol, n_prod, mode, precision, chunk;
    int64_t n_int;
    int64_t split_n1, split_n2;     /* split_n1 == 1: single-pass FFT          */
    int64_t frames_seen;            /* frames consumed so far                  */
    int64_t spectra_done;           /* valid spectra produced so far           */
    int64_t dumps_done;             /* dumps emitted so far                    */
    int64_t device_bytes;           /* device memory held by the plan          */
    int32_t row_arith;              /* arithmetic of the row pass of the two-pass
                                       FFT: 0 FP32, 1 FP16 matrix cores, 2 split
                                       FP16 matrix cores, 3 FP64 (FP32 plans from
                                       2^18 channels); -1 for a single-pass FFT */
    int32_t row_tile;               /* row-pass tile points per polarisation (0 for
                                       N <= 4096) */
} pfbs_plan_info;

pfbs_status pfbs_plan_get_info(const pfbs_plan *plan, pfbs_plan_info *info);

/* Kernel timing.  With enable != 0 every kernel launch that pfbs_execute makes
 * for this plan records its start and stop timestamps into a pair of HIP
 * events through the dispatch itself (hipExtLaunchKernel), so timing adds no
 * packets to the stream.  pfbs_plan_timing_read waits for those events, adds
 * their elapsed times (ms) and launch counts per kernel kind into ms[kind] /
 * launches[kind] for kind < n (kinds: 0 single-pass, 1 column pass, 2 row
 * pass, 3 dump reduction and output form, 4 tap history; PFBS_KERNEL_KINDS in
 * all), and forgets them. */
#define PFBS_KERNEL_KINDS 5
pfbs_status pfbs_plan_timing(pfbs_plan *plan, int32_t enable);
/* The same for a subset of kinds: bit k of `kinds` times kind k (0 = off). */
pfbs_status pfbs_plan_timing_kinds(pfbs_plan *plan, uint32_t kinds);
pfbs_status pfbs_plan_timing_read(pfbs_plan *plan, double *ms, int64_t *launches, int32_t n);

/* Autotuner.  Times candidate settings of the speed-only fields for the plan
 * shape in *desc on its device: split_n2 (the radix split of the two-pass
 * FFT, limited to splits that keep the precision's accuracy: rows no longer
 * than the default split's, or any split where the rows run in FP64),
 * col_pair (column-pass workgroups of one or two spectra: 8 or 16 waves),
 * tap_unroll, row_tile (row-pass tile width, hence waves per workgroup),
 * chunk, col_run and stream_z.  The search is coordinate-wise: each field in
 * turn over its values, the others at their best so far, starting from the
 * plan's automatic choices.  Each candidate runs on the same synthetic stream
 * of device blocks of block_samples time samples (a positive multiple of N;
 * 0 = 2^24; as many distinct blocks as make at least 512 MB, at most 16, so
 * the input streams from HBM and not from the caches), timed with HIP events
 * around three passes over them after one untimed pass (and the starting
 * point run once, untimed, before any candidate is timed, so the device has
 * settled).  Writes the fastest into *best (a copy of
 * *desc with those fields set and tune = 0) and its throughput in complex
 * samples per second into *best_samples_per_s (may be NULL).  At most
 * max_candidates settings are timed (0 = all).  If the environment variable
 * PFBS_TUNE_CACHE names a file, the result is appended to it as one text line
 *   pfbs-tune-v4 <arch> <version> N P mode n_pol n_int precision block split_n2 chunk col_run stream_z tap_unroll col_pair row_tile samples_per_s
 * (version: the source digest of pfbs_version, so a rebuilt library with
 * changed kernels does not reuse old measurements)
 * and later plans created with tune != 0 reuse the newest matching line.
 * Synchronous; allocates device memory for the blocks and the trial plans. */
pfbs_status pfbs_autotune(const pfbs_plan_desc *desc, int64_t block_samples, int32_t max_candidates,
                          pfbs_plan_desc *best, double *best_samples_per_s);

/* Human-readable detail of the calling thread's last failure ("" if none). */
const char *pfbs_last_error(void);

/* Library version: "pfbspec <digest of the sources it was built from>". */
const char *pfbs_version(void);

/* Batched form: several independent sub-band streams (each with its own N, P,
 * mode, n_int, precision and state) processed by three launches per block,
 * in the eight-sub-band spirit of the paper's 16 parallel FFTs (Section 4,
 * initialisation) and its remark on per-batch launch overhead (Section 5):
 * the front phase (every sub-band's single pass or column pass, with its
 * pre-filter), the row phase (every row pass) and the tail (dump reductions
 * and tap histories).  Each workgroup runs the same device code as the
 * sub-band's own plan, so every sub-band's dumps are bitwise those of
 * pfbs_execute on a plan made from the same description.
 *   descs: host array of n (1..64) plan descriptions, all with the same
 *          n_pol, precision FP32 or MIXED, output PRODUCTS, fftshift 0
 *          (others: PFBS_ERR_UNSUPPORTED).                                  */
pfbs_status pfbs_batch_create(pfbs_batch **out, const pfbs_plan_desc *descs, int32_t n);

/* One block per sub-band: d_blocks[i] (device) holds n_time_samples[i]
 * samples for sub-band i; d_dumps[i] / caps[i] / n_dumps[i] as in
 * pfbs_execute.  The per-block work tables go to the device with one
 * asynchronous copy on a stream of the batch, from page-locked staging
 * memory, while `stream` still runs earlier blocks (a ring of four buffers:
 * the host waits only for the copy of four executes back).  With
 * use_graph != 0 the three launches are captured once in a HIP graph (on the
 * batch's own stream; recaptured when the block sizes change) and replayed
 * on `stream`, with workgroup counts for the largest work those block sizes
 * can bring (the surplus workgroups exit at once). */
pfbs_status pfbs_batch_execute(pfbs_batch *b, const void *const *d_blocks,
                               const int64_t *n_time_samples, float *const *d_dumps,
                               const int64_t *caps, int64_t *n_dumps, int32_t use_graph,
                               void *stream);

/* Kernel launches (or graph kernel nodes) of the batch's last execute: at
 * most 3.  -1 if b is not a live batch. */
int32_t pfbs_batch_launches(const pfbs_batch *b);

/* Release the batch and the plans it owns.  NULL is accepted. */
pfbs_status pfbs_batch_destroy(pfbs_batch *b);

/* The plan of sub-band i of a batch (owned by the batch), or NULL. */
pfbs_plan *pfbs_batch_plan(pfbs_batch *b, int32_t i);

/* Page-locked host memory (hipHostMalloc) of `bytes` bytes, for blocks and
 * dumps that travel asynchronously; release with pfbs_host_free (NULL is
 * accepted there). */
pfbs_status pfbs_host_alloc(void **out, int64_t bytes);
pfbs_status pfbs_host_free(void *p);

/* Host-fed streaming (the paper's per-block loop of copy in, compute, copy
 * out, Section 4 algorithm list, with the copies overlapped by streams as
 * its Section 5 suggests): a plan plus `depth` (2..16) device slots, each a
 * block buffer of max_block_samples time samples and a dump buffer, and
 * three streams (copy in, compute, copy out) chained by events, so that block
 * i+1 crosses PCIe while block i is computed.  The plan's device state and
 * rules are those of pfbs_plan_create_ex(desc). */
pfbs_status pfbs_hstream_create(pfbs_hstream **out, const pfbs_plan_desc *desc, int64_t max_block_samples,
                                int32_t depth);

/* Queue one block and return at once.
 *   h_block        : host, int8 [n_time_samples][n_pol][2]; page-locked
 *                    memory (pfbs_host_alloc) makes the copy asynchronous;
 *                    must stay unchanged until the push has completed;
 *   n_time_samples : a positive multiple of N, at most max_block_samples;
 *   h_dumps        : host, float [dump_capacity][n_prod][N], receives this
 *                    block's dumps (as pfbs_execute writes them); valid once
 *                    the push has completed; may be NULL when none complete;
 *   n_dumps_written: host, set at return.
 * A push has completed after pfbs_hstream_sync, or once `depth` later pushes
 * have returned (a push waits on the host for the slot it reuses). */
pfbs_status pfbs_hstream_push(pfbs_hstream *s, const void *h_block, int64_t n_time_samples, float *h_dumps,
                              int64_t dump_capacity, int64_t *n_dumps_written);

/* Wait until every queued push has completed. */
pfbs_status pfbs_hstream_sync(pfbs_hstream *s);

/* Wait for the queued work, then release everything (the plan too).  NULL
 * is accepted. */
pfbs_status pfbs_hstream_destroy(pfbs_hstream *s);

/* The plan inside a host stream (owned by it), or NULL. */
pfbs_plan *pfbs_hstream_plan(pfbs_hstream *s);

#ifdef __cplusplus
}
#endif

#endif /* PFBSPEC_H */
