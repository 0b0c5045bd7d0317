/*
 * rx.h -- C ABI of the MI355X streaming global-RX anomaly scorer.
 *
 * What is computed (paper: Section "System Implementation / Detection
 * Algorithm", Eq. 1): every band is a variable and every pixel a sample; the
 * band mean mu and the B x B covariance Sigma are taken over all pixels of
 * the statistics window (pixels being scored included), and each pixel
 * spectrum s scores
 *       delta = (s - mu)^T Sigma^{-1} (s - mu)
 * (squared Mahalanobis distance).  A threshold marks pixels above a
 * configurable value (same section; the flights use 0.110 of the per-set
 * maximum).  Lines arrive from a push-broom sensor (Section "System
 * Architecture / Data Acquisition"); they are pushed in blocks.  Each block
 * first joins the statistics window and is then scored with the updated
 * statistics (the line-based form the paper proposes in Section
 * "Discussion / Performance"; one block = one 1000-line cube with a
 * 1000-line window reproduces the paper's per-cube detector).
 *
 * Numerics: the statistics are a streaming merge of per-block centred
 * scatter matrices (covariance product on matrix cores in the configured
 * precision, FP32 centring, FP64 merge); the optional ridge, equilibration,
 * Cholesky factorisation and triangular inverse run in FP64 on the GPU;
 * whitening y = W (x - mu) with W^T W = (Sigma + lambda I)^{-1} runs on
 * matrix cores in the configured precision with FP32 accumulation (FP64 on
 * the plain FP64 path), and delta = |y|^2.
 *
 * Conventions for every entry point:
 *  - Returns rx_status; nothing throws, aborts or exits.  On a non-OK status
 *    rx_last_error() returns a thread-local message describing it.
 *  - The caller owns every buffer it passes; the library never frees them.
 *    The library owns all device state behind an rx_stream / rx_server and
 *    frees it in rx_destroy / rx_server_destroy.
 *  - Calls on one rx_stream must be serialised by the caller; different
 *    streams may be driven from different threads.
 *  - hip_stream arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  The library orders its work after everything already
 *    enqueued on hip_stream and, for device outputs, makes hip_stream wait
 *    for the result; it never blocks the host except where stated.
 */
#ifndef RX_H_
#define RX_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rx_stream rx_stream;   /* one sensor stream; opaque, library-owned */
typedef struct rx_server rx_server;   /* many streams sharing one GPU; opaque */

typedef enum {
  RX_OK = 0,
  RX_E_ARG = -1,       /* bad size, enum, null pointer or struct_size */
  RX_E_NOMEM = -2,     /* device or pinned-host allocation failed */
  RX_E_NOTREADY = -3,  /* window holds N <= B pixels and no ridge: Sigma is singular; scores NaN */
  RX_E_SINGULAR = -4,  /* non-positive pivot in the FP64 Cholesky; that block's scores are NaN */
  RX_E_DEVICE = -5,    /* a HIP runtime call failed */
  RX_E_BUDGET = -6,    /* server: admission refused by the HBM budget or stream-slot limit */
  RX_E_STATE = -7      /* call on a destroyed object or in the wrong order */
} rx_status;

typedef enum { RX_IN_U16 = 0, RX_IN_F32 = 1, RX_IN_F64 = 2 } rx_in_type;
/* Layout of pushed lines.  RX_BIL: band-interleaved by line [line][band][sample], what the
 * push-broom imager delivers (paper, Section "System Implementation / Data Acquisition") and
 * what the kernels read.  RX_BIP: band-interleaved by pixel [line][sample][band]; each push is
 * first transposed into a library-owned BIL copy (one extra read and write of the lines on the
 * device; the scores are bit for bit those of the same lines pushed as BIL).  Served streams
 * take BIL blocks only. */
typedef enum { RX_BIL = 0, RX_BIP = 1 } rx_layout;

/* Where rx_push_lines' lines are (its is_device_ptr argument). */
enum { RX_LINES_HOST = 0, RX_LINES_DEVICE = 1, RX_LINES_RESIDENT = 2 };

typedef enum { RX_FP64 = 0, RX_FP32 = 1, RX_BF16 = 2, RX_FP16 = 3, RX_FP8_E4M3 = 4 } rx_prec;
typedef enum { RX_THR_ABS = 0, RX_THR_REL_MAX = 1, RX_THR_TOPK = 2 } rx_thr_mode;

#define RX_MAX_BANDS 320

typedef struct rx_config {
  uint32_t struct_size;   /* must be sizeof(rx_config) (ABI versioning) */
  int32_t bands;          /* B, 1 .. RX_MAX_BANDS */
  int32_t samples;        /* S >= 1 samples (pixels) per line */
  int32_t in_type;        /* rx_in_type of the pushed values */
  int32_t bit_depth;      /* u16 input: values must be < 2^bit_depth (informational), 0 = 16 */
  int32_t layout;         /* rx_layout: RX_BIL or RX_BIP (not for served streams) */
  int32_t syrk_prec;      /* covariance-product precision: FP64, FP32, BF16, FP16 or FP8_E4M3.
                             FP8: each block's centred values are scaled per band by 2^-e
                             (e from the block's first line: its largest deviation from the
                             shift lands at or below 224, half the format's range), rounded
                             to E4M3, multiplied with FP32 accumulation and scaled back
                             exactly; larger values saturate at 448 and are counted */
  int32_t whiten_prec;    /* whitening precision: FP64, FP32, BF16, FP16 or FP8_E4M3 */
  int32_t ddof;           /* covariance normaliser 1/(N - ddof); 0 (default) or 1 */
  int32_t block_lines;    /* 0: each push is one block; >0: pushes are cut into blocks of at
                             most this many lines (the last block of a push may be shorter) */
  int64_t window_lines;   /* 0: cumulative window; R > 0: statistics restart every R lines
                             (blocks never straddle a window edge; 1000 = the paper's cube) */
  double ridge_rel;       /* rho >= 0: lambda = rho * trace(Sigma) / B is added to the diagonal */
  int32_t device;         /* HIP device ordinal */
  int32_t flags;          /* 0, RX_FLAG_CAUSAL or RX_FLAG_ONE_PASS; other bits must be 0 */
} rx_config;

/* rx_config.flags: causal scoring.  Every block is scored with the window
 * as it was before the block joined it (the paper scores a cube with
 * statistics that include it, Section "System Implementation / Detection
 * Algorithm"; the line-based detector it proposes, Section "Discussion /
 * Performance", may instead score new lines against the lines already seen).
 * A block that starts a window (the first block, or a reset) then has no
 * statistics: its scores are NaN and it counts as not ready; so does a block
 * whose earlier window holds N <= B pixels without a ridge.  The scores of
 * a one-block push of 16-bit device input then do not wait for that block's
 * own statistics update (it runs alongside).  Default off: update, then
 * score. */
#define RX_FLAG_CAUSAL 1

/* rx_config.flags: one-pass scoring.  Every block of a push is scored with
 * the window as it was before the push (with one block per push this is the
 * causal reading above, the line-based detector of Section "Discussion /
 * Performance"; the blocks of a longer push are scored together, as the
 * paper scores a cube as one unit).  The statistics still take every block,
 * and a block whose window started inside the push, at or before it, has no
 * earlier statistics: NaN scores, not ready.  16-bit input with 16-byte
 * aligned rows, S % 8 == 0, at most 272 bands and BF16 covariance and
 * whitening products then reads every line once: one kernel stages each
 * chunk of lines, whitens and scores it with the window before the push and
 * adds it to the covariance product (Section "System Implementation /
 * Detection Algorithm", Eq. 1).  Other configurations, a push whose window
 * before it is formed in the push (the first push, after rx_set_stats) and
 * served streams (each submitted block is a push of its own) take the same
 * scores from the two-pass kernels.  Not with RX_FLAG_CAUSAL. */
#define RX_FLAG_ONE_PASS 2

typedef struct rx_counters {
  int64_t lines_pushed;     /* lines accepted so far */
  int64_t blocks;           /* blocks processed */
  int64_t singular_blocks;  /* blocks whose factorisation hit a non-positive pivot */
  int64_t notready_blocks;  /* blocks scored while N <= B without a ridge (or N <= ddof) */
  int64_t pending_px;       /* scores produced and not yet consumed by rx_scores */
  int64_t window_px;        /* N, pixels in the statistics window (finite pixels only) */
  int64_t nonfinite_px;     /* float input: pixels with a NaN or infinite band (left out of the
                               statistics, scored NaN, never marked) */
  int64_t fp8_saturated;    /* FP8 E4M3 whitening: centred, band-scaled input values beyond the
                               format's range (|v| > 464), stored as +-448 */
  int64_t fp8_syrk_saturated; /* FP8 E4M3 covariance product: centred, band-scaled values beyond
                               the format's range (|v| > 464), stored as +-448 */
} rx_counters;

/* Fill *cfg with defaults for B bands and S samples: u16 input, 12-bit,
 * BIL, BF16 covariance and whitening, ddof 0, one block per push,
 * cumulative window, no ridge, device 0.  RX_E_ARG on a null cfg. */
rx_status rx_config_init(rx_config* cfg, int32_t bands, int32_t samples);

/* Create a stream: one push-broom sensor whose lines arrive continuously
 * (paper, Section "System Architecture / Data Acquisition") and whose
 * statistics window starts empty (Section "System Implementation / Detection
 * Algorithm": mean and covariance over the set of pixels).  server may be
 * NULL (stand-alone stream); otherwise the stream is admitted by the
 * server's HBM budget (RX_E_BUDGET if it does not fit or every slot is
 * taken).  Allocates the stream's resident state (window band sums and
 * scatter matrix in FP64) on cfg->device.  *out receives the handle (NULL on
 * failure); RX_E_ARG for a bad config, RX_E_NOMEM / RX_E_DEVICE when the
 * device refuses. */
rx_status rx_init(const rx_config* cfg, rx_server* server, rx_stream** out);

/* Push n_lines >= 1 lines, BIL [n_lines][B][S] (or BIP [n_lines][S][B] with
 * cfg->layout = RX_BIP) of cfg->in_type, contiguous.
 * is_device_ptr = RX_LINES_HOST (0): lines is host memory, copied before the
 * call returns (the caller may reuse it at once): up to eight threads copy
 * it in 8 MiB chunks into the stream's pinned buffers (two per thread, 16
 * MiB each thread), and each chunk's transfer to the device overlaps the
 * copies of later chunks.  RX_LINES_DEVICE (1):
 * lines is device memory on cfg->device, read asynchronously after the work
 * already queued on hip_stream; it must stay unchanged until rx_sync returns
 * or hip_stream passes an rx_wait on this stream.  RX_LINES_RESIDENT (2):
 * device memory whose contents are complete when the call is made (written
 * by work the caller has already synchronised with); the push orders itself
 * against no stream (hip_stream is ignored), which leaves the caller's
 * streams out of the stream's queues; the same lifetime rule as
 * RX_LINES_DEVICE.  Any other value: RX_E_ARG.
 * The lines are cut into blocks (cfg->block_lines, window edges); each block
 * updates the statistics and is then scored.  Scores join the stream's
 * pending FIFO in pixel order (p = line * S + sample).  Asynchronous.
 * RX_E_NOTREADY when a block is scored with N <= B and no ridge (its scores
 * are NaN, the statistics are still updated).
 * Float input: a pixel with any NaN or infinite band is left out of the
 * statistics (N counts finite pixels only), scores NaN and is counted in
 * rx_counters.nonfinite_px; the paper is silent on such input (Section
 * "System Implementation / Detection Algorithm" takes every pixel).  The
 * NOTREADY return above counts pushed pixels; blocks that non-finite pixels
 * leave not ready are found on the device (NaN scores, notready_blocks). */
rx_status rx_push_lines(rx_stream* s, const void* lines, int64_t n_lines, int32_t is_device_ptr,
                        void* hip_stream);

/* Pop up to max_px of the oldest pending scores (FP32) into out: the
 * per-pixel RX score delta of Eq. 1 (paper, Section "System Implementation /
 * Detection Algorithm"), in FP32 as the paper's ground station receives it
 * (Section "System Implementation / Data Transmission").
 * out_is_device = 0: host buffer, the call blocks until they are written.
 * out_is_device = 1: device buffer on cfg->device, written asynchronously
 * after the work already queued on hip_stream (which may still be using the
 * buffer) and ordered before later work on hip_stream.  *n_written = count
 * popped. */
rx_status rx_scores(rx_stream* s, float* out, int64_t max_px, int64_t* n_written,
                    int32_t out_is_device, void* hip_stream);

/* As rx_scores but FP64; on the plain FP64 path (whiten_prec = RX_FP64) these
 * are the FP64 scores, otherwise the FP32 scores widened. */
rx_status rx_scores_f64(rx_stream* s, double* out, int64_t max_px, int64_t* n_written,
                        int32_t out_is_device, void* hip_stream);

/* Threshold mask over all pending scores, without consuming them.
 * mode RX_THR_ABS: delta > tau.  RX_THR_REL_MAX: delta > tau * max(pending)
 * (the paper's normalised threshold, e.g. tau = 0.110).  RX_THR_TOPK: the k
 * largest pending scores, ties to the lower pixel index.  NaN scores are
 * never marked.  Bit j of byte q is pending pixel 8q + j; ceil(n/8) bytes are
 * written (max_bytes must be at least that).  *n_px = pending pixels covered.
 * out_is_device as in rx_scores. */
rx_status rx_mask(rx_stream* s, double tau, int32_t mode, int64_t k, uint8_t* bits,
                  int64_t max_bytes, int64_t* n_px, int32_t out_is_device, void* hip_stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: rx_mask
 * with a device output that allocates nothing.  Same modes, tau, k, bit
 * order and NaN rule as rx_mask; bits is a device pointer on the stream's
 * device (any alignment, at least ceil(n/8) bytes = max_bytes), written after
 * the work already queued on hip_stream and ordered before later work on it.
 * Its working memory (maximum key, top-k state and histogram, the mask words
 * before they are copied to bits) is one fixed device array of
 * RX_MASK_NOALLOC_BYTES per GPU, located by rx_init on that GPU and held
 * until the process ends; the pending set may hold at most
 * RX_MASK_NOALLOC_MAX_PX pixels (RX_E_ARG beyond, nothing queued).  Every
 * call on one GPU shares that array and it keeps the last call's contents:
 * calls that overlap on one GPU (different rx_streams, or different host
 * threads, whose work is not ordered on the device) race and must be
 * serialised by the caller.  The stream itself (rx_init, rx_push_lines)
 * still allocates as usual; only this call does not. */
#define RX_MASK_NOALLOC_BYTES (4096 + (1 << 20))
#define RX_MASK_NOALLOC_MAX_PX (1 << 23)
rx_status rx_mask_noalloc(rx_stream* s, double tau, int32_t mode, int64_t k, uint8_t* bits, int64_t max_bytes,
                          int64_t* n_px, void* hip_stream);

/* ---------------------------------------------------------------- ingest binning
 * Band selection and spectral binning of 16-bit counts (paper, Section
 * "System Implementation / Data Acquisition": out-of-range bands discarded,
 * 300 -> 280, then four consecutive bands summed into one, 280 -> 70).  For a
 * BIL cube in [lines][bands][samples]:
 *   out[l][j][s] = sum over t < k of in[l][b0 + j k + t][s],  j < nb / k,
 * exact integer sums written as uint16 to out [lines][nb / k][samples].
 * in and out are device pointers on the current device (not overlapping);
 * the work is queued on hip_stream.  RX_E_ARG unless 1 <= k <= nb,
 * nb % k == 0, 0 <= b0, b0 + nb <= bands, 1 <= bit_depth <= 16 and
 * k (2^bit_depth - 1) <= 65535 (so no sum can overflow); nothing is written
 * then.  The binned cube is then pushed like any other (bands = nb / k). */
rx_status rx_bin_bands(const uint16_t* in, int64_t lines, int32_t bands, int32_t samples, int32_t b0,
                       int32_t nb, int32_t k, int32_t bit_depth, uint16_t* out, void* hip_stream);

/* ---------------------------------------------------------------- transmission
 * The sender's score encoding and the receiver's inverse (paper, Section
 * "System Implementation / Data Transmission" and "... / Ground Control
 * Station"; the 0.110 threshold of Section "Results / Detector Visual
 * Analysis").  Sender: s_p = sqrt(delta_p) in FP32, m = the largest s_p (so
 * m = sqrt(max delta); NaN scores are skipped, m = 0 when none is finite),
 * code_p = binary16(s_p / m) rounded to nearest even: the cube's highest
 * score codes as 1.0; with m = 0 finite scores code as 0; NaN scores code
 * as a binary16 NaN.  Scores are expected to be >= 0 (a negative one codes
 * as NaN).  Receiver: h_p = the binary16 value, delta^_p = (h_p m)^2 in FP32
 * (the normalisation undone, then squared), and the relative threshold bit
 * h_p^2 > tau (h_p^2 is exact in FP32).
 *
 * rx_tx_encode: scores [n] FP32, codes [n] (binary16 bit patterns) and
 * max_out (one FP32, 4-byte aligned) are device pointers on the current
 * device; the work is queued on hip_stream (NULL: the null stream).  max_out
 * holds an intermediate key while the call's work runs and m once it is done.
 * rx_tx_decode: codes [n] and max_in (m, as written by rx_tx_encode) are
 * device pointers; delta [n] (FP32) and bits (ceil(n/32) 32-bit words,
 * 4-byte aligned; bit j of byte q is pixel 8q + j, as in rx_mask) are
 * device pointers or NULL to skip that output.  Both return RX_E_ARG for
 * n < 0, a NaN tau, or a missing or misaligned pointer; nothing is written
 * then. */
rx_status rx_tx_encode(const float* scores, int64_t n, uint16_t* codes, float* max_out, void* hip_stream);
rx_status rx_tx_decode(const uint16_t* codes, int64_t n, const float* max_in, float tau, float* delta,
                       uint32_t* bits, void* hip_stream);

/* rx_tx_encode over the stream's pending scores, without consuming them
 * (the transmitted set of the paper's cube is the pending set, as for
 * rx_mask).  codes (at least the pending count) and max_out are device
 * pointers on the stream's device; they are written after the work already
 * queued on hip_stream and before later work on it.  *n_px = pending pixels encoded.  FP64 scores of the plain
 * FP64 path are rounded to FP32 first. */
rx_status rx_encode(rx_stream* s, uint16_t* codes, int64_t max_px, int64_t* n_px, float* max_out,
                    void* hip_stream);

/* Make hip_stream wait for every block pushed so far (no host block). */
rx_status rx_wait(rx_stream* s, void* hip_stream);

/* Block the host until every block pushed so far is done.  Returns the
 * first sticky error raised by the device since the previous rx_sync
 * (RX_E_SINGULAR) and clears it. */
rx_status rx_sync(rx_stream* s);

/* Counters (blocks the host, like rx_sync, without clearing errors). */
rx_status rx_get_counters(rx_stream* s, rx_counters* out);

/* Destroy a stream: its statistics window ends with it, as a cube's
 * distribution serves only that cube's pixels (paper, Section "System
 * Implementation / Detection Algorithm": each cube is an independent
 * entity).  Waits for its work, frees its device memory, and releases its
 * server admission (the HBM it was charged returns to the budget).  NULL is
 * accepted (no-op); RX_E_STATE for a handle that is not live (already
 * destroyed). */
rx_status rx_destroy(rx_stream* s);

/* Thread-local message for the last non-OK status on this thread. */
const char* rx_last_error(void);

/* Checkpoint/restore hooks.  rx_get_stats blocks, then writes the window
 * count N (pixels in the statistics: finite pixels only for float input),
 * the mean [B] and the covariance M2/(N - ddof) [B][B] (row-major,
 * full symmetric); mean and cov may be NULL.  rx_set_stats replaces the
 * window with (n, mean, cov): the scatter matrix becomes cov * (n - ddof). */
rx_status rx_get_stats(rx_stream* s, int64_t* n, double* mean, double* cov);
rx_status rx_set_stats(rx_stream* s, int64_t n, const double* mean, const double* cov);

/* Phase timing for measurement: with enable = 1, every later push records a
 * pair of HIP events on the stream the kernels run on around each phase
 * (0 centring shift, 1 covariance product, 2 statistics merge, 3 FP64
 * factorisation, 4 whitening + score; a one-pass kernel, covariance product
 * and scores together, counts as 1).  rx_phase_times blocks, then writes the
 * accumulated milliseconds ms[5] and launch counts launches[5] since the
 * last rx_profile call (which also resets them). */
rx_status rx_profile(rx_stream* s, int32_t enable);
rx_status rx_phase_times(rx_stream* s, double* ms, int64_t* launches);

/* Test hook (host only, no device work): how the covariance product of a
 * block of `lines` lines under cfg is cut into splits (independent partial
 * products summed in a fixed order, Section "System Implementation /
 * Detection Algorithm": the covariance over the block's pixels).
 * *splits = the number of splits, *max_chunks = the most 64-sample line
 * chunks one split holds.  For 16-bit input each split's exact raw band sums
 * are 32-bit per thread, 8 values per chunk: the plan keeps
 * 8 * 65535 * max_chunks < 2^32 for any block length.  RX_E_ARG for a bad
 * config, lines outside [1, 2^31 - 1] or a null output. */
rx_status rx_split_plan(const rx_config* cfg, int64_t lines, int32_t* splits, int64_t* max_chunks);

/* Test hook: the FP64 whitening factor W (lower triangular, [B][B]
 * row-major, W^T W = (Sigma + lambda I)^{-1}) of the most recent block. */
rx_status rx_get_whitener(rx_stream* s, double* w);

/* ---------------------------------------------------------------- serving
 * A server admits many streams on one GPU under an HBM budget and runs their
 * blocks together: rx_server_submit queues a block for a stream (device
 * lines; the server copies nothing), rx_server_step launches every queued
 * block of every stream in one batched pass (one launch per kernel and
 * precision group), and completions are reported with their arrival stamps
 * so latency can be measured.  A stream's result is the same alone and in
 * any mix (bit-identical: no reduction depends on the batch composition). */
rx_status rx_server_create(size_t hbm_budget_bytes, int32_t max_streams, int32_t device,
                           rx_server** out);
rx_status rx_server_destroy(rx_server* srv);

/* Bytes of device memory a stream with this config reserves when its blocks
 * have at most max_block_lines lines (the admission charge; a served stream
 * takes blocks of at most cfg->block_lines lines, 128 when that is 0). */
rx_status rx_stream_footprint(const rx_config* cfg, int32_t max_block_lines, size_t* bytes);

/* Queue one block of n_lines (<= the stream's block limit) device lines for
 * a stream admitted on srv.  The lines must stay unchanged until the block
 * is reported done by rx_server_poll.  tag is returned on completion.  A
 * block must not straddle a window edge (RX_E_ARG at step time). */
rx_status rx_server_submit(rx_server* srv, rx_stream* s, const void* lines_dev, int64_t n_lines, uint64_t tag);

/* Launch the oldest queued block of every stream that has one, all in one
 * batched pass (statistics, factorisations and whitening of every stream
 * in shared launches).  Asynchronous; *n_blocks = blocks launched.  The
 * server runs a step over three HIP queues (statistics; factorisation;
 * whitening), so one step's statistics overlap the previous step's
 * factorisation and whitening. */
rx_status rx_server_step(rx_server* srv, int32_t* n_blocks);

/* Report finished blocks in launch order: up to max_tags tags are written.
 * block = 0 returns at once; block = 1 waits for every launched block. */
rx_status rx_server_poll(rx_server* srv, uint64_t* tags, int32_t max_tags, int32_t* n_done, int32_t block);

/* Wait for every launched block. */
rx_status rx_server_sync(rx_server* srv);

/* Persistent request loop (the paper's stages run continuously on their own
 * cores, Section "System Implementation / Flight System"; here one library
 * thread per server).  rx_server_start starts a thread that, until
 * rx_server_stop, launches a batched step whenever blocks are queued and
 * fewer than two steps are in flight (blocks arriving meanwhile join the
 * next step: continuous batching), and stamps every finished block with
 * rx_clock_ns() as soon as its step's completion event is seen (within tens
 * of microseconds).  While it runs, rx_server_step returns RX_E_STATE and
 * rx_server_poll / rx_server_poll_ns return the blocks it has collected
 * (block = 1: after every queued and launched block has finished).  Calls
 * on the server's streams (rx_scores, rx_mask, ...) take the server's lock
 * and may be made from other threads.  rx_server_stop joins the thread and
 * returns the first error the loop met (launched blocks keep running; poll
 * or rx_server_sync to wait for them).  RX_E_STATE when already running /
 * not live. */
rx_status rx_server_start(rx_server* srv);
rx_status rx_server_stop(rx_server* srv);

/* As rx_server_poll, also writing each block's completion stamp (ns of
 * rx_clock_ns, taken by the request loop; 0 for blocks collected by a
 * direct poll without the loop) to done_ns[] when it is not NULL. */
rx_status rx_server_poll_ns(rx_server* srv, uint64_t* tags, int64_t* done_ns, int32_t max_tags, int32_t* n_done,
                            int32_t block);

/* The library's monotonic clock in nanoseconds (steady clock), for stamping
 * block arrivals on the same time base as rx_server_poll_ns. */
int64_t rx_clock_ns(void);

/* Queue depth, blocks in flight and admitted bytes (any pointer may be NULL). */
rx_status rx_server_queued(rx_server* srv, int32_t* queued, int32_t* inflight, size_t* used_bytes);

#ifdef __cplusplus
}
#endif

#endif /* RX_H_ */
