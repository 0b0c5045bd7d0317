// Host runtime behind include/rx.h: stream contexts, block splitting,
// batch descriptors, kernel sequencing, the pending-score FIFO, masks,
// checkpoint hooks and the multi-stream server.
//
// Per batch of blocks (one stream) the device work is five launches on one
// HIP stream:  shift -> covariance product -> merge -> FP64 factor ->
// whitening + score.  A server step packs one batch from each of many
// streams into the same five launches (up to MAXB batches per launch,
// grouped by input type and precision).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rx.h"
#include "rx_dev.h"

using namespace rxk;

extern "C" hipError_t rxk_launch_stats(int in_type, int prec, int phase, const LaunchSet* ls, int wg,
                                       const LaunchSet* ls2, int wg2, hipStream_t st);
extern "C" hipError_t rxk_launch_factor(int wprec, const LaunchSet* ls, int wg, hipStream_t st);
extern "C" hipError_t rxk_launch_copy_slot(const LaunchSet* ls, int nb, hipStream_t st);
extern "C" hipError_t rxk_launch_onepass(const LaunchSet* ls, int wg, int Bw, hipStream_t st);
extern "C" hipError_t rxk_launch_whiten(int in_type, int wprec, const LaunchSet* ls, int wg, int Bw,
                                        hipStream_t st);
extern "C" hipError_t rxk_launch_mask(const void* sc, int f64, int64_t n, int mode, double tau, int64_t k,
                                      uint32_t* bits, void* scratch, hipStream_t st);
extern "C" hipError_t rxk_launch_tx_encode(const void* sc, int f64, int64_t n, uint16_t* codes, float* mslot,
                                           hipStream_t st);
extern "C" hipError_t rxk_launch_bin(const uint16_t* in, uint16_t* out, int64_t lines, int bands, int samples, int b0,
                                     int nbo, int k, hipStream_t st);
extern "C" hipError_t rxk_launch_bip_to_bil(const void* in, void* out, int64_t lines, int bands, int samples, int esz,
                                            hipStream_t st);
extern "C" hipError_t rxk_launch_tx_decode(const uint16_t* codes, int64_t n, const float* mslot, float tau,
                                           float* delta, uint32_t* bits, hipStream_t st);

extern "C" hipError_t rxk_noalloc_scratch(void** ptr, size_t* head, size_t* bytes);
extern "C" hipError_t rxk_launch_copy_bytes(const void* a, void* b, int64_t n, hipStream_t st);
extern "C" hipError_t rxk_launch_zero_words(uint32_t* w, int64_t n, hipStream_t st);

static_assert(sizeof(LaunchSet) < 4000, "kernel-argument descriptor set too large");

// ---------------------------------------------------------------------------- errors
static thread_local std::string g_err;

static rx_status fail(rx_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPC(call)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(RX_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------- allocation-free mask
// Device address of the allocation-free mask's working memory on each GPU
// (a fixed device array in the whitening kernels' code object; each device
// holds its own copy at its own address), looked up once per device by
// rx_init with that device current.
static constexpr int kMaxDevices = 64;
static std::mutex g_na_mu;
static void* g_na_ptr[kMaxDevices] = {};
static size_t g_na_head = 0, g_na_bytes = 0;

static rx_status noalloc_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(RX_E_ARG, "device %d beyond the library's %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (g_na_ptr[dev]) return RX_OK;
  void* p = nullptr;
  size_t head = 0, bytes = 0;
  const hipError_t e = rxk_noalloc_scratch(&p, &head, &bytes);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(RX_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
  }
  g_na_ptr[dev] = p;
  g_na_head = head;
  g_na_bytes = bytes;
  return RX_OK;
}

// ---------------------------------------------------------------------------- device buffers
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct rx_stream;
static hipError_t sync_all(rx_stream* s);

// Grow a buffer owned by stream `owner` (NULL: nothing can be using it).
// Growing is rare (first push, a larger batch); the old buffer may still be
// read by work queued on any of the owner's queues (a served stream's queue is
// its server's), so those queues are drained first -- not the whole device,
// which would stall every other stream.
static rx_status dev_ensure(DevBuf& b, size_t bytes, rx_stream* owner) {
  if (bytes <= b.cap) return RX_OK;
  if (b.p) {
    if (owner) HIPC(sync_all(owner));
    HIPC(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  const size_t nb = std::max<size_t>(bytes, 256);
  if (hipMalloc(&b.p, nb) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RX_E_NOMEM, "hipMalloc(%zu bytes) failed", nb);
  }
  b.cap = nb;
  return RX_OK;
}

static void dev_free(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

// ---------------------------------------------------------------------------- geometry
static constexpr uint32_t kMagic = 0x52585354u;   // "RXST"
static constexpr int kSplitChunks = 64;            // pixel chunks per covariance split, 64x64 super-tile kernel
// Pixel chunks per covariance split, whole-triangle kernel (one workgroup per
// CU): 91 makes a 100-line block of 640 samples 11 splits, so 20 such blocks
// pushed together take one pass of 220 CUs and leave room for the 20
// factorisation workgroups of the previous push running beside them.
static constexpr int kSplitChunks2 = 91;
static constexpr int kMaxBlocksPerBatch = 64;      // reset bits are a 64-bit mask

static int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
static int pad16(int b) { return 16 * ceil_div(b, 16); }
static int pad32(int b) { return 32 * ceil_div(b, 32); }
static size_t in_elem_size(int t) { return t == RX_IN_U16 ? 2 : (t == RX_IN_F32 ? 4 : 8); }
// Splits depend only on the block (never on the batch), so a block's result
// is the same alone and in any batch.
static bool whole_triangle(int sp) { return sp == RX_BF16 || sp == RX_FP16 || sp == RX_FP8_E4M3; }
// The covariance kernels keep each split's raw band sums of 16-bit input as
// exact uint32 per thread, and a thread adds 8 values of at most 65535 per
// chunk: a split of at most kMaxChunksPerSplit chunks cannot wrap
// (8 * 65535 * 8192 = 4 294 901 760 < 2^32).  Splits are capped at
// kMaxSplits per block unless a block is so long that this would exceed that.
static constexpr int64_t kMaxChunksPerSplit = 8192;
static constexpr int kMaxSplits = 256;              // splits per block (about one per CU)
static int splits_for(int64_t lines, int cpl, int sp) {
  const int per = whole_triangle(sp) ? kSplitChunks2 : kSplitChunks;
  const int64_t nch = lines * cpl;
  const int64_t cap = std::max<int64_t>(kMaxSplits, (nch + kMaxChunksPerSplit - 1) / kMaxChunksPerSplit);
  return (int)std::min<int64_t>(cap, std::max<int64_t>(1, (nch + per - 1) / per));
}

// One-pass kernel: its covariance splits for a batch of nblk
// blocks, the block of `lines` lines having ks for the covariance kernels:
// at least ks, and enough that the launch holds one workgroup per CU, at
// most kMaxSplits and one 32-sample chunk per split.  Its 32-bit raw sums
// take at most 8191 chunks a split; 0 when no count satisfies both.
static int onepass_splits(int ks, int64_t lines, int S, int nblk, int ncu) {
  const int64_t nch = lines * ceil_div(S, 32);
  int64_t k = std::max<int64_t>(ks, ncu / std::max(1, nblk));
  k = std::min<int64_t>(std::min<int64_t>(k, kMaxSplits), nch);
  k = std::max<int64_t>(k, (nch + 8190) / 8191);
  return k > kMaxSplits ? 0 : (int)k;
}

// One-pass kernel: the out-band whitening tiles each of its 16 waves takes
// (at most two), so that the four SIMDs (wave w on SIMD w % 4) get similar
// matrix-core work once the covariance super-tiles are counted: wave w owns
// lower super-tile w (row-major) and multiplies 4 fragments per stored
// fragment row of it; whitening tile i takes i / 2 + 1 steps for each of
// the two 16-sample groups.  Heaviest tiles first, each to the least loaded
// SIMD, then its least loaded wave with a free place.
static void make_wrows(int T, uint8_t wrow[16][2]) {
  int wl[16], sl[4] = {0, 0, 0, 0}, cnt[16];
  const int nsr = (T + 3) / 4;
  for (int w = 0; w < 16; ++w) {
    int I = 0, t = w;
    while (t > I) { t -= I + 1; ++I; }
    const int J = t;
    int rows = 0;
    if (I < nsr)
      for (int ii = 0; ii < 4; ++ii) {
        bool any = false;
        for (int j = 0; j < 4; ++j)
          any |= 4 * I + ii < T && 4 * J + j < T && (I > J || ii >= j);
        rows += any;
      }
    wl[w] = 4 * rows;
    sl[w % 4] += wl[w];
    cnt[w] = 0;
    wrow[w][0] = wrow[w][1] = 0xff;
  }
  for (int i = T - 1; i >= 0; --i) {
    const int cost = 2 * (i / 2 + 1);
    int bw = -1;
    for (int w = 0; w < 16; ++w) {
      if (cnt[w] == 2) continue;
      if (bw < 0 || sl[w % 4] < sl[bw % 4] || (sl[w % 4] == sl[bw % 4] && wl[w] < wl[bw])) bw = w;
    }
    wrow[bw][cnt[bw]++] = (uint8_t)i;
    wl[bw] += cost;
    sl[bw % 4] += cost;
  }
}

// Rectangles of at most 4 x 4 16-band tiles covering the lower triangle of
// T x T tiles (bands of 4 tile rows cut into 4-column pieces: at most 15
// for T <= 20), assigned to waves so the four SIMDs of a CU get similar work.
static int make_rects(int T, uint8_t rect[16][4]) {
  struct Rc { int r0, c0, nr, nc, n; };
  std::vector<Rc> v;
  for (int r0 = 0; r0 < T; r0 += 4) {
    const int nr = std::min(4, T - r0), ncols = r0 + nr;
    for (int c0 = 0; c0 < ncols; c0 += 4) {
      const int nc = std::min(4, ncols - c0);
      int n = 0;
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) n += (r0 + i >= c0 + j);
      if (n > 0) v.push_back(Rc{r0, c0, nr, nc, n});
    }
  }
  std::stable_sort(v.begin(), v.end(), [](const Rc& a, const Rc& b) { return a.n > b.n; });
  int load[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
  std::memset(rect, 0, 16 * 4);
  int nw = 0;
  for (const Rc& r : v) {
    int best = 0;
    for (int q = 1; q < 4; ++q)
      if (cnt[q] < 4 && (cnt[best] >= 4 || load[q] < load[best])) best = q;
    const int w = best + 4 * cnt[best];
    rect[w][0] = (uint8_t)r.r0; rect[w][1] = (uint8_t)r.c0; rect[w][2] = (uint8_t)r.nr; rect[w][3] = (uint8_t)r.nc;
    load[best] += r.n;
    cnt[best] += 1;
    nw = std::max(nw, w + 1);
  }
  return nw;
}

struct Block {
  int64_t line0;   // first line within the push
  int lines;
  bool reset;
};

struct Sizes {
  size_t shift, part, psum, mu, m2, nsnap, w64, wlp, scl, status, ev, coef, valid, nbadl, lfac, sscale;
};

// Doubles per block of the factor hand-off: T diagonal inverses and
// T (T - 1) / 2 off-diagonal tiles of 256 doubles, then the Bp scales.
static int64_t lf_stride_for(int Bp) {
  const int64_t T = Bp / 16;
  return 256 * (T + T * (T - 1) / 2) + Bp;
}

static Sizes scratch_sizes(int B, int S, int in_type, int sp, int nblk, int blk_lines, int ks_min = 0) {
  const int Bp = pad16(B), Bw = pad32(Bp);
  const int nsr = ceil_div(Bp, SUP), nsup = nsr * (nsr + 1) / 2;
  const int ks = std::max(ks_min, splits_for(blk_lines, ceil_div(S, KC), sp));
  const size_t psz = sp == RX_FP64 ? 8 : 4;
  Sizes z;
  z.shift = (size_t)nblk * Bp * 8;
  z.part = (size_t)nblk * ks * Bp * Bp * psz;
  (void)nsup;
  z.psum = (size_t)nblk * ks * Bp * 8;
  z.mu = (size_t)nblk * Bp * 8;
  z.m2 = (size_t)nblk * Bp * Bp * 8;
  z.nsnap = (size_t)nblk * 8;
  z.w64 = (size_t)nblk * Bp * Bp * 8;
  z.wlp = (size_t)nblk * Bp * Bw * 4;
  z.scl = (size_t)nblk * Bp * 4;
  z.status = (size_t)nblk * 8;             // status, then the FP8 clip flags
  z.ev = (size_t)nblk * Bp * 8;
  z.coef = (size_t)nblk * 8;
  z.lfac = (size_t)nblk * lf_stride_for(Bp) * 8;
  z.sscale = sp == RX_FP8_E4M3 ? (size_t)nblk * Bp * 4 : 0;
  // float input: per-pixel validity (by parity, read by the whitening) and
  // per-line counts of pixels with a non-finite band
  const bool fl = in_type != RX_IN_U16;
  z.valid = fl ? (size_t)nblk * blk_lines * S : 0;
  z.nbadl = fl ? (size_t)nblk * blk_lines * 4 : 0;
  return z;
}

// ---------------------------------------------------------------------------- stream
struct rx_stream {
  uint32_t magic = kMagic;
  rx_config cfg{};
  int B = 0, Bp = 0, Bw = 0, S = 0, in_type = 0, sp = 0, wp = 0, cpl = 0;
  int causal = 0;                         // blocks scored with the window before them
  int onepass = 0;                        // ... before their push (causal is then set too)
  int ncu = 0;                            // compute units of the device
  // one-pass: the window count before the push, and whether a window has
  // started within the push so far
  int64_t N_push = 0;
  bool push_reset = false;
  // causal: the previous batch's last snapshot slot (the window before the
  // next batch, already factored), valid until the statistics are replaced
  // or the snapshot buffers are reallocated
  bool prev_valid = false;
  int prev_par = 0, prev_slot = 0;
  size_t esz = 0;
  int dev = 0;
  // Three queues: A (centring shift, covariance product, merge), B (FP64
  // factorisation), st = C (whitening, masks, score pops).  One batch's
  // factorisation and whitening overlap the next batch's product and merge;
  // served streams run everything on the server's single queue.
  hipStream_t st = nullptr, stA = nullptr, stB = nullptr;
  bool own_st = false;
  hipEvent_t ev_in = nullptr, ev_done = nullptr, ev_stage = nullptr;
  hipEvent_t ev_fact = nullptr, ev_merged[2] = {nullptr, nullptr}, ev_white[2] = {nullptr, nullptr};
  // end of the latest push (recorded on st): a push finding it complete runs
  // on st alone; after such a push, the next pipelined one makes stA wait for it
  hipEvent_t ev_last = nullptr;
  bool st_only_tail = false;
  int npar = 1, par = 0, last_par = 0;    // parity sets of the per-batch buffers (queued batches alternate)
  rx_server* srv = nullptr;
  size_t footprint = 0;
  // resident window state (ping-pong): raw band sums then the pixel count N
  // (Bp + 1 values), scatter matrix
  DevBuf s1[2], m2[2];
  int cur = 0;
  int64_t N = 0;                          // pixels pushed into the window (N on the device is lower
                                          // when float input holds non-finite pixels)
  int64_t lines_seen = 0;
  // batch scratch
  DevBuf nsing, evb, dvb, coefb, nbvb, nbadl, shift, part, psum, sscale;
  // by parity: a batch's M2 and count snapshots are read by its factor, and
  // its mean snapshot, W, scales and status by its whitening, while the next
  // batch's product and merge run on queue A
  DevBuf m2s[2], nsnap[2], mu[2], w64[2], wlp[2], isc[2], osc[2], status[2], valid[2], lfac[2];
  unsigned last_nsing = 0;
  // pending scores
  DevBuf pend[2];
  int pcur = 0;
  int64_t head = 0, tail = 0;
  int sc_f64 = 0;
  // band-interleaved-by-pixel input: each push is first transposed into
  // this BIL copy (on queue A), which the path then reads; ev_bip marks the
  // end of the last push that read it
  DevBuf bip;
  hipEvent_t ev_bip = nullptr;
  hipEvent_t ev_shift = nullptr;          // one-pass kernel: the batch's centring shifts are written
  // host input staging: pinned chunk buffers, two per copy thread (see
  // stage_host_input), and the device copy of the push's lines
  struct HostSlot {
    void* p = nullptr;
    hipEvent_t ev = nullptr;      // the slot's latest host-to-device copy
    bool busy = false;
  };
  std::vector<HostSlot> hslots;
  DevBuf stage;
  bool stage_busy = false;
  // masks and conversions
  DevBuf maskbits, maskscr, cvt;
  // last factor
  int64_t last_w_off = -1;
  // optional per-phase timing with HIP events on the stream the kernels run on
  bool prof = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_open;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[5] = {0, 0, 0, 0, 0};
  int64_t prof_n[5] = {0, 0, 0, 0, 0};
  rx_counters cnt{};
  rx_status sticky = RX_OK;
  // a launch failed after the stream's state had advanced: its statistics and
  // FIFO no longer match what was launched, so every later call refuses
  bool broken = false;
  int64_t q_lines = 0;                    // served: lines submitted and not yet launched
};

struct rx_server;
static std::mutex* server_mutex(rx_stream* s);
// Calls on a served stream take the server's lock: its request loop may be
// launching the stream's blocks (and moving its score FIFO) meanwhile.
struct SrvLock {
  std::unique_lock<std::mutex> lk;
  explicit SrvLock(rx_stream* s) {
    if (std::mutex* m = server_mutex(s)) lk = std::unique_lock<std::mutex>(*m);
  }
};

static rx_status check_stream(rx_stream* s) {
  if (!s) return fail(RX_E_ARG, "null stream");
  if (s->magic != kMagic) return fail(RX_E_STATE, "stream handle is not live");
  if (s->broken) return fail(RX_E_STATE, "a launch on this stream failed earlier; destroy it");
  return RX_OK;
}

// ---------------------------------------------------------------------------- server (declared early)
struct Pending {
  rx_stream* s;
  const void* x;
  int64_t lines;
  uint64_t tag;
};
struct InFlight {
  hipEvent_t ev;
  std::vector<std::pair<rx_stream*, uint64_t>> items;
};
struct Done {
  uint64_t tag;
  int64_t t_ns;          // completion seen by the request loop (rx_clock_ns); 0 when polled directly
};
static int64_t clock_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
struct rx_server {
  uint32_t magic = 0x52585356u;   // "RXSV"
  size_t budget = 0, used = 0;
  int max_streams = 0, n_streams = 0;
  int dev = 0;
  // three queues as for an unserved stream: A (shift, covariance, merge),
  // B (factorisation), st = C (whitening, score pops); consecutive steps
  // overlap, ordered by the events below (step parity spar)
  hipStream_t st = nullptr, stA = nullptr, stB = nullptr;
  hipEvent_t ev_merged[2] = {nullptr, nullptr}, ev_fact = nullptr, ev_white[2] = {nullptr, nullptr};
  int spar = 0;
  std::deque<Pending> queue;
  std::deque<InFlight> inflight;
  std::deque<Done> done;                  // finished blocks collected by the request loop
  std::vector<hipEvent_t> free_events;
  std::mutex mu;
  // persistent request loop (rx_server_start / rx_server_stop)
  std::thread loop;
  std::condition_variable cv;
  bool running = false, stop = false;
  rx_status loop_err = RX_OK;
  std::string loop_msg;
  int64_t loop_steps = 0;
};
static std::mutex* server_mutex(rx_stream* s) { return (s && s->srv) ? &s->srv->mu : nullptr; }

// ---------------------------------------------------------------------------- config
extern "C" rx_status rx_config_init(rx_config* cfg, int32_t bands, int32_t samples) {
  if (!cfg) return fail(RX_E_ARG, "null config");
  std::memset(cfg, 0, sizeof *cfg);
  cfg->struct_size = sizeof(rx_config);
  cfg->bands = bands;
  cfg->samples = samples;
  cfg->in_type = RX_IN_U16;
  cfg->bit_depth = 12;
  cfg->layout = RX_BIL;
  cfg->syrk_prec = RX_BF16;
  cfg->whiten_prec = RX_BF16;
  return RX_OK;
}

static rx_status validate(const rx_config* c) {
  if (!c) return fail(RX_E_ARG, "null config");
  if (c->struct_size != sizeof(rx_config)) return fail(RX_E_ARG, "struct_size %u != %zu", c->struct_size, sizeof(rx_config));
  if (c->bands < 1 || c->bands > RX_MAX_BANDS) return fail(RX_E_ARG, "bands must be in [1, %d]", RX_MAX_BANDS);
  if (c->samples < 1) return fail(RX_E_ARG, "samples must be >= 1");
  if (c->in_type < RX_IN_U16 || c->in_type > RX_IN_F64) return fail(RX_E_ARG, "bad in_type");
  if (c->layout != RX_BIL && c->layout != RX_BIP) return fail(RX_E_ARG, "layout must be RX_BIL or RX_BIP");
  if (c->syrk_prec < RX_FP64 || c->syrk_prec > RX_FP8_E4M3) return fail(RX_E_ARG, "bad syrk_prec");
  if (c->whiten_prec < RX_FP64 || c->whiten_prec > RX_FP8_E4M3) return fail(RX_E_ARG, "bad whiten_prec");
  if (c->ddof != 0 && c->ddof != 1) return fail(RX_E_ARG, "ddof must be 0 or 1");
  if (c->block_lines < 0 || c->window_lines < 0) return fail(RX_E_ARG, "block_lines and window_lines must be >= 0");
  if (!(c->ridge_rel >= 0.0) || !std::isfinite(c->ridge_rel)) return fail(RX_E_ARG, "ridge_rel must be finite and >= 0");
  if ((c->flags & ~(RX_FLAG_CAUSAL | RX_FLAG_ONE_PASS)) != 0) return fail(RX_E_ARG, "unknown flags");
  if ((c->flags & RX_FLAG_CAUSAL) && (c->flags & RX_FLAG_ONE_PASS))
    return fail(RX_E_ARG, "RX_FLAG_CAUSAL and RX_FLAG_ONE_PASS are exclusive");
  if (c->in_type == RX_IN_U16 && (c->bit_depth < 0 || c->bit_depth > 16)) return fail(RX_E_ARG, "bit_depth must be in [0, 16]");
  return RX_OK;
}

static size_t stream_bytes(const rx_config* c, int max_block_lines) {
  const int Bp = pad16(c->bands);
  // causal and one-pass: the window before the block (push)
  const int slots = 1 + ((c->flags & (RX_FLAG_CAUSAL | RX_FLAG_ONE_PASS)) ? 1 : 0);
  const Sizes z = scratch_sizes(c->bands, c->samples, c->in_type, c->syrk_prec, slots, std::max(1, max_block_lines));
  const size_t state = 2 * ((size_t)(Bp + 1) * 8 + (size_t)Bp * Bp * 8);
  // the snapshot, factor and validity buffers come in two parity sets
  // (served streams too: consecutive server steps overlap)
  const size_t par = z.mu + z.m2 + z.nsnap + z.w64 + z.wlp + 2 * z.scl + z.status + z.valid + z.lfac;
  const size_t scr = z.shift + z.part + z.psum + 2 * par + 2 * z.ev + 2 * z.coef + z.nbadl + z.sscale;
  const size_t esz = c->whiten_prec == RX_FP64 ? 8 : 4;
  const size_t pend = 2 * (size_t)std::max(1, max_block_lines) * c->samples * esz;
  return state + scr + pend;
}

extern "C" rx_status rx_stream_footprint(const rx_config* cfg, int32_t max_block_lines, size_t* bytes) {
  rx_status r = validate(cfg);
  if (r != RX_OK) return r;
  if (!bytes || max_block_lines < 1) return fail(RX_E_ARG, "null bytes or max_block_lines < 1");
  *bytes = stream_bytes(cfg, max_block_lines);
  return RX_OK;
}

extern "C" rx_status rx_split_plan(const rx_config* cfg, int64_t lines, int32_t* splits, int64_t* max_chunks) {
  rx_status r = validate(cfg);
  if (r != RX_OK) return r;
  if (lines < 1 || lines > INT32_MAX || !splits || !max_chunks) return fail(RX_E_ARG, "bad block or null output");
  const int cpl = ceil_div(cfg->samples, KC);
  const int ks = splits_for(lines, cpl, cfg->syrk_prec);
  const int64_t nch = lines * cpl;
  *splits = ks;
  *max_chunks = (nch + ks - 1) / ks;       // split s holds chunks [nch s / ks, nch (s + 1) / ks)
  return RX_OK;
}

// ---------------------------------------------------------------------------- init / destroy
// Wait for every queue of a stream (A and B feed C, but host reads of the
// statistics, counters or W must not depend on that).
static hipError_t sync_all(rx_stream* s) {
  hipError_t e = hipStreamSynchronize(s->st);
  if (e == hipSuccess && s->stA && s->stA != s->st) e = hipStreamSynchronize(s->stA);
  if (e == hipSuccess && s->stB && s->stB != s->st) e = hipStreamSynchronize(s->stB);
  return e;
}

static void free_stream(rx_stream* s) {
  DevBuf* bufs[] = {&s->s1[0], &s->s1[1], &s->m2[0], &s->m2[1], &s->shift, &s->part, &s->psum, &s->m2s[1],
                    &s->nsnap[1], &s->mu[0],
                    &s->mu[1], &s->m2s[0], &s->nsnap[0], &s->w64[0], &s->w64[1], &s->wlp[0], &s->wlp[1], &s->isc[0],
                    &s->isc[1], &s->osc[0], &s->osc[1], &s->status[0], &s->status[1], &s->evb, &s->dvb, &s->coefb,
                    &s->nbvb, &s->valid[0], &s->valid[1], &s->lfac[0], &s->lfac[1], &s->nbadl, &s->bip, &s->sscale, &s->nsing, &s->pend[0], &s->pend[1], &s->stage, &s->maskbits, &s->maskscr, &s->cvt};
  for (DevBuf* b : bufs) dev_free(*b);
  for (auto& hs : s->hslots) {
    if (hs.p) (void)hipHostFree(hs.p);
    if (hs.ev) (void)hipEventDestroy(hs.ev);
  }
  s->hslots.clear();
  for (auto& pe : s->prof_open) { s->prof_pool.push_back(pe.second.first); s->prof_pool.push_back(pe.second.second); }
  for (hipEvent_t e : s->prof_pool) (void)hipEventDestroy(e);
  s->prof_pool.clear();
  s->prof_open.clear();
  hipEvent_t evs[] = {s->ev_in, s->ev_done, s->ev_stage, s->ev_merged[0], s->ev_merged[1],
                      s->ev_fact, s->ev_white[0], s->ev_white[1], s->ev_last, s->ev_bip, s->ev_shift};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (s->own_st) {
    if (s->st) (void)hipStreamDestroy(s->st);
    if (s->stA) (void)hipStreamDestroy(s->stA);
    if (s->stB) (void)hipStreamDestroy(s->stB);
  }
  s->magic = 0;
}

static rx_status alloc_scratch(rx_stream* s, int nblk, int blk_lines, int ks_min = 0) {
  const Sizes z = scratch_sizes(s->B, s->S, s->in_type, s->sp, nblk, blk_lines, ks_min);
  rx_status r;
  if ((r = dev_ensure(s->shift, z.shift, s)) != RX_OK) return r;
  if ((r = dev_ensure(s->part, z.part, s)) != RX_OK) return r;
  if ((r = dev_ensure(s->psum, z.psum, s)) != RX_OK) return r;
  if (z.sscale && (r = dev_ensure(s->sscale, z.sscale, s)) != RX_OK) return r;
  bool zeroed = false;
  for (int q = 0; q < s->npar; ++q) {
    if ((r = dev_ensure(s->m2s[q], z.m2, s)) != RX_OK) return r;
    if ((r = dev_ensure(s->nsnap[q], z.nsnap, s)) != RX_OK) return r;
    if ((r = dev_ensure(s->mu[q], z.mu, s)) != RX_OK) return r;
    // the factor never writes above the diagonal tiles of W or its
    // low-precision copy (nor the copy's padding columns): those stay as
    // zeroed here
    const size_t w_before = s->w64[q].cap, wl_before = s->wlp[q].cap;
    if ((r = dev_ensure(s->w64[q], z.w64, s)) != RX_OK) return r;
    if ((r = dev_ensure(s->wlp[q], z.wlp, s)) != RX_OK) return r;
    if (s->w64[q].cap != w_before) { HIPC(hipMemsetAsync(s->w64[q].p, 0, s->w64[q].cap, s->st)); zeroed = true; }
    if (s->wlp[q].cap != wl_before) { HIPC(hipMemsetAsync(s->wlp[q].p, 0, s->wlp[q].cap, s->st)); zeroed = true; }
    if ((r = dev_ensure(s->isc[q], z.scl, s)) != RX_OK) return r;
    if ((r = dev_ensure(s->osc[q], z.scl, s)) != RX_OK) return r;
    if ((r = dev_ensure(s->status[q], z.status, s)) != RX_OK) return r;
    if (z.valid && (r = dev_ensure(s->valid[q], z.valid, s)) != RX_OK) return r;
    if ((r = dev_ensure(s->lfac[q], z.lfac, s)) != RX_OK) return r;
  }
  // buffers zeroed on queue C must be clear before queue B's factor writes
  // them (only after a growth: otherwise B must not wait behind C)
  if (zeroed && s->stB != s->st) {
    HIPC(hipEventRecord(s->ev_done, s->st));
    HIPC(hipStreamWaitEvent(s->stB, s->ev_done, 0));
  }
  if ((r = dev_ensure(s->evb, z.ev, s)) != RX_OK) return r;
  if ((r = dev_ensure(s->dvb, z.ev, s)) != RX_OK) return r;
  if ((r = dev_ensure(s->coefb, z.coef, s)) != RX_OK) return r;
  if ((r = dev_ensure(s->nbvb, z.coef, s)) != RX_OK) return r;
  if (z.nbadl && (r = dev_ensure(s->nbadl, z.nbadl, s)) != RX_OK) return r;
  return RX_OK;
}

extern "C" rx_status rx_init(const rx_config* cfg, rx_server* srv, rx_stream** out) {
  if (!out) return fail(RX_E_ARG, "null output handle");
  *out = nullptr;
  rx_status r = validate(cfg);
  if (r != RX_OK) return r;
  int ndev = 0;
  HIPC(hipGetDeviceCount(&ndev));
  if (cfg->device < 0 || cfg->device >= ndev) return fail(RX_E_ARG, "device %d not present (%d devices)", cfg->device, ndev);
  if (srv && srv->dev != cfg->device) return fail(RX_E_ARG, "stream device differs from the server's");
  if (srv && cfg->layout != RX_BIL) return fail(RX_E_ARG, "served streams take BIL blocks");
  HIPC(hipSetDevice(cfg->device));
  if ((r = noalloc_setup(cfg->device)) != RX_OK) return r;

  rx_stream* s = new rx_stream();
  s->cfg = *cfg;
  s->B = cfg->bands;
  s->Bp = pad16(s->B);
  s->Bw = pad32(s->Bp);
  s->S = cfg->samples;
  s->in_type = cfg->in_type;
  s->causal = (cfg->flags & (RX_FLAG_CAUSAL | RX_FLAG_ONE_PASS)) ? 1 : 0;
  s->onepass = (cfg->flags & RX_FLAG_ONE_PASS) ? 1 : 0;
  s->sp = cfg->syrk_prec;
  s->wp = cfg->whiten_prec;
  s->cpl = ceil_div(s->S, KC);
  s->esz = in_elem_size(s->in_type);
  s->dev = cfg->device;
  s->sc_f64 = s->wp == RX_FP64 ? 1 : 0;
  if (hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, s->dev) != hipSuccess || s->ncu < 1) {
    (void)hipGetLastError();
    s->ncu = 1;
  }

  auto bail = [&](rx_status st) {
    std::string keep = g_err;
    free_stream(s);
    delete s;
    g_err = keep;
    return st;
  };
  if (srv) {
    std::lock_guard<std::mutex> lk(srv->mu);
    const int mbl = cfg->block_lines > 0 ? cfg->block_lines : 128;
    const size_t need = stream_bytes(cfg, mbl);
    if (srv->n_streams >= srv->max_streams) { delete s; return fail(RX_E_BUDGET, "server has no free stream slot"); }
    if (srv->used + need > srv->budget) {
      delete s;
      return fail(RX_E_BUDGET, "stream needs %zu bytes, %zu of %zu left", need, srv->budget - srv->used, srv->budget);
    }
    srv->used += need;
    srv->n_streams += 1;
    s->srv = srv;
    s->footprint = need;
    s->st = srv->st;
    s->stA = srv->stA;
    s->stB = srv->stB;
    s->npar = 2;
  } else {
    s->own_st = true;
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stA, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stB, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(RX_E_DEVICE, "hipStreamCreate failed"));
    s->npar = 2;
  }
  hipEvent_t* evs[] = {&s->ev_in, &s->ev_done, &s->ev_stage, &s->ev_merged[0],
                       &s->ev_merged[1], &s->ev_fact, &s->ev_white[0], &s->ev_white[1], &s->ev_last, &s->ev_bip,
                       &s->ev_shift};
  for (hipEvent_t* e : evs)
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return bail(fail(RX_E_DEVICE, "hipEventCreate failed"));
  const size_t s1b = (size_t)(s->Bp + 1) * 8, m2b = (size_t)s->Bp * s->Bp * 8;
  for (int i = 0; i < 2; ++i) {
    if ((r = dev_ensure(s->s1[i], s1b, s)) != RX_OK) return bail(r);
    if ((r = dev_ensure(s->m2[i], m2b, s)) != RX_OK) return bail(r);
    if (hipMemsetAsync(s->s1[i].p, 0, s1b, s->st) != hipSuccess || hipMemsetAsync(s->m2[i].p, 0, m2b, s->st) != hipSuccess)
      return bail(fail(RX_E_DEVICE, "hipMemsetAsync failed"));
  }
  if ((r = dev_ensure(s->nsing, 256, s)) != RX_OK) return bail(r);
  if (hipMemsetAsync(s->nsing.p, 0, 256, s->st) != hipSuccess) return bail(fail(RX_E_DEVICE, "hipMemsetAsync failed"));
  if (s->srv) {
    const int mbl = cfg->block_lines > 0 ? cfg->block_lines : 128;
    if ((r = alloc_scratch(s, 1, mbl)) != RX_OK) return bail(r);
    if ((r = dev_ensure(s->pend[0], (size_t)2 * mbl * s->S * (s->sc_f64 ? 8 : 4), s)) != RX_OK) return bail(r);
  }
  if (hipStreamSynchronize(s->st) != hipSuccess) return bail(fail(RX_E_DEVICE, "hipStreamSynchronize failed"));
  *out = s;
  return RX_OK;
}

extern "C" rx_status rx_destroy(rx_stream* s) {
  if (!s) return RX_OK;
  if (s->magic != kMagic) return fail(RX_E_STATE, "stream handle is not live");
  (void)hipSetDevice(s->dev);
  if (s->srv) {
    // under the server's lock: its queued blocks leave the queue before the
    // request loop can launch them, then the launched ones are waited for
    rx_server* srv = s->srv;
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto it = srv->queue.begin(); it != srv->queue.end();) it = (it->s == s) ? srv->queue.erase(it) : it + 1;
    for (auto& f : srv->inflight)
      for (auto& it : f.items)
        if (it.first == s) it.first = nullptr;
    (void)sync_all(s);
    srv->used -= s->footprint;
    srv->n_streams -= 1;
    free_stream(s);
    delete s;
    return RX_OK;
  }
  (void)sync_all(s);
  free_stream(s);
  delete s;
  return RX_OK;
}

// ---------------------------------------------------------------------------- pending FIFO
static rx_status pending_reserve(rx_stream* s, int64_t npx) {
  const size_t es = s->sc_f64 ? 8 : 4;
  const int64_t live = s->tail - s->head;
  DevBuf& cur = s->pend[s->pcur];
  if ((size_t)(s->tail + npx) * es <= cur.cap) return RX_OK;
  DevBuf& alt = s->pend[1 - s->pcur];
  const size_t need = (size_t)(live + npx) * es;
  rx_status r = dev_ensure(alt, std::max(need, cur.cap * 2), s);
  if (r != RX_OK) return r;
  if (live > 0)
    HIPC(hipMemcpyAsync(alt.p, static_cast<char*>(cur.p) + (size_t)s->head * es, (size_t)live * es,
                        hipMemcpyDeviceToDevice, s->st));
  s->pcur = 1 - s->pcur;
  s->head = 0;
  s->tail = live;
  return RX_OK;
}

// ---------------------------------------------------------------------------- batch preparation
struct Job {
  rx_stream* s;
  BatchDesc d;
  int in_type, sp, wp, Bw;
  int par;
  int wg_valid, wg_shift, wg_syrk, wg_merge, wg_mmat, wg_factor, wg_whiten;
  int copy = 0;           // causal: slot nblk is copied from the previous batch (k_copy_slot)
  int fused = 0;          // one-pass: covariance product and scores in one kernel (k_onepass)
  int wg_fused = 0;
  int fast = 0;           // ... and the whitening waits only for the input (one block, pipelined)
};

// Cut n_lines starting at stream line `pos` into blocks.
static void cut_blocks(const rx_stream* s, int64_t pos, int64_t n_lines, std::vector<Block>& out) {
  int64_t off = 0;
  while (off < n_lines) {
    int64_t take = n_lines - off;
    if (s->cfg.block_lines > 0) take = std::min<int64_t>(take, s->cfg.block_lines);
    const int64_t R = s->cfg.window_lines;
    bool reset = false;
    if (R > 0) {
      take = std::min<int64_t>(take, R - (pos + off) % R);
      reset = ((pos + off) % R) == 0;
    }
    out.push_back(Block{off, take > INT32_MAX ? 0 : (int)take, reset});
    off += take;
  }
}

// Group a push's blocks into batches (launched together): runs of up to
// kMaxBlocksPerBatch blocks of one length, plus one shorter block at the end.
static std::vector<std::pair<size_t, size_t>> plan_batches(const std::vector<Block>& blks) {
  std::vector<std::pair<size_t, size_t>> out;
  size_t i = 0;
  while (i < blks.size()) {
    size_t k = i + 1;
    while (k < blks.size() && (int)(k - i) < kMaxBlocksPerBatch && blks[k].lines == blks[i].lines) ++k;
    if (k < blks.size() && (int)(k - i) < kMaxBlocksPerBatch && blks[k].lines < blks[i].lines) ++k;
    out.push_back({i, k});
    i = k;
  }
  return out;
}

// One-pass kernel: the configurations it covers (the input pointer must also
// give 16-byte aligned rows).
static bool onepass_kernel_config(const rx_stream* s) {
  return s->onepass && s->in_type == RX_IN_U16 && s->sp == RX_BF16 && s->wp == RX_BF16 && s->Bp <= 272 &&
         ((size_t)s->S * s->esz) % 16 == 0;
}

// Everything the batches of a push (or of a server step) can allocate,
// reserved before any stream state changes: scratch for each batch (buffers
// only grow, so the largest need wins) and FIFO room for all their pixels.
// A failure here leaves the stream's statistics, FIFO and parity untouched.
static rx_status reserve_batches(rx_stream* s, const std::vector<Block>& blks,
                                 const std::vector<std::pair<size_t, size_t>>& batches) {
  const int pp = s->prev_par;
  const DevBuf* kept[6] = {&s->mu[pp], &s->wlp[pp], &s->w64[pp], &s->isc[pp], &s->osc[pp], &s->status[pp]};
  size_t cap0[6];
  for (int i = 0; i < 6; ++i) cap0[i] = kept[i]->cap;
  int64_t lines = 0;
  for (const auto& bt : batches) {
    const int nb = (int)(bt.second - bt.first);
    int ks_min = 0;
    if (onepass_kernel_config(s))
      ks_min = onepass_splits(splits_for(blks[bt.first].lines, s->cpl, s->sp), blks[bt.first].lines, s->S, nb, s->ncu);
    rx_status r = alloc_scratch(s, nb + s->causal, blks[bt.first].lines, ks_min);
    if (r != RX_OK) return r;
    for (size_t i = bt.first; i < bt.second; ++i) lines += blks[i].lines;
  }
  for (int i = 0; i < 6; ++i)
    if (kept[i]->cap != cap0[i]) s->prev_valid = false;   // reallocated: the previous slot is gone
  return pending_reserve(s, lines * s->S);
}

// Fill a job for blocks[i0, i1) of a push whose lines start at x (after
// reserve_batches).  Updates the host copy of N, the pending tail and the
// parity; cannot fail once the reservation is made.
static rx_status prepare_job(rx_stream* s, const void* x, const std::vector<Block>& blks, size_t i0, size_t i1,
                             Job& j, bool& notready, bool allow_copy = false) {
  const int nblk = (int)(i1 - i0);
  const int L = blks[i0].lines, last = blks[i1 - 1].lines;
  const int pp = s->prev_par;
  int64_t lines = 0;
  for (size_t i = i0; i < i1; ++i) lines += blks[i].lines;
  const int64_t npx = lines * s->S;
  const bool lag_empty = s->push_reset;     // one-pass: a window started in an earlier batch of the push
  // reserve_batches has sized every buffer and the FIFO for this batch
  if ((size_t)(s->tail + npx) * (s->sc_f64 ? 8 : 4) > s->pend[s->pcur].cap)
    return fail(RX_E_STATE, "internal: batch prepared without a reservation");

  BatchDesc& d = j.d;
  std::memset(&d, 0, sizeof d);
  d.x = static_cast<const char*>(x) + (size_t)blks[i0].line0 * s->B * s->S * s->esz;
  d.B = s->B;
  d.Bp = s->Bp;
  d.S = s->S;
  d.nblk = nblk;
  d.blk_lines = L;
  d.last_lines = last;
  d.cpl = s->cpl;
  d.ks = splits_for(L, s->cpl, s->sp);
  d.ks_last = splits_for(last, s->cpl, s->sp);
  d.nrect = make_rects(s->Bp / 16, d.rect);
  d.nsr = ceil_div(s->Bp, SUP);
  d.nsup = d.nsr * (d.nsr + 1) / 2;
  d.vec_ok = ((reinterpret_cast<uintptr_t>(d.x) & 15) == 0) && (((size_t)s->S * s->esz) % 16 == 0);
  d.vec8_ok = s->in_type == RX_IN_U16 && ((reinterpret_cast<uintptr_t>(d.x) & 7) == 0) && (s->S % 4 == 0);
  d.ddof = s->cfg.ddof;
  d.rho = s->cfg.ridge_rel;
  uint64_t rb = 0;
  for (int b = 0; b < nblk; ++b) {
    const Block& bk = blks[i0 + b];
    if (bk.reset) {
      rb |= 1ull << b;
      s->N = 0;
    }
    if (s->onepass) {
      if (bk.reset) s->push_reset = true;
      if (s->push_reset || (s->cfg.ridge_rel == 0.0 && s->N_push <= s->B) || s->N_push <= s->cfg.ddof) notready = true;
    } else if (s->causal && ((s->cfg.ridge_rel == 0.0 && s->N <= s->B) || s->N <= s->cfg.ddof)) {
      notready = true;
    }
    s->N += (int64_t)bk.lines * s->S;
    if (!s->causal && s->cfg.ridge_rel == 0.0 && s->N <= s->B) notready = true;
  }
  d.reset_bits = rb;
  d.onepass = s->onepass;
  d.lag_empty = s->onepass && lag_empty;
  const int q = s->par;                     // parity set of this batch's buffers
  j.par = q;
  d.shift = static_cast<double*>(s->shift.p);
  d.sscale = static_cast<float*>(s->sscale.p);
  d.part = s->part.p;
  d.psum = static_cast<double*>(s->psum.p);
  d.mu_snap = static_cast<double*>(s->mu[q].p);
  d.m2_snap = static_cast<double*>(s->m2s[q].p);
  d.n_snap = static_cast<double*>(s->nsnap[q].p);
  d.ev = static_cast<double*>(s->evb.p);
  d.dv = static_cast<double*>(s->dvb.p);
  d.coef = static_cast<double*>(s->coefb.p);
  d.nbv = static_cast<double*>(s->nbvb.p);
  if (s->in_type != RX_IN_U16) {
    d.valid = static_cast<uint8_t*>(s->valid[q].p);
    d.nbadl = static_cast<int*>(s->nbadl.p);
  }
  d.s1_in = static_cast<const double*>(s->s1[s->cur].p);
  d.s1_out = static_cast<double*>(s->s1[1 - s->cur].p);
  d.m2_in = static_cast<const double*>(s->m2[s->cur].p);
  d.m2_out = static_cast<double*>(s->m2[1 - s->cur].p);
  d.w64 = static_cast<double*>(s->w64[q].p);
  d.wlp = s->wlp[q].p;
  d.iscale = static_cast<float*>(s->isc[q].p);
  d.oscale = static_cast<float*>(s->osc[q].p);
  d.status = static_cast<int*>(s->status[q].p);
  d.lfac = static_cast<double*>(s->lfac[q].p);
  d.lf_stride = lf_stride_for(s->Bp);
  d.clipflag = d.status + nblk + s->causal;
  // causal: copy the previous batch's last slot (two parity sets, so this
  // batch's merge and factor cannot overwrite it) or else form slot nblk here
  const bool copy = s->causal && allow_copy && s->npar == 2 && s->prev_valid;
  d.causal = s->causal ? (copy ? 2 : 1) : 0;
  const int esz_w = s->wp == RX_FP64 ? 0 : s->wp == RX_FP32 ? 4 : s->wp == RX_FP8_E4M3 ? 1 : 2;
  d.wl_bytes = (int64_t)s->Bp * s->Bw * esz_w;
  if (copy) {
    const int ps = s->prev_slot;
    d.src_mu = static_cast<const double*>(s->mu[pp].p) + (int64_t)ps * s->Bp;
    d.src_wlp = static_cast<const char*>(s->wlp[pp].p) + ps * d.wl_bytes;
    d.src_w64 = static_cast<const double*>(s->w64[pp].p) + (int64_t)ps * s->Bp * s->Bp;
    d.src_isc = static_cast<const float*>(s->isc[pp].p) + (int64_t)ps * s->Bp;
    d.src_osc = static_cast<const float*>(s->osc[pp].p) + (int64_t)ps * s->Bp;
    d.src_status = static_cast<const int*>(s->status[pp].p) + ps;
  }
  j.copy = copy ? 1 : 0;
  // one-pass with the window before the push in place: one read of the lines
  // (16-bit, 16-byte aligned rows with S % 8 == 0, BF16 products, <= 272 bands)
  j.fused = (copy && onepass_kernel_config(s) && d.vec_ok) ? 1 : 0;
  if (j.fused) {
    const int ks = onepass_splits(d.ks, L, s->S, nblk, s->ncu), ksl = onepass_splits(d.ks_last, last, s->S, nblk, s->ncu);
    if (ks > 0 && ksl > 0) {
      d.ks = ks;
      d.ks_last = ksl;
      make_wrows(s->Bp / 16, d.wrow);
    } else {
      j.fused = 0;
    }
  }
  d.nsing = static_cast<unsigned int*>(s->nsing.p);
  d.cnt64 = reinterpret_cast<unsigned long long*>(static_cast<char*>(s->nsing.p) + 8);
  d.scores = static_cast<char*>(s->pend[s->pcur].p) + (size_t)s->tail * (s->sc_f64 ? 8 : 4);

  j.s = s;
  j.in_type = s->in_type;
  j.sp = s->sp;
  j.wp = s->wp;
  j.Bw = s->Bw;
  j.wg_valid = s->in_type != RX_IN_U16 ? (int)lines : 0;
  j.wg_shift = nblk * (s->Bp / 4);
  j.wg_syrk = (whole_triangle(s->sp) ? 1 : d.nsup) * ((nblk - 1) * d.ks + d.ks_last);
  j.wg_merge = ceil_div(s->Bp, 64);
  j.wg_mmat = 0;                            // merge, matrix part: row strips of 4 x 64 entries
  for (int g = 0; g < s->Bp / 4; ++g) j.wg_mmat += (4 * g + 67) / 64;
  j.wg_factor = nblk + (d.causal == 1 ? 1 : 0);   // causal, slot formed here: also the window before the batch
  if (s->onepass) {
    // only the window after the batch (the next batch's window before the
    // push, or the next push's) and a slot nblk formed here score anything
    d.fslot0 = nblk - 1;
    j.wg_factor = 1 + (d.causal == 1 ? 1 : 0);
  }
  j.wg_whiten = (int)(lines * s->cpl);
  j.wg_fused = (nblk - 1) * d.ks + d.ks_last;

  s->cur ^= 1;
  s->tail += npx;
  s->last_w_off = (int64_t)(nblk - 1) * s->Bp * s->Bp;
  s->last_par = q;
  s->par = (q + 1) % s->npar;
  s->cnt.blocks += nblk;
  if (s->causal) {
    s->prev_valid = true;
    s->prev_par = q;
    // one-pass: a later batch of the same push takes this batch's slot nblk,
    // the window before the push
    s->prev_slot = (s->onepass && i1 < blks.size()) ? nblk : nblk - 1;
  }
  return RX_OK;
}

// Phase timing: a pair of events around one phase's launches.
static rx_status prof_mark(rx_stream* s, int phase, bool begin, hipStream_t st) {
  if (!s || !s->prof) return RX_OK;
  auto take = [&]() -> hipEvent_t {
    if (!s->prof_pool.empty()) { hipEvent_t e = s->prof_pool.back(); s->prof_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  };
  if (begin) {
    hipEvent_t a = take();
    HIPC(hipEventRecord(a, st));
    s->prof_open.push_back({phase, {a, nullptr}});
  } else {
    hipEvent_t b = take();
    HIPC(hipEventRecord(b, st));
    s->prof_open.back().second.second = b;
  }
  return RX_OK;
}

static rx_status prof_collect(rx_stream* s) {
  for (auto& pe : s->prof_open) {
    float ms = 0.0f;
    if (pe.second.second) {
      HIPC(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
      s->prof_ms[pe.first] += ms;
      s->prof_n[pe.first] += 1;
      s->prof_pool.push_back(pe.second.second);
    }
    s->prof_pool.push_back(pe.second.first);
  }
  s->prof_open.clear();
  return RX_OK;
}

// Launch the five phases for a set of jobs (each stream at most once) on the
// queues `qs`: A (shift, covariance product, merge), B (factorisation), C
// (whitening).  When the three differ (one unserved stream, one job) the
// batch is ordered with events on its parity set of buffers:
//   A runs shift, product and merge in order; before the merge it waits for
//     the whitening that last read this parity's snapshots (two batches
//     back; that whitening followed the factor that read the M2 snapshot);
//   B waits for A's merge, then factors;
//   C waits for B's factorisation, then whitens.
// prof (nullable): stream whose phase timers bracket the launches.
struct Queues {
  hipStream_t A, B, C;
};
// Events that order the three queues of a pipelined launch: those of an
// unserved stream (par = the batch's parity set) or of a server (par = the
// step's parity: a served stream's two parity sets alternate per block, so
// the previous use of a set by any stream in the step is at least two steps
// back, and the whitening of step n - 2 has then read it).
struct Pipe {
  hipEvent_t* ev_merged;   // [2]
  hipEvent_t ev_fact;
  hipEvent_t* ev_white;    // [2]
  int par;
  bool causal_copy;        // a causal stream whose next batch copies this batch's last slot
  bool in_event = true;    // a lone stream's input is ordered by its ev_in (not for resident lines)
};
static rx_status launch_jobs(std::vector<Job>& jobs, Queues qs, const Pipe* pe, rx_stream* prof = nullptr) {
  const bool piped = qs.A != qs.C;
  rx_stream* ps = piped && jobs.size() == 1 ? jobs[0].s : nullptr;   // a lone stream's input event
  if (piped && !pe) return fail(RX_E_STATE, "internal: pipelined launch without its events");
  auto run_groups = [&](auto key, auto launch) -> rx_status {
    std::vector<bool> done(jobs.size(), false);
    for (size_t a = 0; a < jobs.size(); ++a) {
      if (done[a]) continue;
      std::vector<size_t> grp;
      for (size_t c = a; c < jobs.size(); ++c)
        if (!done[c] && key(jobs[c]) == key(jobs[a])) grp.push_back(c);
      for (size_t g0 = 0; g0 < grp.size(); g0 += MAXB) {
        const size_t g1 = std::min(grp.size(), g0 + MAXB);
        rx_status r = launch(grp, g0, g1);
        if (r != RX_OK) return r;
      }
      for (size_t c : grp) done[c] = true;
    }
    return RX_OK;
  };
  auto fill = [&](LaunchSet& ls, const std::vector<size_t>& grp, size_t g0, size_t g1, int Job::*wg) {
    ls.nb = (int)(g1 - g0);
    ls.wg0[0] = 0;
    for (size_t i = g0; i < g1; ++i) {
      ls.d[i - g0] = jobs[grp[i]].d;
      ls.wg0[i - g0 + 1] = ls.wg0[i - g0] + jobs[grp[i]].*wg;
    }
    return ls.wg0[ls.nb];
  };
  {
    // causal batches whose window-before slot is the previous batch's last
    // one: copy it on the whitening queue once the previous factorisation
    // (the latest ev_fact) is done; this batch's merge and factor skip it
    LaunchSet cs;
    cs.nb = 0;
    cs.wg0[0] = 0;
    for (const Job& j : jobs)
      if (j.copy) {
        if (cs.nb == MAXB) return fail(RX_E_STATE, "too many batches in one launch");
        cs.d[cs.nb] = j.d;
        cs.wg0[cs.nb + 1] = CPWG * (cs.nb + 1);   // k_copy_slot: CPWG workgroups per batch
        ++cs.nb;
      }
    if (cs.nb > 0) {
      if (piped) HIPC(hipStreamWaitEvent(qs.C, pe->ev_fact, 0));
      HIPC(rxk_launch_copy_slot(&cs, cs.nb, qs.C));
    }
  }
  auto whiten_all = [&]() -> rx_status {
    rx_status r = run_groups([](const Job& j) { return (j.in_type * 16 + j.wp) * 1024 + j.Bw; },
                             [&](const std::vector<size_t>& grp, size_t g0, size_t g1) -> rx_status {
                               LaunchSet a;
                               const int n = fill(a, grp, g0, g1, &Job::wg_whiten);
                               rx_status q;
                               if ((q = prof_mark(prof, 4, true, qs.C)) != RX_OK) return q;
                               HIPC(rxk_launch_whiten(jobs[grp[g0]].in_type, jobs[grp[g0]].wp, &a, n, jobs[grp[g0]].Bw,
                                                      qs.C));
                               return prof_mark(prof, 4, false, qs.C);
                             });
    if (r != RX_OK) return r;
    if (piped) HIPC(hipEventRecord(pe->ev_white[pe->par], qs.C));
    return RX_OK;
  };
  // a one-block causal batch whitens with the copied slot only: it needs the
  // input, not this batch's statistics, so it is queued first (its scores do
  // not wait behind the host time of the statistics launches)
  const bool early = ps && jobs[0].fast;
  // one-pass kernel: a lone stream's pipelined batch with its window-before
  // slot copied (it scores the batch as it forms the covariance partials)
  const bool fused = ps && jobs[0].fused;
  if (fused && !piped) return fail(RX_E_STATE, "internal: one-pass launch without its queues");
  if (early) {
    if (pe->in_event) HIPC(hipStreamWaitEvent(qs.C, ps->ev_in, 0));
    rx_status r0 = whiten_all();
    if (r0 != RX_OK) return r0;
  }
  rx_status r = run_groups([](const Job& j) { return j.in_type * 16 + j.sp; },
                           [&](const std::vector<size_t>& grp, size_t g0, size_t g1) -> rx_status {
                             LaunchSet a, b, c, e;
                             const int it = jobs[grp[g0]].in_type, sp = jobs[grp[g0]].sp;
                             rx_status q;
                             if ((q = prof_mark(prof, 0, true, qs.A)) != RX_OK) return q;
                             if (it != RX_IN_U16) {        // validity pass first (float input)
                               // valid[par] is read by the whitening of the batch
                               // that last used this parity: wait for it first
                               if (piped) HIPC(hipStreamWaitEvent(qs.A, pe->ev_white[pe->par], 0));
                               const int n0 = fill(a, grp, g0, g1, &Job::wg_valid);
                               HIPC(rxk_launch_stats(it, sp, 3, &a, n0, nullptr, 0, qs.A));
                             }
                             const int n1 = fill(a, grp, g0, g1, &Job::wg_shift);
                             const int n2 = fill(b, grp, g0, g1, &Job::wg_syrk);
                             const int n3 = fill(c, grp, g0, g1, &Job::wg_merge);
                             const int n4 = fill(e, grp, g0, g1, &Job::wg_mmat);
                             HIPC(rxk_launch_stats(it, sp, 0, &a, n1, nullptr, 0, qs.A));
                             if ((q = prof_mark(prof, 0, false, qs.A)) != RX_OK) return q;
                             if (fused) {
                               // the one-pass kernel runs where the scores are read (queue C),
                               // after the shifts (queue A) and the window-before copy (queue C)
                               HIPC(hipEventRecord(ps->ev_shift, qs.A));
                               HIPC(hipStreamWaitEvent(qs.C, ps->ev_shift, 0));
                               LaunchSet f;
                               const int nf = fill(f, grp, g0, g1, &Job::wg_fused);
                               if ((q = prof_mark(prof, 1, true, qs.C)) != RX_OK) return q;
                               HIPC(rxk_launch_onepass(&f, nf, jobs[grp[g0]].Bw, qs.C));
                               if ((q = prof_mark(prof, 1, false, qs.C)) != RX_OK) return q;
                               // the merge below waits for this event: the partials are written
                               HIPC(hipEventRecord(pe->ev_white[pe->par], qs.C));
                             } else {
                               if ((q = prof_mark(prof, 1, true, qs.A)) != RX_OK) return q;
                               HIPC(rxk_launch_stats(it, sp, 1, &b, n2, nullptr, 0, qs.A));
                               if ((q = prof_mark(prof, 1, false, qs.A)) != RX_OK) return q;
                             }
                             if (piped) HIPC(hipStreamWaitEvent(qs.A, pe->ev_white[pe->par], 0));
                             // causal: the latest whitening (and the copy before it) read
                             // the other parity's last slot, which this merge's successor
                             // overwrites; waiting here keeps one batch between them
                             if (piped && pe->causal_copy) HIPC(hipStreamWaitEvent(qs.A, pe->ev_white[pe->par ^ 1], 0));
                             if ((q = prof_mark(prof, 2, true, qs.A)) != RX_OK) return q;
                             HIPC(rxk_launch_stats(it, sp, 2, &c, n3, &e, n4, qs.A));
                             if ((q = prof_mark(prof, 2, false, qs.A)) != RX_OK) return q;
                             if (piped) {
                               HIPC(hipEventRecord(pe->ev_merged[pe->par], qs.A));
                               HIPC(hipStreamWaitEvent(qs.B, pe->ev_merged[pe->par], 0));
                             }
                             return RX_OK;
                           });
  if (r != RX_OK) return r;
  // one factor launch per whitening precision: each batch takes its own
  // operand pitch, and the template is sized by the launch's largest band count
  r = run_groups([](const Job& j) { return j.wp; },
                 [&](const std::vector<size_t>& grp, size_t g0, size_t g1) -> rx_status {
                   LaunchSet a;
                   const int n = fill(a, grp, g0, g1, &Job::wg_factor);
                   rx_status q;
                   if ((q = prof_mark(prof, 3, true, qs.B)) != RX_OK) return q;
                   HIPC(rxk_launch_factor(jobs[grp[g0]].wp, &a, n, qs.B));
                   return prof_mark(prof, 3, false, qs.B);
                 });
  if (r != RX_OK) return r;
  if (piped) {
    HIPC(hipEventRecord(pe->ev_fact, qs.B));
    if (!early && !fused) HIPC(hipStreamWaitEvent(qs.C, pe->ev_fact, 0));
  }
  return (early || fused) ? RX_OK : whiten_all();
}

// ---------------------------------------------------------------------------- push
// Host lines reach the device staging buffer in chunks of kHostChunk bytes:
// up to kHostThreads threads (the calling one and helpers started for the
// push) each take every T-th chunk, copy it into one of their two pinned
// buffers and queue its host-to-device copy on queue A, so the host copies
// of later chunks overlap the transfers of earlier ones.  A pinned buffer is
// refilled once its previous transfer is done (its event, a host wait);
// the staging buffer is overwritten on queue A only after the previous
// push's whitening, its last reader, is done (ev_stage).
static constexpr size_t kHostChunk = size_t(8) << 20;
static constexpr int kHostThreads = 8;

static rx_status stage_host_input(rx_stream* s, const void* lines, size_t bytes, const void** x) {
  if (s->stage_busy) {
    HIPC(hipStreamWaitEvent(s->stA, s->ev_stage, 0));
    s->stage_busy = false;
  }
  rx_status r = dev_ensure(s->stage, bytes, s);
  if (r != RX_OK) return r;
  const size_t nch = (bytes + kHostChunk - 1) / kHostChunk;
  const int T = (int)std::min<size_t>(kHostThreads, nch);
  while ((int)s->hslots.size() < 2 * T) {
    rx_stream::HostSlot hs;
    if (hipHostMalloc(&hs.p, kHostChunk, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(RX_E_NOMEM, "hipHostMalloc(%zu) failed", kHostChunk);
    }
    if (hipEventCreateWithFlags(&hs.ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipHostFree(hs.p);
      return fail(RX_E_DEVICE, "hipEventCreate failed");
    }
    s->hslots.push_back(hs);
  }
  // worker w copies chunks w, w + T, ... through its slots 2w and 2w + 1
  std::vector<hipError_t> err(T, hipSuccess);
  auto work = [&](int w) {
    hipError_t e = hipSetDevice(s->dev);
    int k = 0;
    for (size_t c = w; e == hipSuccess && c < nch; c += T, ++k) {
      rx_stream::HostSlot& hs = s->hslots[2 * w + (k & 1)];
      if (hs.busy && (e = hipEventSynchronize(hs.ev)) != hipSuccess) break;
      hs.busy = false;
      const size_t off = c * kHostChunk, len = std::min(kHostChunk, bytes - off);
      std::memcpy(hs.p, static_cast<const char*>(lines) + off, len);
      e = hipMemcpyAsync(static_cast<char*>(s->stage.p) + off, hs.p, len, hipMemcpyHostToDevice, s->stA);
      if (e == hipSuccess) e = hipEventRecord(hs.ev, s->stA);
      hs.busy = e == hipSuccess;
    }
    err[w] = e;
  };
  std::vector<std::thread> helpers;
  try {
    for (int w = 1; w < T; ++w) helpers.emplace_back(work, w);
  } catch (...) {
    for (auto& t : helpers) t.join();
    return fail(RX_E_STATE, "could not start the host copy threads");
  }
  work(0);
  for (auto& t : helpers) t.join();
  for (int w = 0; w < T; ++w)
    if (err[w] != hipSuccess) return fail(RX_E_DEVICE, "host input copy: %s", hipGetErrorString(err[w]));
  s->stage_busy = true;
  *x = s->stage.p;
  return RX_OK;
}

extern "C" rx_status rx_push_lines(rx_stream* s, const void* lines, int64_t n_lines, int32_t is_device_ptr,
                                   void* hip_stream) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  if (s->srv) return fail(RX_E_STATE, "served streams take blocks through rx_server_submit");
  if (!lines) return fail(RX_E_ARG, "null lines");
  if (n_lines < 1) return fail(RX_E_ARG, "n_lines must be >= 1");
  if (is_device_ptr < RX_LINES_HOST || is_device_ptr > RX_LINES_RESIDENT)
    return fail(RX_E_ARG, "is_device_ptr must be RX_LINES_HOST, RX_LINES_DEVICE or RX_LINES_RESIDENT");
  const bool resident = is_device_ptr == RX_LINES_RESIDENT;
  HIPC(hipSetDevice(s->dev));
  const size_t bytes = (size_t)n_lines * s->B * s->S * s->esz;
  const void* x = lines;
  std::vector<Block> blks;
  cut_blocks(s, s->lines_seen, n_lines, blks);
  for (const Block& bk : blks)
    if (bk.lines < 1) return fail(RX_E_ARG, "a block exceeds %d lines; set block_lines", INT32_MAX);
  // every allocation of the push happens here, before the stream changes
  const auto batches = plan_batches(blks);
  if ((r = reserve_batches(s, blks, batches)) != RX_OK) return r;
  const bool bip = s->cfg.layout == RX_BIP;
  if (bip && (r = dev_ensure(s->bip, bytes, s)) != RX_OK) return r;
  // A one-block device push to an idle stream (every earlier push done) runs
  // on one queue: no cross-queue handoffs, the lowest latency for a lone
  // block.  Other pushes go over the three queues, so that consecutive
  // pushes overlap (a multi-block push's factorisation and whitening run
  // beside the next push's covariance).  After a one-queue push, queue A
  // first waits for it: its shift and covariance reuse the scratch that push
  // read on queue C.
  bool one_queue = false;
  if (is_device_ptr && blks.size() == 1 && !s->causal) {
    const hipError_t q = hipEventQuery(s->ev_last);
    if (q != hipSuccess && q != hipErrorNotReady) return fail(RX_E_DEVICE, "hipEventQuery failed: %s", hipGetErrorString(q));
    one_queue = q == hipSuccess;
  }
  const Queues qs = one_queue ? Queues{s->st, s->st, s->st} : Queues{s->stA, s->stB, s->st};
  if (!one_queue && s->st_only_tail) HIPC(hipStreamWaitEvent(s->stA, s->ev_last, 0));
  if (!is_device_ptr) {
    if ((r = stage_host_input(s, lines, bytes, &x)) != RX_OK) return r;
  } else if (!resident) {
    HIPC(hipEventRecord(s->ev_in, static_cast<hipStream_t>(hip_stream)));
    HIPC(hipStreamWaitEvent(qs.A, s->ev_in, 0));     // queues B and C follow A by events
  }
  if (bip) {
    // BIP lines -> the BIL copy, once the previous push has stopped reading it
    HIPC(hipStreamWaitEvent(qs.A, s->ev_bip, 0));
    HIPC(rxk_launch_bip_to_bil(x, s->bip.p, n_lines, s->B, s->S, (int)s->esz, qs.A));
    x = s->bip.p;
    if (is_device_ptr) HIPC(hipEventRecord(s->ev_in, qs.A));   // the fast causal path waits for the copy
  }
  bool notready = false;
  s->N_push = s->N;
  s->push_reset = false;
  for (const auto& bt : batches) {
    const size_t i = bt.first, k = bt.second;
    std::vector<Job> jobs(1);
    if ((r = prepare_job(s, x, blks, i, k, jobs[0], notready, true)) != RX_OK) { s->broken = true; return r; }
    // (float input: the whitening also reads the validity pass's output)
    // (one-pass: every block of the batch whitens with the copied slot)
    jobs[0].fast = jobs[0].copy && (k - i == 1 || s->onepass) && is_device_ptr && !one_queue &&
                   s->in_type == RX_IN_U16 && !jobs[0].fused;
    if (one_queue) jobs[0].fused = 0;
    // resident lines need no input event (a BIP push's copy on queue A does)
    const Pipe pe{s->ev_merged, s->ev_fact, s->ev_white, jobs[0].par, s->causal != 0, !resident || bip};
    if ((r = launch_jobs(jobs, qs, &pe, s)) != RX_OK) { s->broken = true; return r; }
  }
  if (!is_device_ptr) HIPC(hipEventRecord(s->ev_stage, s->st));   // last reader of the staging buffer
  if (bip) HIPC(hipEventRecord(s->ev_bip, s->st));                 // last reader of the BIL copy
  HIPC(hipEventRecord(s->ev_last, s->st));
  s->st_only_tail = one_queue;
  s->lines_seen += n_lines;
  s->cnt.lines_pushed += n_lines;
  if (notready) return fail(RX_E_NOTREADY, "a block was scored with N <= B and no ridge; its scores are NaN");
  return RX_OK;
}

// ---------------------------------------------------------------------------- outputs
__global__ void k_f64_to_f32(const double* a, float* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_f32_to_f64(const float* a, double* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// A device output of the caller's may still be in use by earlier work on the
// caller's stream (a fill, a reader, torch recycling the memory): the
// library's queue waits for that work before writing it.
static rx_status after_caller(rx_stream* s, void* hip_stream) {
  HIPC(hipEventRecord(s->ev_in, static_cast<hipStream_t>(hip_stream)));
  HIPC(hipStreamWaitEvent(s->st, s->ev_in, 0));
  return RX_OK;
}

static rx_status pop_scores(rx_stream* s, void* out, int want_f64, int64_t max_px, int64_t* n_written,
                            int32_t out_is_device, void* hip_stream) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!n_written || (!out && max_px > 0) || max_px < 0) return fail(RX_E_ARG, "bad output arguments");
  HIPC(hipSetDevice(s->dev));
  const int64_t n = std::min(max_px, s->tail - s->head);
  *n_written = n;
  if (n == 0) return RX_OK;
  const size_t es = s->sc_f64 ? 8 : 4, eo = want_f64 ? 8 : 4;
  const char* src = static_cast<const char*>(s->pend[s->pcur].p) + (size_t)s->head * es;
  const void* from = src;
  if ((int)s->sc_f64 != want_f64) {
    if ((r = dev_ensure(s->cvt, (size_t)n * eo, s)) != RX_OK) return r;
    const int g = ceil_div(n, 256);
    if (want_f64) hipLaunchKernelGGL(k_f32_to_f64, dim3(g), dim3(256), 0, s->st, (const float*)src, (double*)s->cvt.p, n);
    else hipLaunchKernelGGL(k_f64_to_f32, dim3(g), dim3(256), 0, s->st, (const double*)src, (float*)s->cvt.p, n);
    HIPC(hipGetLastError());
    from = s->cvt.p;
  }
  if (out_is_device) {
    if ((r = after_caller(s, hip_stream)) != RX_OK) return r;
    HIPC(hipMemcpyAsync(out, from, (size_t)n * eo, hipMemcpyDeviceToDevice, s->st));
    HIPC(hipEventRecord(s->ev_done, s->st));
    HIPC(hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), s->ev_done, 0));
  } else {
    HIPC(hipStreamSynchronize(s->st));
    HIPC(hipMemcpy(out, from, (size_t)n * eo, hipMemcpyDeviceToHost));
  }
  s->head += n;
  if (s->head == s->tail) s->head = s->tail = 0;
  return RX_OK;
}

extern "C" rx_status rx_scores(rx_stream* s, float* out, int64_t max_px, int64_t* n_written, int32_t out_is_device,
                               void* hip_stream) {
  return pop_scores(s, out, 0, max_px, n_written, out_is_device, hip_stream);
}
extern "C" rx_status rx_scores_f64(rx_stream* s, double* out, int64_t max_px, int64_t* n_written,
                                   int32_t out_is_device, void* hip_stream) {
  return pop_scores(s, out, 1, max_px, n_written, out_is_device, hip_stream);
}

// ---------------------------------------------------------------------------- band selection and binning
extern "C" rx_status rx_bin_bands(const uint16_t* in, int64_t lines, int32_t bands, int32_t samples, int32_t b0,
                                  int32_t nb, int32_t k, int32_t bit_depth, uint16_t* out, void* hip_stream) {
  if (lines < 0 || bands < 1 || samples < 1) return fail(RX_E_ARG, "bad cube shape");
  if (k < 1 || nb < k || nb % k != 0) return fail(RX_E_ARG, "nb must be a positive multiple of k >= 1");
  if (b0 < 0 || (int64_t)b0 + nb > bands) return fail(RX_E_ARG, "bands [b0, b0 + nb) outside [0, bands)");
  if (bit_depth < 1 || bit_depth > 16) return fail(RX_E_ARG, "bit_depth must be in 1..16");
  if ((int64_t)k * ((1ll << bit_depth) - 1) > 65535)
    return fail(RX_E_ARG, "sums of %d counts of %d bits can exceed 16 bits", k, bit_depth);
  if (lines > 0 && (!in || !out)) return fail(RX_E_ARG, "null input or output");
  HIPC(rxk_launch_bin(in, out, lines, bands, samples, b0, nb / k, k, static_cast<hipStream_t>(hip_stream)));
  return RX_OK;
}

// ---------------------------------------------------------------------------- transmission encoding
static bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

extern "C" rx_status rx_tx_encode(const float* scores, int64_t n, uint16_t* codes, float* max_out, void* hip_stream) {
  if (n < 0) return fail(RX_E_ARG, "n must be >= 0");
  if (!max_out || !aligned4(max_out)) return fail(RX_E_ARG, "max_out must be a 4-byte aligned device pointer");
  if (n > 0 && (!scores || !codes)) return fail(RX_E_ARG, "null scores or codes");
  HIPC(rxk_launch_tx_encode(scores, 0, n, codes, max_out, static_cast<hipStream_t>(hip_stream)));
  return RX_OK;
}

extern "C" rx_status rx_tx_decode(const uint16_t* codes, int64_t n, const float* max_in, float tau, float* delta,
                                  uint32_t* bits, void* hip_stream) {
  if (n < 0) return fail(RX_E_ARG, "n must be >= 0");
  if (std::isnan(tau)) return fail(RX_E_ARG, "tau is NaN");
  if (!max_in || !aligned4(max_in)) return fail(RX_E_ARG, "max_in must be a 4-byte aligned device pointer");
  if (n > 0 && !codes) return fail(RX_E_ARG, "null codes");
  if (bits && !aligned4(bits)) return fail(RX_E_ARG, "bits must be 4-byte aligned");
  HIPC(rxk_launch_tx_decode(codes, n, max_in, tau, delta, bits, static_cast<hipStream_t>(hip_stream)));
  return RX_OK;
}

extern "C" rx_status rx_encode(rx_stream* s, uint16_t* codes, int64_t max_px, int64_t* n_px, float* max_out,
                               void* hip_stream) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!n_px) return fail(RX_E_ARG, "null n_px");
  if (!max_out || !aligned4(max_out)) return fail(RX_E_ARG, "max_out must be a 4-byte aligned device pointer");
  HIPC(hipSetDevice(s->dev));
  const int64_t n = s->tail - s->head;
  *n_px = n;
  if (n > 0 && (!codes || max_px < n)) return fail(RX_E_ARG, "codes buffer needs %lld entries", (long long)n);
  const void* src = static_cast<const char*>(s->pend[s->pcur].p) + (size_t)s->head * (s->sc_f64 ? 8 : 4);
  if ((r = after_caller(s, hip_stream)) != RX_OK) return r;
  HIPC(rxk_launch_tx_encode(src, s->sc_f64, n, codes, max_out, s->st));
  HIPC(hipEventRecord(s->ev_done, s->st));
  HIPC(hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), s->ev_done, 0));
  return RX_OK;
}

extern "C" rx_status rx_mask(rx_stream* s, double tau, int32_t mode, int64_t k, uint8_t* bits, int64_t max_bytes,
                             int64_t* n_px, int32_t out_is_device, void* hip_stream) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!n_px) return fail(RX_E_ARG, "null n_px");
  if (mode < RX_THR_ABS || mode > RX_THR_TOPK) return fail(RX_E_ARG, "bad threshold mode");
  if (mode == RX_THR_TOPK && k < 0) return fail(RX_E_ARG, "k must be >= 0");
  if (mode != RX_THR_TOPK && std::isnan(tau)) return fail(RX_E_ARG, "tau is NaN");
  HIPC(hipSetDevice(s->dev));
  const int64_t n = s->tail - s->head;
  const int64_t nbytes = (n + 7) / 8;
  *n_px = n;
  if (n == 0) return RX_OK;
  if (!bits || max_bytes < nbytes) return fail(RX_E_ARG, "mask buffer needs %lld bytes", (long long)nbytes);
  const int64_t words = (n + 31) / 32;
  if ((r = dev_ensure(s->maskbits, (size_t)words * 4, s)) != RX_OK) return r;
  if ((r = dev_ensure(s->maskscr, 4096, s)) != RX_OK) return r;
  const void* src = static_cast<const char*>(s->pend[s->pcur].p) + (size_t)s->head * (s->sc_f64 ? 8 : 4);
  if (mode == RX_THR_TOPK && k == 0) {
    HIPC(hipMemsetAsync(s->maskbits.p, 0, (size_t)words * 4, s->st));
  } else {
    HIPC(rxk_launch_mask(src, s->sc_f64, n, mode, tau, k, static_cast<uint32_t*>(s->maskbits.p), s->maskscr.p, s->st));
  }
  if (out_is_device) {
    if ((r = after_caller(s, hip_stream)) != RX_OK) return r;
    HIPC(hipMemcpyAsync(bits, s->maskbits.p, (size_t)nbytes, hipMemcpyDeviceToDevice, s->st));
    HIPC(hipEventRecord(s->ev_done, s->st));
    HIPC(hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), s->ev_done, 0));
  } else {
    HIPC(hipStreamSynchronize(s->st));
    HIPC(hipMemcpy(bits, s->maskbits.p, (size_t)nbytes, hipMemcpyDeviceToHost));
  }
  return RX_OK;
}

// rx_mask for callers that cannot allocate: the maximum key, top-k state and
// histogram and the mask words live in the GPU's fixed working array (set
// up by rx_init); the words are then copied to the caller's device bits by a
// kernel.  No hipMalloc, hipFree, memset or library allocation on this path.
extern "C" rx_status rx_mask_noalloc(rx_stream* s, double tau, int32_t mode, int64_t k, uint8_t* bits,
                                     int64_t max_bytes, int64_t* n_px, void* hip_stream) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!n_px) return fail(RX_E_ARG, "null n_px");
  if (mode < RX_THR_ABS || mode > RX_THR_TOPK) return fail(RX_E_ARG, "bad threshold mode");
  if (mode == RX_THR_TOPK && k < 0) return fail(RX_E_ARG, "k must be >= 0");
  if (mode != RX_THR_TOPK && std::isnan(tau)) return fail(RX_E_ARG, "tau is NaN");
  void* ws = nullptr;
  size_t head = 0, cap = 0;
  {
    std::lock_guard<std::mutex> lk(g_na_mu);
    ws = g_na_ptr[s->dev];
    head = g_na_head;
    cap = g_na_bytes;
  }
  if (!ws) return fail(RX_E_STATE, "the allocation-free mask is not set up on device %d", s->dev);
  const int64_t n = s->tail - s->head;
  const int64_t nbytes = (n + 7) / 8, words = (n + 31) / 32;
  *n_px = n;
  if (n == 0) return RX_OK;
  if (!bits || max_bytes < nbytes) return fail(RX_E_ARG, "mask buffer needs %lld bytes", (long long)nbytes);
  const int64_t max_px = (int64_t)(cap - head) / 4 * 32;
  if (n > max_px)
    return fail(RX_E_ARG, "%lld pending pixels exceed the allocation-free mask's limit of %lld", (long long)n,
                (long long)max_px);
  HIPC(hipSetDevice(s->dev));
  const void* src = static_cast<const char*>(s->pend[s->pcur].p) + (size_t)s->head * (s->sc_f64 ? 8 : 4);
  uint32_t* wbits = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + head);
  if ((r = after_caller(s, hip_stream)) != RX_OK) return r;
  if (mode == RX_THR_TOPK && k == 0) HIPC(rxk_launch_zero_words(wbits, words, s->st));
  else HIPC(rxk_launch_mask(src, s->sc_f64, n, mode, tau, k, wbits, ws, s->st));
  HIPC(rxk_launch_copy_bytes(wbits, bits, nbytes, s->st));
  HIPC(hipEventRecord(s->ev_done, s->st));
  HIPC(hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), s->ev_done, 0));
  return RX_OK;
}

// ---------------------------------------------------------------------------- sync / counters / hooks
static rx_status refresh_counters(rx_stream* s) {
  HIPC(hipSetDevice(s->dev));
  HIPC(sync_all(s));
  struct { unsigned ns, nr; unsigned long long bad, clip, sclip; } c{};
  HIPC(hipMemcpy(&c, s->nsing.p, sizeof c, hipMemcpyDeviceToHost));
  double n = 0.0;
  HIPC(hipMemcpy(&n, static_cast<double*>(s->s1[s->cur].p) + s->Bp, sizeof n, hipMemcpyDeviceToHost));
  const unsigned ns = c.ns;
  if (ns > s->last_nsing && s->sticky == RX_OK) s->sticky = RX_E_SINGULAR;
  s->last_nsing = ns;
  s->cnt.singular_blocks = ns;
  s->cnt.notready_blocks = c.nr;
  s->cnt.nonfinite_px = (int64_t)c.bad;
  s->cnt.fp8_saturated = (int64_t)c.clip;
  s->cnt.fp8_syrk_saturated = (int64_t)c.sclip;
  s->cnt.pending_px = s->tail - s->head;
  s->cnt.window_px = (int64_t)n;
  return RX_OK;
}

extern "C" rx_status rx_wait(rx_stream* s, void* hip_stream) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  HIPC(hipSetDevice(s->dev));
  HIPC(hipEventRecord(s->ev_done, s->st));
  HIPC(hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), s->ev_done, 0));
  return RX_OK;
}

extern "C" rx_status rx_sync(rx_stream* s) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if ((r = refresh_counters(s)) != RX_OK) return r;
  const rx_status st = s->sticky;
  s->sticky = RX_OK;
  if (st == RX_E_SINGULAR) return fail(st, "a block hit a non-positive pivot in the FP64 Cholesky; its scores are NaN");
  return RX_OK;
}

extern "C" rx_status rx_get_counters(rx_stream* s, rx_counters* out) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!out) return fail(RX_E_ARG, "null counters");
  if ((r = refresh_counters(s)) != RX_OK) return r;
  *out = s->cnt;
  return RX_OK;
}

extern "C" const char* rx_last_error(void) { return g_err.c_str(); }

extern "C" rx_status rx_profile(rx_stream* s, int32_t enable) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  HIPC(hipSetDevice(s->dev));
  HIPC(sync_all(s));
  if ((r = prof_collect(s)) != RX_OK) return r;
  s->prof = enable != 0;
  for (int i = 0; i < 5; ++i) { s->prof_ms[i] = 0.0; s->prof_n[i] = 0; }
  return RX_OK;
}

extern "C" rx_status rx_phase_times(rx_stream* s, double* ms, int64_t* launches) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!ms || !launches) return fail(RX_E_ARG, "null output");
  HIPC(hipSetDevice(s->dev));
  HIPC(sync_all(s));
  if ((r = prof_collect(s)) != RX_OK) return r;
  for (int i = 0; i < 5; ++i) { ms[i] = s->prof_ms[i]; launches[i] = s->prof_n[i]; }
  return RX_OK;
}

extern "C" rx_status rx_get_stats(rx_stream* s, int64_t* n, double* mean, double* cov) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!n) return fail(RX_E_ARG, "null n");
  HIPC(hipSetDevice(s->dev));
  HIPC(sync_all(s));
  const int B = s->B, Bp = s->Bp;
  std::vector<double> s1(Bp + 1), m2((size_t)Bp * Bp);
  HIPC(hipMemcpy(s1.data(), s->s1[s->cur].p, (size_t)(Bp + 1) * 8, hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(m2.data(), s->m2[s->cur].p, (size_t)Bp * Bp * 8, hipMemcpyDeviceToHost));
  const int64_t N = (int64_t)s1[Bp];            // finite pixels in the window
  *n = N;
  if (mean)
    for (int k = 0; k < B; ++k) mean[k] = N > 0 ? s1[k] / (double)N : NAN;
  if (cov) {
    const double den = (double)(N - s->cfg.ddof);
    for (int i = 0; i < B; ++i)
      for (int j = 0; j <= i; ++j) cov[(size_t)i * B + j] = cov[(size_t)j * B + i] = m2[(size_t)i * Bp + j] / den;
  }
  return RX_OK;
}

extern "C" rx_status rx_set_stats(rx_stream* s, int64_t n, const double* mean, const double* cov) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (n < 0 || (n > 0 && (!mean || !cov))) return fail(RX_E_ARG, "bad statistics");
  if (n > 0 && n <= s->cfg.ddof) return fail(RX_E_ARG, "n must exceed ddof");
  HIPC(hipSetDevice(s->dev));
  HIPC(sync_all(s));
  const int B = s->B, Bp = s->Bp;
  std::vector<double> s1(Bp + 1, 0.0), m2((size_t)Bp * Bp, 0.0);
  if (n > 0) {
    const double den = (double)(n - s->cfg.ddof);
    for (int k = 0; k < B; ++k) s1[k] = mean[k] * (double)n;
    for (int i = 0; i < B; ++i)
      for (int j = 0; j <= i; ++j) m2[(size_t)i * Bp + j] = cov[(size_t)i * B + j] * den;
  }
  s1[Bp] = (double)n;
  HIPC(hipMemcpy(s->s1[s->cur].p, s1.data(), (size_t)(Bp + 1) * 8, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(s->m2[s->cur].p, m2.data(), (size_t)Bp * Bp * 8, hipMemcpyHostToDevice));
  s->N = n;
  s->prev_valid = false;          // causal: the next batch forms its window-before slot itself
  return RX_OK;
}

extern "C" rx_status rx_get_whitener(rx_stream* s, double* w) {
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  SrvLock held(s);
  if (!w) return fail(RX_E_ARG, "null output");
  if (s->last_w_off < 0) return fail(RX_E_STATE, "no block has been factored yet");
  HIPC(hipSetDevice(s->dev));
  HIPC(sync_all(s));
  const int B = s->B, Bp = s->Bp;
  std::vector<double> full((size_t)Bp * Bp);
  HIPC(hipMemcpy(full.data(), static_cast<double*>(s->w64[s->last_par].p) + s->last_w_off, full.size() * 8,
                 hipMemcpyDeviceToHost));
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < B; ++j) w[(size_t)i * B + j] = full[(size_t)i * Bp + j];
  return RX_OK;
}

// ---------------------------------------------------------------------------- server
static void free_server(rx_server* srv) {
  for (auto& f : srv->inflight) srv->free_events.push_back(f.ev);
  for (hipEvent_t e : srv->free_events) (void)hipEventDestroy(e);
  hipEvent_t evs[] = {srv->ev_merged[0], srv->ev_merged[1], srv->ev_fact, srv->ev_white[0], srv->ev_white[1]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (srv->st) (void)hipStreamDestroy(srv->st);
  if (srv->stA) (void)hipStreamDestroy(srv->stA);
  if (srv->stB) (void)hipStreamDestroy(srv->stB);
  srv->magic = 0;
  delete srv;
}

extern "C" rx_status rx_server_create(size_t hbm_budget_bytes, int32_t max_streams, int32_t device, rx_server** out) {
  if (!out) return fail(RX_E_ARG, "null output handle");
  *out = nullptr;
  if (max_streams < 1) return fail(RX_E_ARG, "max_streams must be >= 1");
  int ndev = 0;
  HIPC(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(RX_E_ARG, "device %d not present", device);
  HIPC(hipSetDevice(device));
  rx_server* srv = new rx_server();
  srv->budget = hbm_budget_bytes;
  srv->max_streams = max_streams;
  srv->dev = device;
  if (hipStreamCreateWithFlags(&srv->st, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&srv->stA, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&srv->stB, hipStreamNonBlocking) != hipSuccess) {
    free_server(srv);
    return fail(RX_E_DEVICE, "hipStreamCreate failed");
  }
  hipEvent_t* evs[] = {&srv->ev_merged[0], &srv->ev_merged[1], &srv->ev_fact, &srv->ev_white[0], &srv->ev_white[1]};
  for (hipEvent_t* e : evs)
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      free_server(srv);
      return fail(RX_E_DEVICE, "hipEventCreate failed");
    }
  // the parity events start out recorded (nothing to wait for)
  for (int q = 0; q < 2; ++q)
    if (hipEventRecord(srv->ev_white[q], srv->st) != hipSuccess) {
      free_server(srv);
      return fail(RX_E_DEVICE, "hipEventRecord failed");
    }
  *out = srv;
  return RX_OK;
}

static rx_status stop_loop(rx_server* srv);

extern "C" rx_status rx_server_destroy(rx_server* srv) {
  if (!srv) return RX_OK;
  if (srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  (void)hipSetDevice(srv->dev);
  if (srv->n_streams > 0) return fail(RX_E_STATE, "destroy the server's %d streams first", srv->n_streams);
  (void)stop_loop(srv);
  (void)hipStreamSynchronize(srv->st);
  (void)hipStreamSynchronize(srv->stA);
  (void)hipStreamSynchronize(srv->stB);
  free_server(srv);
  return RX_OK;
}

extern "C" rx_status rx_server_submit(rx_server* srv, rx_stream* s, const void* lines_dev, int64_t n_lines,
                                      uint64_t tag) {
  if (!srv || srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  rx_status r = check_stream(s);
  if (r != RX_OK) return r;
  if (s->srv != srv) return fail(RX_E_STATE, "stream is not admitted on this server");
  if (!lines_dev || n_lines < 1) return fail(RX_E_ARG, "bad block");
  const int mbl = s->cfg.block_lines > 0 ? s->cfg.block_lines : 128;
  if (n_lines > mbl) return fail(RX_E_ARG, "block of %lld lines exceeds the stream's %d", (long long)n_lines, mbl);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    // the block starts where the stream's queued blocks end: it must end at or
    // before the next window edge (refused here, so a step never meets it)
    const int64_t R = s->cfg.window_lines, pos = s->lines_seen + s->q_lines;
    if (R > 0 && pos % R + n_lines > R)
      return fail(RX_E_ARG, "block of %lld lines at line %lld straddles a window edge (every %lld lines)",
                  (long long)n_lines, (long long)pos, (long long)R);
    srv->queue.push_back(Pending{s, lines_dev, n_lines, tag});
    s->q_lines += n_lines;
  }
  srv->cv.notify_one();
  return RX_OK;
}

// One batched step: the oldest queued block of every stream that has one,
// launched over the server's three queues (with the lock held).  Queue A
// runs the statistics of this step while queues B and C still run the
// factorisation and whitening of the previous one.
static rx_status step_locked(rx_server* srv, int32_t* n_blocks) {
  if (n_blocks) *n_blocks = 0;
  // one block per stream per step (a stream's blocks depend on each other):
  // the oldest queued block of each stream, left in the queue until every
  // allocation of the step has succeeded
  std::vector<size_t> pick;
  std::vector<std::vector<Block>> blks;
  for (size_t q = 0; q < srv->queue.size(); ++q) {
    bool seen = false;
    for (size_t t : pick) seen |= (srv->queue[t].s == srv->queue[q].s);
    if (seen || srv->queue[q].s->broken) continue;
    pick.push_back(q);
  }
  if (pick.empty()) return RX_OK;
  blks.resize(pick.size());
  for (size_t i = 0; i < pick.size(); ++i) {
    const Pending& pq = srv->queue[pick[i]];
    cut_blocks(pq.s, pq.s->lines_seen, pq.lines, blks[i]);
    if (blks[i].size() != 1) return fail(RX_E_STATE, "internal: a queued block straddles a window edge");
  }
  for (size_t i = 0; i < pick.size(); ++i) {
    rx_status r = reserve_batches(srv->queue[pick[i]].s, blks[i], {{0, 1}});
    if (r != RX_OK) return r;                 // nothing taken, no stream changed
  }
  // from here on the step is committed
  std::vector<Pending> take;
  for (size_t t : pick) take.push_back(srv->queue[t]);
  for (size_t i = pick.size(); i-- > 0;) srv->queue.erase(srv->queue.begin() + (std::ptrdiff_t)pick[i]);
  std::vector<Job> jobs(take.size());
  InFlight f;
  for (size_t i = 0; i < take.size(); ++i) {
    rx_stream* s = take[i].s;
    bool notready = false;
    s->N_push = s->N;                      // a served block is a push of its own
    s->push_reset = false;
    rx_status r = prepare_job(s, take[i].x, blks[i], 0, 1, jobs[i], notready);
    if (r != RX_OK) {
      for (size_t k = 0; k <= i; ++k) take[k].s->broken = true;
      return r;
    }
    s->lines_seen += take[i].lines;
    s->q_lines -= take[i].lines;
    s->cnt.lines_pushed += take[i].lines;
    f.items.push_back({s, take[i].tag});
  }
  const Pipe pe{srv->ev_merged, srv->ev_fact, srv->ev_white, srv->spar, false};
  rx_status r = launch_jobs(jobs, Queues{srv->stA, srv->stB, srv->st}, &pe);
  if (r == RX_OK && srv->free_events.empty()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) r = fail(RX_E_DEVICE, "hipEventCreate failed");
    else srv->free_events.push_back(e);
  }
  if (r == RX_OK) {
    f.ev = srv->free_events.back();
    if (hipEventRecord(f.ev, srv->st) != hipSuccess) r = fail(RX_E_DEVICE, "hipEventRecord failed");
    else srv->free_events.pop_back();
  }
  if (r != RX_OK) {
    // the streams' state has advanced past blocks whose work did not launch
    for (auto& t : take) t.s->broken = true;
    return r;
  }
  srv->spar ^= 1;
  srv->inflight.push_back(std::move(f));
  srv->loop_steps += 1;
  if (n_blocks) *n_blocks = (int32_t)take.size();
  return RX_OK;
}

extern "C" rx_status rx_server_step(rx_server* srv, int32_t* n_blocks) {
  if (!srv || srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  if (n_blocks) *n_blocks = 0;
  HIPC(hipSetDevice(srv->dev));
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->running) return fail(RX_E_STATE, "the server's request loop is running; it steps by itself");
  return step_locked(srv, n_blocks);
}

// Move finished steps (in launch order) to the done list; block: wait for all.
static rx_status collect_locked(rx_server* srv, bool block, int64_t stamp) {
  while (!srv->inflight.empty()) {
    InFlight& f = srv->inflight.front();
    if (block) {
      HIPC(hipEventSynchronize(f.ev));
    } else {
      const hipError_t q = hipEventQuery(f.ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return fail(RX_E_DEVICE, "hipEventQuery: %s", hipGetErrorString(q));
    }
    const int64_t t = stamp ? clock_ns() : 0;
    for (auto& it : f.items) srv->done.push_back(Done{it.second, t});
    srv->free_events.push_back(f.ev);
    srv->inflight.pop_front();
  }
  return RX_OK;
}

// The persistent request loop: launch a step whenever blocks are queued and
// fewer than kLoopDepth steps are in flight (blocks arriving meanwhile join
// the next step), and stamp finished steps as soon as their event completes.
static constexpr size_t kLoopDepth = 2;
static void loop_main(rx_server* srv) {
  (void)hipSetDevice(srv->dev);
  std::unique_lock<std::mutex> lk(srv->mu);
  while (!srv->stop) {
    bool progress = false;
    const size_t before = srv->done.size();
    rx_status r = collect_locked(srv, false, true);
    if (r == RX_OK && srv->inflight.size() < kLoopDepth && !srv->queue.empty()) {
      int32_t nb = 0;
      r = step_locked(srv, &nb);
      progress = nb > 0;
    }
    if (r != RX_OK && srv->loop_err == RX_OK) {
      srv->loop_err = r;
      srv->loop_msg = g_err;
    }
    progress |= srv->done.size() != before;
    if (!progress) {
      // nothing to launch: sleep until a submission or a short poll period
      // (completions are stamped within about that period)
      srv->cv.wait_for(lk, std::chrono::microseconds(srv->inflight.empty() ? 2000 : 20));
    }
  }
}

extern "C" rx_status rx_server_start(rx_server* srv) {
  if (!srv || srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->running) return fail(RX_E_STATE, "the request loop is already running");
  srv->stop = false;
  srv->loop_err = RX_OK;
  srv->running = true;
  try {
    srv->loop = std::thread(loop_main, srv);
  } catch (...) {
    srv->running = false;
    return fail(RX_E_STATE, "could not start the request loop thread");
  }
  return RX_OK;
}

static rx_status stop_loop(rx_server* srv) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->running) return RX_OK;
    srv->stop = true;
  }
  srv->cv.notify_all();
  srv->loop.join();
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->running = false;
  if (srv->loop_err != RX_OK) return fail(srv->loop_err, "request loop: %s", srv->loop_msg.c_str());
  return RX_OK;
}

extern "C" rx_status rx_server_stop(rx_server* srv) {
  if (!srv || srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  return stop_loop(srv);
}

extern "C" int64_t rx_clock_ns(void) { return clock_ns(); }

extern "C" rx_status rx_server_poll_ns(rx_server* srv, uint64_t* tags, int64_t* done_ns, int32_t max_tags,
                                       int32_t* n_done, int32_t block) {
  if (!srv || srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  if (!n_done || (!tags && max_tags > 0)) return fail(RX_E_ARG, "bad output arguments");
  *n_done = 0;
  HIPC(hipSetDevice(srv->dev));
  std::unique_lock<std::mutex> lk(srv->mu);
  if (!srv->running || block) {
    rx_status r = collect_locked(srv, block && !srv->running, srv->running);
    if (r != RX_OK) return r;
    if (block && srv->running)                 // the loop collects: wait until it has everything
      while (!srv->inflight.empty() || !srv->queue.empty()) {
        if (srv->loop_err != RX_OK) return fail(srv->loop_err, "request loop: %s", srv->loop_msg.c_str());
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
  }
  int32_t n = 0;
  while (!srv->done.empty() && n < max_tags) {
    tags[n] = srv->done.front().tag;
    if (done_ns) done_ns[n] = srv->done.front().t_ns;
    srv->done.pop_front();
    ++n;
  }
  *n_done = n;
  if (srv->loop_err != RX_OK) return fail(srv->loop_err, "request loop: %s", srv->loop_msg.c_str());
  return RX_OK;
}

extern "C" rx_status rx_server_poll(rx_server* srv, uint64_t* tags, int32_t max_tags, int32_t* n_done, int32_t block) {
  return rx_server_poll_ns(srv, tags, nullptr, max_tags, n_done, block);
}

extern "C" rx_status rx_server_sync(rx_server* srv) {
  if (!srv || srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  HIPC(hipSetDevice(srv->dev));
  HIPC(hipStreamSynchronize(srv->stA));
  HIPC(hipStreamSynchronize(srv->stB));
  HIPC(hipStreamSynchronize(srv->st));
  return RX_OK;
}

extern "C" rx_status rx_server_queued(rx_server* srv, int32_t* queued, int32_t* inflight, size_t* used_bytes) {
  if (!srv || srv->magic != 0x52585356u) return fail(RX_E_STATE, "server handle is not live");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (queued) *queued = (int32_t)srv->queue.size();
  if (inflight) {
    int32_t c = 0;
    for (auto& f : srv->inflight) c += (int32_t)f.items.size();
    *inflight = c;
  }
  if (used_bytes) *used_bytes = srv->used;
  return RX_OK;
}
