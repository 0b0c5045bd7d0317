// Device-side building blocks shared by the RX kernels (gfx950 / CDNA4 only).
//
// Layout conventions
//  * Input lines are BIL: x[line][band][sample]; pixel p = line * S + sample.
//  * Bands are padded to Bp = 16 * ceil(B / 16) in every device matrix; the
//    padding rows/columns hold zeros (identity on the diagonal of the
//    equilibrated covariance) so every 16x16 matrix-core tile is whole.
//  * Matrix-core tiles are 16 x 16 outputs (v_mfma_*_16x16x*): lane l owns
//    four outputs of column l%16 -- rows 4*(l/16)+j (j = 0..3) for the FP32-
//    accumulating formats, rows (l/16)+4*j for v_mfma_f64_16x16x4f64 (checked
//    on gfx950 with a unique-value probe); operand lanes own row/column l%16
//    and the k-group l/16 of KV consecutive k values.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rxk {

enum InType { IN_U16 = 0, IN_F32 = 1, IN_F64 = 2 };
enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_F16 = 3, P_FP8 = 4 };

constexpr int TILE = 16;      // matrix-core output tile edge (bands)
constexpr int SUP = 64;       // covariance super-tile edge owned by one workgroup
constexpr int MAXT = 20;      // max 16-band tiles: B <= 320
constexpr int KC = 64;        // pixels per chunk (one line segment)
constexpr int MAXB = 8;       // batches per launch (kernel-argument descriptors)
constexpr int NT = 256;       // threads per workgroup of the streaming kernels
constexpr int CPWG = 32;      // workgroups per batch of the snapshot-slot copy (causal mode)

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) double f64x4;

// ------------------------------------------------------------------ per-precision traits
// storage: element type kept in LDS / global for the operand;  frag: operand
// register type;  acc: accumulator vector;  KV: k values per lane;  KK: k per
// instruction.
template <int P> struct MM;

template <> struct MM<P_F64> {
  using storage = double; using frag = double; using acc = f64x4; using accs = double;
  static constexpr int KV = 1, KK = 4;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int j) { return g + 4 * j; }
};
template <> struct MM<P_F32> {
  using storage = float; using frag = float; using acc = f32x4; using accs = float;
  static constexpr int KV = 1, KK = 4;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int j) { return 4 * g + j; }
};
template <> struct MM<P_BF16> {
  using storage = uint16_t; using frag = bf16x8; using acc = f32x4; using accs = float;
  static constexpr int KV = 8, KK = 32;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int j) { return 4 * g + j; }
};
template <> struct MM<P_F16> {
  using storage = uint16_t; using frag = f16x8; using acc = f32x4; using accs = float;
  static constexpr int KV = 8, KK = 32;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int j) { return 4 * g + j; }
};
template <> struct MM<P_FP8> {
  using storage = uint8_t; using frag = long; using acc = f32x4; using accs = float;
  static constexpr int KV = 8, KK = 32;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int j) { return 4 * g + j; }
};

// ------------------------------------------------------------------ conversions (RNE)
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  __bf16 h = (__bf16)f;                       // round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ uint16_t f32_to_f16_bits(float f) {
  _Float16 h = (_Float16)f;                   // round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}
// OCP FP8 E4M3 (bias 7, max finite 448, no infinities, 0x7F/0xFF are NaN):
// round to nearest even; magnitudes above 448 saturate to 448; subnormals
// (m * 2^-9) are kept.
__device__ __forceinline__ uint8_t f32_to_e4m3(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  uint32_t sign = (u >> 24) & 0x80u;
  float a = __builtin_fabsf(f);
  if (!(a == a)) return (uint8_t)(sign | 0x7Fu);
  if (a >= 448.0f) return (uint8_t)(sign | 0x7Eu);
  if (a < 0.015625f) {                        // below 2^-6: subnormal grid of 2^-9
    float m = __builtin_rintf(a * 512.0f);    // 0..8 (8 = smallest normal)
    return (uint8_t)(sign | (uint32_t)m);
  }
  int e = (int)((__builtin_bit_cast(uint32_t, a) >> 23) & 0xff) - 127;   // -6..8
  float scaled = __builtin_ldexpf(a, -e);     // [1, 2)
  float m = __builtin_rintf((scaled - 1.0f) * 8.0f);
  uint32_t mi = (uint32_t)m;
  if (mi == 8u) { mi = 0; ++e; }
  if (e > 8 || (e == 8 && mi == 7u)) return (uint8_t)(sign | 0x7Eu);
  return (uint8_t)(sign | ((uint32_t)(e + 7) << 3) | mi);
}

template <int P> __device__ __forceinline__ typename MM<P>::storage to_storage(float v);
template <> __device__ __forceinline__ double to_storage<P_F64>(float v) { return v; }
template <> __device__ __forceinline__ float to_storage<P_F32>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t to_storage<P_BF16>(float v) { return f32_to_bf16_bits(v); }
template <> __device__ __forceinline__ uint16_t to_storage<P_F16>(float v) { return f32_to_f16_bits(v); }
template <> __device__ __forceinline__ uint8_t to_storage<P_FP8>(float v) { return f32_to_e4m3(v); }

// Round two FP32 values to the operand format (RNE) and pack them, low
// value first.  BF16 and FP16 convert both in one instruction.
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) _Float16 f16x2;
typedef __attribute__((ext_vector_type(2))) unsigned short u16x2;
template <int P> __device__ __forceinline__ uint32_t cvt_pack2(float a, float b);
template <> __device__ __forceinline__ uint32_t cvt_pack2<P_BF16>(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
template <> __device__ __forceinline__ uint32_t cvt_pack2<P_F16>(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, f16x2));
}
// Load one operand fragment: KV consecutive storage elements at p.
template <int P> __device__ __forceinline__ typename MM<P>::frag load_frag(const typename MM<P>::storage* p);
template <> __device__ __forceinline__ double load_frag<P_F64>(const double* p) { return *p; }
template <> __device__ __forceinline__ float load_frag<P_F32>(const float* p) { return *p; }
template <> __device__ __forceinline__ bf16x8 load_frag<P_BF16>(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
template <> __device__ __forceinline__ f16x8 load_frag<P_F16>(const uint16_t* p) {
  return __builtin_bit_cast(f16x8, *reinterpret_cast<const uint4*>(p));
}
template <> __device__ __forceinline__ long load_frag<P_FP8>(const uint8_t* p) {
  return __builtin_bit_cast(long, *reinterpret_cast<const uint2*>(p));
}

// ------------------------------------------------------------------ input element access
template <int IN> struct InT;
template <> struct InT<IN_U16> { using T = uint16_t; };
template <> struct InT<IN_F32> { using T = float; };
template <> struct InT<IN_F64> { using T = double; };

template <typename T> __device__ __forceinline__ double to_d(T v) { return (double)v; }

// Eight consecutive input values from a 16-byte aligned address (vector loads).
__device__ __forceinline__ void load8(const uint16_t* p, uint16_t v[8]) {
  const uint4 q = *reinterpret_cast<const uint4*>(p);
  v[0] = q.x & 0xffff; v[1] = q.x >> 16; v[2] = q.y & 0xffff; v[3] = q.y >> 16;
  v[4] = q.z & 0xffff; v[5] = q.z >> 16; v[6] = q.w & 0xffff; v[7] = q.w >> 16;
}
// The same from an 8-byte aligned address (two 8-byte loads): 16-bit rows
// with S % 4 == 0, such as the imager's 900-sample lines.
__device__ __forceinline__ void load8_a8(const uint16_t* p, uint16_t v[8]) {
  const uint2 a = reinterpret_cast<const uint2*>(p)[0], b = reinterpret_cast<const uint2*>(p)[1];
  v[0] = a.x & 0xffff; v[1] = a.x >> 16; v[2] = a.y & 0xffff; v[3] = a.y >> 16;
  v[4] = b.x & 0xffff; v[5] = b.x >> 16; v[6] = b.y & 0xffff; v[7] = b.y >> 16;
}
template <typename T> __device__ __forceinline__ void load8_a8(const T*, T*) {}
__device__ __forceinline__ void load8(const float* p, float v[8]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ __forceinline__ void load8(const double* p, double v[8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 a = *reinterpret_cast<const double2*>(p + 2 * i);
    v[2 * i] = a.x; v[2 * i + 1] = a.y;
  }
}

// Eight input values <-> 16-byte words, in registers (no memory round trip).
__device__ __forceinline__ void unpack8(const uint4* w, uint16_t v[8]) {
  v[0] = w[0].x & 0xffff; v[1] = w[0].x >> 16; v[2] = w[0].y & 0xffff; v[3] = w[0].y >> 16;
  v[4] = w[0].z & 0xffff; v[5] = w[0].z >> 16; v[6] = w[0].w & 0xffff; v[7] = w[0].w >> 16;
}
__device__ __forceinline__ void pack8(const uint16_t v[8], uint4* w) {
  w[0] = uint4{(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
               (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16)};
}
__device__ __forceinline__ void unpack8(const uint4* w, float v[8]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    v[4 * i] = __builtin_bit_cast(float, w[i].x); v[4 * i + 1] = __builtin_bit_cast(float, w[i].y);
    v[4 * i + 2] = __builtin_bit_cast(float, w[i].z); v[4 * i + 3] = __builtin_bit_cast(float, w[i].w);
  }
}
__device__ __forceinline__ void pack8(const float v[8], uint4* w) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
    w[i] = uint4{__builtin_bit_cast(uint32_t, v[4 * i]), __builtin_bit_cast(uint32_t, v[4 * i + 1]),
                 __builtin_bit_cast(uint32_t, v[4 * i + 2]), __builtin_bit_cast(uint32_t, v[4 * i + 3])};
}
__device__ __forceinline__ void unpack8(const uint4* w, double v[8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __builtin_bit_cast(double, uint2{w[i].x, w[i].y});
    v[2 * i + 1] = __builtin_bit_cast(double, uint2{w[i].z, w[i].w});
  }
}
__device__ __forceinline__ void pack8(const double v[8], uint4* w) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint2 a = __builtin_bit_cast(uint2, v[2 * i]), b = __builtin_bit_cast(uint2, v[2 * i + 1]);
    w[i] = uint4{a.x, a.y, b.x, b.y};
  }
}

// ------------------------------------------------------------------ wave reductions
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Add a per-lane count to a stream counter: one atomic per wave, and none
// when the whole wave counted nothing (the usual case).
__device__ __forceinline__ void wave_count(unsigned long long* ctr, uint32_t v) {
  if (__ballot(v != 0u) == 0ull) return;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) atomicAdd(ctr, (unsigned long long)v);
}
// A finite value whose E4M3 rounding is clipped: above 464, the midpoint
// between 448 and the next step (480) that the format lacks.
__device__ __forceinline__ uint32_t e4m3_clips(float c) {
  const float a = __builtin_fabsf(c);
  return (a > 464.0f && a < __builtin_huge_valf()) ? 1u : 0u;
}
template <typename T> __device__ __forceinline__ bool finite_val(T v) { return __builtin_isfinite(v); }
template <> __device__ __forceinline__ bool finite_val<uint16_t>(uint16_t) { return true; }

// ------------------------------------------------------------------ batch descriptors
// One batch = a run of consecutive blocks of one stream pushed together
// (same B, S, input type and precisions).  Scratch arrays are strided per
// block.  The descriptors travel by value in the kernel arguments.
struct BatchDesc {
  const void* x;          // BIL input of the whole batch [lines][B][S]
  int B, Bp, S;           // bands, padded bands (multiple of 16), samples
  int nblk;               // blocks in the batch
  int blk_lines;          // lines of every block but the last
  int last_lines;         // lines of the last block
  int cpl;                // chunks (of KC samples) per line
  int ks, ks_last;        // covariance split count per block / for the last block
  int nsr, nsup;          // super-rows ceil(Bp/64); lower super-tiles nsr(nsr+1)/2
  int vec_ok;             // 16-byte vector loads of input rows are aligned
  int vec8_ok;            // 16-bit input: 8-byte loads of rows are aligned (S % 4 == 0)
  int nrect;              // covariance rectangles (16-tile units) owned by the waves of one workgroup
  uint8_t rect[16][4];    // per wave: first tile row, first tile column, tile rows, tile columns
  int ddof;
  double rho;             // ridge: lambda = rho * tr(Sigma) / B
  uint64_t reset_bits;    // bit b: block b starts a new statistics window
  int causal;             // block b is scored with the window before it (snapshot slot b - 1;
                          // slot nblk holds the window before the batch): 1 = slot nblk is
                          // formed by the merge and factored here, 2 = it is copied from the
                          // previous batch's last slot (the src_* pointers) by k_copy_slot
  int onepass;            // causal mode, every block scored with slot nblk (the window before the push)
  int lag_empty;          // one-pass: a window started earlier in the push (every block scores NaN)
  int fslot0;             // first factored snapshot slot (one-pass: only the last, and slot nblk
                          // when it is formed here, score anything)
  uint8_t wrow[16][2];     // one-pass kernel: out-band tiles each wave whitens (0xff: none)
  const double* src_mu; const void* src_wlp; const double* src_w64;
  const float* src_isc; const float* src_osc; const int* src_status;
  int64_t wl_bytes;       // whitening operand bytes per slot (0 on the FP64 path)
  // non-finite input (float input only; null for 16-bit input): a pixel with
  // a NaN or infinite band is left out of the statistics and scores NaN
  uint8_t* valid;         // [lines of the batch][S] 1 = every band finite
  int* nbadl;             // [lines of the batch] pixels with a non-finite band
  // statistics scratch
  double* shift;          // [nblk][Bp] per-block centring shift (FP32-representable on mixed paths)
  float* sscale;          // [nblk][Bp] FP8 covariance operand: band scale 2^-e (0 past the band count)
  void* part;             // [nblk][ks][Bp*Bp] centred scatter partials, lower part (float, or double on FP64)
  double* psum;           // [nblk][ks][Bp] raw per-band sums of each split (written by diagonal super-tiles)
  double* mu_snap;        // [nblk][Bp] window mean after block b
  double* m2_snap;        // [nblk][Bp*Bp] window scatter matrix after block b (lower triangle)
  double* n_snap;         // [nblk] window pixel count after block b
  double* ev;             // [nblk][Bp] block mean minus shift
  double* dv;             // [nblk][Bp] block mean minus the window mean before the block
  double* coef;           // [nblk] pairwise-update weight N n_b / (N + n_b), 0 for an empty window,
                          // -1 for a block with no finite pixel (the window is unchanged)
  double* nbv;            // [nblk] pixels of block b that enter the statistics
  // resident window state (ping-pong between batches)
  const double* s1_in; double* s1_out;   // [Bp + 1] raw band sums of the window, then its pixel count N
  const double* m2_in; double* m2_out;   // [Bp*Bp] scatter matrix of the window (lower)
  // factorisation
  double* w64;            // [nblk][Bp*Bp] W = L^{-1} S (row-major lower, FP64)
  void* wlp;              // [nblk][Bp*Bp] whitening operand in whiten precision, scaled
  double* lfac;           // [nblk][lf_stride] factor hand-off between the factor kernels: the
                          // diagonal inverses Y_k and the off-diagonal L_ik tiles in matrix-core
                          // operand order, then the equilibration scale [Bp]
  int64_t lf_stride;      // doubles per block of lfac
  float* iscale;          // [nblk][Bp] input scale 2^-e_k applied to centred values
  float* oscale;          // [nblk][Bp] output row scale 2^f_i
  int* status;            // [nblk] 0 ok, 1 singular, 2 not ready
  int* clipflag;          // [nblk] FP8 whitening of 16-bit input: 1 if a value of block b was clipped
  unsigned int* nsing;    // stream counters: [0] singular blocks, [1] blocks scored while not ready
  unsigned long long* cnt64;   // stream counters: [0] pixels with a non-finite band,
                               // [1] FP8 whitening operand values that saturated,
                               // [2] FP8 covariance operand values that saturated
  void* scores;           // scores of the batch's pixels (float, or double on FP64 whitening)
};

struct LaunchSet {
  int nb;                 // batches in this launch
  int wg0[MAXB + 1];      // prefix of workgroup counts per batch
  BatchDesc d[MAXB];
};

__device__ __forceinline__ int find_batch(const LaunchSet& ls, int wg, int& local) {
  int b = 0;
  while (b + 1 < ls.nb && wg >= ls.wg0[b + 1]) ++b;
  local = wg - ls.wg0[b];
  return b;
}

__device__ __forceinline__ int blk_lines_of(const BatchDesc& d, int b) {
  return b == d.nblk - 1 ? d.last_lines : d.blk_lines;
}
// Whitening operand in matrix-core fragment order: fragments before out-band
// tile i, the sum over m = 1..i of ceil(m / 2) (tile i spans the 32-band
// in-band steps 0..i/2 of the lower triangle).
__host__ __device__ constexpr int fr_off(int i) {
  return (i / 2) * (i / 2 + 1) + ((i & 1) ? (i / 2 + 1) : 0);
}

// Workgroup barrier that orders LDS accesses only.  A plain __syncthreads()
// also waits for every outstanding global access of the wave, which would
// drain the direct-to-LDS loads queued for later chunks; those are waited for
// explicitly, chunk by chunk, before the barrier that publishes them.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Snapshot slot whose statistics score block b: the window after block b
// (update, then score), in causal mode the window before it, in one-pass
// mode the window before the push (slot nblk for every block).
__device__ __forceinline__ int snap_slot(const BatchDesc& d, int b) {
  return d.causal ? ((b == 0 || d.onepass) ? d.nblk : b - 1) : b;
}
// Causal mode: a block that starts a new window has no statistics before it;
// one-pass mode: neither has a block after such a start within the push.
__device__ __forceinline__ bool causal_empty(const BatchDesc& d, int b) {
  if (!d.causal) return false;
  if (d.onepass) return d.lag_empty || (d.reset_bits & (b >= 63 ? ~0ull : ((2ull << b) - 1ull))) != 0;
  return (d.reset_bits >> b) & 1ull;
}
// Blocks of the batch that snapshot slot s scores, split into those with
// statistics (counted as singular / not ready by the slot's status) and
// those without (not ready whatever the slot holds).
__device__ __forceinline__ void slot_scores(const BatchDesc& d, int s, int& nwith, int& nwithout) {
  nwith = nwithout = 0;
  if (!d.causal) { nwith = 1; return; }
  if (d.onepass) {
    if (s != d.nblk) return;
    for (int b = 0; b < d.nblk; ++b) (causal_empty(d, b) ? nwithout : nwith) += 1;
    return;
  }
  const int b = s == d.nblk ? 0 : (s + 1 < d.nblk ? s + 1 : -1);
  if (b >= 0) (causal_empty(d, b) ? nwithout : nwith) = 1;
}
__device__ __forceinline__ int ks_of(const BatchDesc& d, int b) {
  return b == d.nblk - 1 ? d.ks_last : d.ks;
}
// Super-tile index -> (I, J), I >= J, row-major over the lower triangle.
__device__ __forceinline__ void sup_ij(int sup, int& I, int& J) {
  I = 0;
  while ((I + 1) * (I + 2) / 2 <= sup) ++I;
  J = sup - I * (I + 1) / 2;
}

}  // namespace rxk
