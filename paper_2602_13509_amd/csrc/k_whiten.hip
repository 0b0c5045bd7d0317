// Whitening and score: delta_p = |W (x_p - mu)|^2 = (x_p - mu)^T (Sigma + lambda I)^{-1} (x_p - mu)
// (Eq. 1 of the paper, Section "System Implementation / Detection
// Algorithm"), and the threshold masks of the same section.
//
// k_whiten: one workgroup per pixel chunk (KC samples of one line).  Wave w
// owns pixels 16w..16w+15 of the chunk; the whitened vector y never leaves
// registers: out-band tiles i (16 rows of W) accumulate over in-band steps
// k <= i only (W is lower triangular), then delta sums the squares across
// the tile rows and the four lane groups.
//  * 8-value operand formats (BF16, FP16, FP8): the chunk is centred in FP32
//    (mean split into hi + lo FP32 parts), scaled by the band's power of two,
//    rounded once, and staged in LDS transposed as [pixel][band] so each lane
//    reads 8 consecutive bands of one pixel.
//  * 1-value formats (FP32, FP64): operands come straight from the BIL rows
//    (16 consecutive samples of one band per lane group, coalesced).
#include "rx_dev.h"

#include <algorithm>
#include <climits>

namespace rxk {

constexpr int MAXBW = 16 * MAXT;    // 320: padded band pitch of the whitening operand

template <int IN, int P>
__global__ void __launch_bounds__(NT) k_whiten(LaunchSet ls, int Bw) {
  using M = MM<P>;
  using S = typename M::storage;
  using T = typename InT<IN>::T;
  int g;
  const int bi = find_batch(ls, blockIdx.x, g);
  const BatchDesc& d = ls.d[bi];
  const int B = d.B, Bp = d.Bp, nT = Bp / 16;
  const int lineb = g / d.cpl;                        // line within the batch
  const int bd = min(lineb / d.blk_lines, d.nblk - 1);  // block of the line
  const int b = snap_slot(d, bd);                      // snapshot slot that scores it
  const int s0 = (g % d.cpl) * KC;
  const int nvalid = min(KC, d.S - s0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int n = lane & 15, kg = lane >> 4;
  const T* xl = static_cast<const T*>(d.x) + (int64_t)lineb * B * d.S + s0;
  const double* mu = d.mu_snap + (int64_t)b * Bp;
  constexpr bool F64OUT = (P == P_F64);
  const int64_t out0 = (int64_t)lineb * d.S + s0;

  if (d.status[b] != 0 || causal_empty(d, bd)) {      // singular / not ready: NaN scores
    if (tid < nvalid) {
      if (F64OUT) static_cast<double*>(d.scores)[out0 + tid] = __builtin_nan("");
      else static_cast<float*>(d.scores)[out0 + tid] = __builtin_nanf("");
    }
    return;
  }
  typename M::acc acc[MAXT];
#pragma unroll
  for (int i = 0; i < MAXT; ++i) acc[i] = typename M::acc{};

  if constexpr (M::KV == 8) {
    constexpr int PAD = 16 / (int)sizeof(S);
    constexpr int LDB = MAXBW + PAD;
    __shared__ S dt[KC * LDB];
    const float* isc = d.iscale + (int64_t)b * Bp;
    const uint8_t* vl = (IN == IN_U16) ? nullptr : d.valid + (int64_t)lineb * d.S + s0;
    uint32_t nclip = 0;                               // FP8: operand values clipped at 448
    for (int it = tid; it < Bw * 8; it += NT) {
      const int k = it >> 3, k0 = 8 * (it & 7);
      float dv[8];
      if (k < B) {
        const T* row = xl + (int64_t)k * d.S;
        const double mud = mu[k];
        const float mhi = (float)mud, mlo = (float)(mud - (double)mhi), sc = isc[k];
        T v[8];
        if (d.vec_ok && k0 + 8 <= nvalid) {
          load8(row + k0, v);
        } else if (IN == IN_U16 && d.vec8_ok && k0 + 8 <= nvalid) {
          load8_a8(row + k0, v);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = (k0 + j < nvalid) ? row[k0 + j] : T(0);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float c;
          if constexpr (IN == IN_F64) c = (float)(v[j] - mud);
          else c = ((float)v[j] - mhi) - mlo;
          dv[j] = (k0 + j < nvalid) ? c * sc : 0.0f;
        }
        if constexpr (P == P_FP8) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (k0 + j < nvalid && (IN == IN_U16 || vl[k0 + j] != 0)) nclip += e4m3_clips(dv[j]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) dv[j] = 0.0f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) dt[(k0 + j) * LDB + k] = to_storage<P>(dv[j]);
    }
    __syncthreads();
    if constexpr (P == P_FP8) wave_count(d.cnt64 + 1, nclip);
    if (16 * w >= nvalid) return;
    const S* wl = static_cast<const S*>(d.wlp) + (int64_t)b * Bp * Bw;
    const int nsteps = Bw / 32;
    for (int s = 0; s < nsteps; ++s) {
      const typename M::frag bf = load_frag<P>(&dt[(16 * w + n) * LDB + 32 * s + 8 * kg]);
#pragma unroll
      for (int i = 0; i < MAXT; ++i) {
        if (i < nT && i >= 2 * s) {
          const typename M::frag af = load_frag<P>(&wl[(int64_t)(16 * i + n) * Bw + 32 * s + 8 * kg]);
          acc[i] = M::mma(af, bf, acc[i]);
        }
      }
    }
  } else {
    if (16 * w >= nvalid) return;
    using V = typename M::storage;           // float or double operand
    const V* wm = (P == P_F64) ? reinterpret_cast<const V*>(d.w64 + (int64_t)b * Bp * Bp)
                               : static_cast<const V*>(d.wlp) + (int64_t)b * Bp * Bw;
    const int pitch = (P == P_F64) ? Bp : Bw;
    const bool pv = (16 * w + n) < nvalid;
    const int nsteps = Bp / 4;
    for (int s = 0; s < nsteps; ++s) {
      const int k = 4 * s + kg;
      V bv = V(0);
      if (k < B && pv) {
        const T xv = xl[(int64_t)k * d.S + 16 * w + n];
        if constexpr (P == P_F64) {
          bv = to_d(xv) - mu[k];
        } else {
          const double mud = mu[k];
          if constexpr (IN == IN_F64) bv = (float)(xv - mud);
          else {
            const float mhi = (float)mud, mlo = (float)(mud - (double)mhi);
            bv = ((float)xv - mhi) - mlo;
          }
        }
      }
#pragma unroll
      for (int i = 0; i < MAXT; ++i) {
        if (i < nT && i >= (s >> 2)) {
          const V av = wm[(int64_t)(16 * i + n) * pitch + 4 * s + kg];
          acc[i] = M::mma(av, bv, acc[i]);
        }
      }
    }
  }

  // ---- delta = sum of squares of the whitened vector (FP32 accumulate; FP64 on the FP64 path)
  using A = typename M::accs;
  A dl = A(0);
  const float* osc = d.oscale + (int64_t)b * Bp;
#pragma unroll
  for (int i = 0; i < MAXT; ++i) {
    if (i < nT) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        A y = acc[i][j];
        if constexpr (M::KV == 8) y *= osc[16 * i + M::out_row(kg, j)];
        if constexpr (sizeof(A) == 4) dl = __builtin_fmaf(y, y, dl);
        else dl = __builtin_fma(y, y, dl);
      }
    }
  }
  dl += __shfl_xor(dl, 16, 64);
  dl += __shfl_xor(dl, 32, 64);
  if (kg == 0 && 16 * w + n < nvalid) {
    if constexpr (IN != IN_U16) {                      // a pixel with a non-finite band scores NaN
      if (d.valid[(int64_t)lineb * d.S + s0 + 16 * w + n] == 0) dl = A(__builtin_nan(""));
    }
    if constexpr (F64OUT) static_cast<double*>(d.scores)[out0 + 16 * w + n] = dl;
    else static_cast<float*>(d.scores)[out0 + 16 * w + n] = dl;
  }
}

// ---------------------------------------------------------------------------- whitening, 16-bit input
// k_whiten2: the same score for 16-bit integer input and the 8-value operand
// formats, organised for operand reuse.
//  * One workgroup per CU walks an even share of the launch's tiles of 16 G
//    pixels (consecutive samples of one line).  The whitening operand of the
//    current block sits in LDS in matrix-core operand order (lane-major
//    fragments of 16 bytes, or 8 for FP8), staged once per block the
//    workgroup touches, together with the split mean, band and row scales.
//  * A wave owns a whole tile: lane (n, kg) loads samples G n .. G n + G - 1
//    of bands 32 s + 8 kg + j in one load, so sample G n + g is column n of
//    the g-th 16-pixel product; all G products reuse every operand fragment
//    read from LDS (and every band constant).  The centred, scaled and
//    rounded tile stays in registers; the waves of a SIMD overlap one
//    another's loads and products.  No workgroup barrier inside a block.
//  * Arithmetic is that of k_whiten: centring in FP32 with the mean split
//    hi + lo, the band's power-of-two scale, one rounding to the operand
//    format, FP32 accumulation, the row scale on the output, squares summed
//    over tile rows then over the four lane groups.
constexpr int W2NT = 512;                     // 8 waves
constexpr int W2W = W2NT / 64;
constexpr int W2_FREE_CUS = 32;                // CUs the tile kernel leaves to other queues
constexpr int W2G = 4;                        // 16-pixel products per tile
constexpr int W2TP = 16 * W2G;                // pixels per tile
constexpr int MAXS = (MAXT + 1) / 2;          // 32-band operand steps
constexpr int MAXFR = fr_off(MAXT);

template <int P> __device__ __forceinline__ typename MM<P>::frag pack_frag(const typename MM<P>::storage e[8]);
template <> __device__ __forceinline__ bf16x8 pack_frag<P_BF16>(const uint16_t e[8]) {
  uint4 w;
  pack8(e, &w);
  return __builtin_bit_cast(bf16x8, w);
}
template <> __device__ __forceinline__ f16x8 pack_frag<P_F16>(const uint16_t e[8]) {
  uint4 w;
  pack8(e, &w);
  return __builtin_bit_cast(f16x8, w);
}
template <> __device__ __forceinline__ long pack_frag<P_FP8>(const uint8_t e[8]) {
  const uint2 w{(uint32_t)e[0] | ((uint32_t)e[1] << 8) | ((uint32_t)e[2] << 16) | ((uint32_t)e[3] << 24),
                (uint32_t)e[4] | ((uint32_t)e[5] << 8) | ((uint32_t)e[6] << 16) | ((uint32_t)e[7] << 24)};
  return __builtin_bit_cast(long, w);
}

// Eight centred values -> one operand fragment.
template <int P> __device__ __forceinline__ typename MM<P>::frag cvt_frag(const float c[8]) {
  if constexpr (P == P_FP8) {
    uint8_t e[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) e[j] = f32_to_e4m3(c[j]);
    return pack_frag<P_FP8>(e);
  } else {
    const uint4 w{cvt_pack2<P>(c[0], c[1]), cvt_pack2<P>(c[2], c[3]), cvt_pack2<P>(c[4], c[5]),
                  cvt_pack2<P>(c[6], c[7])};
    return __builtin_bit_cast(typename MM<P>::frag, w);
  }
}

// G consecutive 16-bit samples of one band row, as loaded.
template <int G> struct Raw;
template <> struct Raw<2> {
  uint32_t w;
  __device__ __forceinline__ void load(const char* p) { w = *reinterpret_cast<const uint32_t*>(p); }
  __device__ __forceinline__ uint32_t at(int g) const { return g ? (w >> 16) : (w & 0xffffu); }
};
template <> struct Raw<4> {
  uint2 w;
  __device__ __forceinline__ void load(const char* p) { w = *reinterpret_cast<const uint2*>(p); }
  __device__ __forceinline__ uint32_t at(int g) const {
    const uint32_t v = g < 2 ? w.x : w.y;
    return (g & 1) ? (v >> 16) : (v & 0xffffu);
  }
};
template <int G> __device__ __forceinline__ void store_scores(float* p, const float* v);
template <> __device__ __forceinline__ void store_scores<2>(float* p, const float* v) {
  *reinterpret_cast<float2*>(p) = float2{v[0], v[1]};
}
template <> __device__ __forceinline__ void store_scores<4>(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = float4{v[0], v[1], v[2], v[3]};
}

// Pixel groups per tile: four where the operand tile fits the register
// budget without spilling (16-bit operands up to 288 bands, FP8 up to 160),
// two otherwise.
__host__ __device__ constexpr int w2_groups(int p, int ns) {
  return (p == P_FP8) ? (ns <= 5 ? 4 : 2) : (ns <= 9 ? 4 : 2);
}

// ls.wg0 holds the prefix of tiles per batch (not workgroups).  NS is the
// number of 32-band steps, ceil(nT / 2), the same for every batch of the
// launch.  Requires S % 4 == 0 and 8-byte aligned rows (vec8_ok); the last
// tile of a line may reach past its end (those samples are read from the
// line's start and their scores are not stored).
template <int P, int NS, int G>
__global__ void __launch_bounds__(W2NT) k_whiten2(LaunchSet ls, int Bw, int64_t ntile_all) {
  using M = MM<P>;
  using S = typename M::storage;
  using F = typename M::frag;
  constexpr int TP = 16 * G;                   // pixels per tile
  constexpr int FB = 8 * (int)sizeof(S);       // operand bytes per lane
  __shared__ __attribute__((aligned(16))) uint8_t wf[MAXFR * 64 * FB];
  __shared__ __attribute__((aligned(16))) float nqh[16 * MAXT];   // -(mean hi) * band scale
  __shared__ __attribute__((aligned(16))) float nql[16 * MAXT];   // -(mean lo) * band scale
  __shared__ __attribute__((aligned(16))) float iss[16 * MAXT];   // band scale 2^-e
  __shared__ __attribute__((aligned(16))) float oss[16 * MAXT];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = lane & 15, kg = lane >> 4;
  const int64_t T0 = ntile_all * blockIdx.x / gridDim.x, T1 = ntile_all * (blockIdx.x + 1) / gridDim.x;

  for (int64_t cur = T0; cur < T1;) {
    // locate (batch, block) of tile cur and the end of this block's share
    int bi = 0;
    while (bi + 1 < ls.nb && cur >= ls.wg0[bi + 1]) ++bi;
    const BatchDesc& d = ls.d[bi];
    const int B = d.B, Bp = d.Bp, nT = Bp / 16, Sm = d.S;
    const int tpl = (Sm + TP - 1) / TP;
    const int64_t tl = cur - ls.wg0[bi];                       // tile within the batch
    const int64_t tpb = (int64_t)d.blk_lines * tpl;            // tiles per (full) block
    const int b = (int)min(tl / tpb, (int64_t)d.nblk - 1);
    const int64_t blk_end = ls.wg0[bi] + (int64_t)b * tpb + (int64_t)blk_lines_of(d, b) * tpl;
    const int sb = snap_slot(d, b);                              // snapshot slot that scores block b
    const int64_t seg_end = min(T1, blk_end);
    const int64_t tb0 = cur - ls.wg0[bi];                      // segment, batch-relative tiles
    const int nseg = (int)(seg_end - cur);
    cur = seg_end;
    float* out = static_cast<float*>(d.scores);

    if (d.status[sb] != 0 || causal_empty(d, b)) {              // singular / not ready: NaN scores
      for (int q = tid; q < nseg * TP; q += W2NT) {
        const int64_t t = tb0 + q / TP;
        const int smp = TP * (int)(t % tpl) + q % TP;
        if (smp < Sm) out[(t / tpl) * Sm + smp] = __builtin_nanf("");
      }
      continue;
    }

    __syncthreads();                                            // previous segment's readers are done
    {
      const S* wl = static_cast<const S*>(d.wlp) + (int64_t)sb * Bp * Bw;
      const int nfr = fr_off(nT);
      for (int it = tid; it < nfr * 64; it += W2NT) {
        const int f = it >> 6, l = it & 63;
        int i = 0;
        while (fr_off(i + 1) <= f) ++i;
        const int st = f - fr_off(i);
        const S* src = wl + (int64_t)(16 * i + (l & 15)) * Bw + 32 * st + 8 * (l >> 4);
        if constexpr (P == P_BF16) {
          // BF16 keeps FP32's exponent range, so the row's power-of-two output
          // scale folds into the staged operand exactly; the products then
          // come out already scaled (bit for bit what scaling them would give)
          const float o = d.oscale[(int64_t)sb * Bp + 16 * i + (l & 15)];
          uint4 w = *reinterpret_cast<const uint4*>(src);
          uint32_t* q = reinterpret_cast<uint32_t*>(&w);
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const float lo = __builtin_bit_cast(float, q[h] << 16) * o;
            const float hi = __builtin_bit_cast(float, q[h] & 0xffff0000u) * o;
            q[h] = (__builtin_bit_cast(uint32_t, lo) >> 16) | (__builtin_bit_cast(uint32_t, hi) & 0xffff0000u);
          }
          *reinterpret_cast<uint4*>(wf + it * 16) = w;
        } else if constexpr (FB == 16) {
          *reinterpret_cast<uint4*>(wf + it * 16) = *reinterpret_cast<const uint4*>(src);
        } else {
          *reinterpret_cast<uint2*>(wf + it * 8) = *reinterpret_cast<const uint2*>(src);
        }
      }
      const double* mu = d.mu_snap + (int64_t)sb * Bp;
      const float* isc = d.iscale + (int64_t)sb * Bp;
      const float* osc = d.oscale + (int64_t)sb * Bp;
      for (int k = tid; k < 16 * MAXT; k += W2NT) {
        float mh = 0.0f, ml = 0.0f, is = 0.0f;
        if (k < B) {
          const double m = mu[k];
          mh = (float)m;
          ml = (float)(m - (double)mh);
          is = isc[k];
        }
        // the band scale is a power of two, so these products are exact and
        // fma(v, s, -mh s) - ml s equals ((v - mh) - ml) s bit for bit
        nqh[k] = -(mh * is);
        nql[k] = -(ml * is);
        iss[k] = is;                                            // zero past the band count
        oss[k] = k < Bp ? osc[k] : 0.0f;
      }
    }
    __syncthreads();

    const uint16_t* xb = static_cast<const uint16_t*>(d.x);
    Raw<G> raw[NS][8];
    // Only the last 32-band step can reach past the band count (the earlier
    // steps end at or below 16 (nT - 1) < B); its rows are clamped to B - 1
    // and zeroed by the band scale.
    auto load_raw = [&](int64_t t) {
      const int64_t line = t / tpl;
      const int smp = TP * (int)(t % tpl) + G * n;
      // wave-uniform line base + 32-bit byte offsets (a line of B <= 320 rows
      // is far below 4 GiB): global loads with a scalar base
      const char* xl = reinterpret_cast<const char*>(xb + line * B * Sm);
      const uint32_t o = 2u * (uint32_t)(smp < Sm ? smp : 0);
      const uint32_t lo = o + 2u * (uint32_t)(8 * kg) * (uint32_t)Sm;
      const uint32_t rs = 2u * (uint32_t)Sm;
      uint32_t ro = 0;
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        if (st + 1 < NS) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            raw[st][j].load(xl + (lo + ro));
            ro += rs;
            asm volatile("" : "+s"(ro));
          }
          ro += 24u * rs;
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const uint32_t k = (uint32_t)min(32 * st + 8 * kg + j, B - 1);
            raw[st][j].load(xl + (o + k * rs));
          }
        }
      }
    };

    int64_t t = tb0 + wv;
    const int64_t tend = tb0 + nseg;
    bool clipped = false;                                       // FP8: a value beyond the format's range
    for (; t < tend; t += W2W) {
      load_raw(t);
      const int smp = TP * (int)(t % tpl) + G * n;
      const bool ok = smp < Sm;
      F xf[G][NS];
      uint32_t top = 0;                                         // FP8: bit 8q+7 set if a byte coded +-448
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        // re-read per tile: hoisting these tile-invariant values would hold
        // 24 registers per step for the whole loop
        int k0 = 32 * st + 8 * kg;
        asm volatile("" : "+v"(k0));
        const float4 qh0 = *reinterpret_cast<const float4*>(&nqh[k0]);
        const float4 qh1 = *reinterpret_cast<const float4*>(&nqh[k0 + 4]);
        const float4 ql0 = *reinterpret_cast<const float4*>(&nql[k0]);
        const float4 ql1 = *reinterpret_cast<const float4*>(&nql[k0 + 4]);
        const float4 is0 = *reinterpret_cast<const float4*>(&iss[k0]);
        const float4 is1 = *reinterpret_cast<const float4*>(&iss[k0 + 4]);
        const float qh[8] = {qh0.x, qh0.y, qh0.z, qh0.w, qh1.x, qh1.y, qh1.z, qh1.w};
        const float ql[8] = {ql0.x, ql0.y, ql0.z, ql0.w, ql1.x, ql1.y, ql1.z, ql1.w};
        const float is[8] = {is0.x, is0.y, is0.z, is0.w, is1.x, is1.y, is1.z, is1.w};
        // samples past the row end are converted too (their loads read
        // sample 0 of the line); a column never mixes into another column
        // of the product and their scores are not stored
#pragma unroll
        for (int g = 0; g < G; ++g) {
          float c[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) c[j] = __builtin_fmaf((float)raw[st][j].at(g), is[j], qh[j]) + ql[j];
          xf[g][st] = cvt_frag<P>(c);
          if constexpr (P == P_FP8) {
            // a byte coding +-448, the largest finite value, is where
            // clipped values land (so do values in (432, 464], which round to it)
            const uint2 w = __builtin_bit_cast(uint2, xf[g][st]);
            const uint32_t x0 = (w.x & 0x7F7F7F7Fu) ^ 0x7E7E7E7Eu, x1 = (w.y & 0x7F7F7F7Fu) ^ 0x7E7E7E7Eu;
            top |= ((x0 - 0x01010101u) & ~x0) | ((x1 - 0x01010101u) & ~x1);
          }
        }
      }

      float dl[G];
#pragma unroll
      for (int g = 0; g < G; ++g) dl[g] = 0.0f;
#pragma unroll
      for (int i = 0; i < 2 * NS; ++i) {
        if (i < 2 * NS - 1 || i < nT) {
          typename M::acc a[G];
#pragma unroll
          for (int g = 0; g < G; ++g) a[g] = typename M::acc{};
#pragma unroll
          for (int st = 0; st <= i / 2; ++st) {
            const F af = *reinterpret_cast<const F*>(wf + ((fr_off(i) + st) * 64 + lane) * FB);
#pragma unroll
            for (int g = 0; g < G; ++g) a[g] = M::mma(af, xf[g][st], a[g]);
          }
          if constexpr (P == P_BF16) {                          // row scale already in the operand
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int g = 0; g < G; ++g) dl[g] = __builtin_fmaf(a[g][j], a[g][j], dl[g]);
          } else {
            const float4 os = *reinterpret_cast<const float4*>(&oss[16 * i + 4 * kg]);
            const float o4[4] = {os.x, os.y, os.z, os.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int g = 0; g < G; ++g) {
                const float y = a[g][j] * o4[j];
                dl[g] = __builtin_fmaf(y, y, dl[g]);
              }
          }
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        dl[g] += __shfl_xor(dl[g], 16, 64);
        dl[g] += __shfl_xor(dl[g], 32, 64);
      }
      if (kg == 0 && ok) store_scores<G>(&out[(t / tpl) * Sm + smp], dl);
      if constexpr (P == P_FP8) clipped |= (ok && (top & 0x80808080u) != 0);
    }
    // rare: a value of this segment was clipped; k_fp8_clips counts the
    // block's clipped values exactly afterwards
    if constexpr (P == P_FP8)
      if (__ballot(clipped) != 0ull && lane == 0) d.clipflag[sb] = 1;
  }
}

// Exact count of the FP8 operand values that k_whiten2 clipped, for the
// blocks it flagged (none in the usual case: every workgroup then exits at
// once).  One workgroup per line; the centred, band-scaled value is formed
// exactly as k_whiten2 forms it.
__global__ void __launch_bounds__(NT) k_fp8_clips(LaunchSet ls) {
  int line;
  const int bi = find_batch(ls, blockIdx.x, line);
  const BatchDesc& d = ls.d[bi];
  const int bd = min(line / d.blk_lines, d.nblk - 1);
  const int b = snap_slot(d, bd);
  if (d.status[b] != 0 || causal_empty(d, bd) || d.clipflag[b] == 0) return;
  const int B = d.B, Bp = d.Bp, Sm = d.S;
  const uint16_t* xl = static_cast<const uint16_t*>(d.x) + (int64_t)line * B * Sm;
  const double* mu = d.mu_snap + (int64_t)b * Bp;
  const float* isc = d.iscale + (int64_t)b * Bp;
  uint32_t nclip = 0;
  for (int k = 0; k < B; ++k) {
    const double m = mu[k];
    const float mh = (float)m, ml = (float)(m - (double)mh), is = isc[k];
    const float qh = -(mh * is), ql = -(ml * is);
    for (int s = threadIdx.x; s < Sm; s += NT)
      nclip += e4m3_clips(__builtin_fmaf((float)xl[(int64_t)k * Sm + s], is, qh) + ql);
  }
  wave_count(d.cnt64 + 1, nclip);
}

// ---------------------------------------------------------------------------- masks
__device__ __forceinline__ uint64_t okey(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_okey(uint64_t k) {
  const uint64_t u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __builtin_bit_cast(double, u);
}
__device__ __forceinline__ double score_at(const void* sc, int f64, int64_t i) {
  return f64 ? static_cast<const double*>(sc)[i] : (double)static_cast<const float*>(sc)[i];
}

struct TopkState {
  uint64_t prefix, mask;
  int64_t remaining, ties;
  int all;
};

// Maximum score key: per-wave, then per-workgroup reduction, one atomic per
// workgroup (the launch keeps the workgroup count small).
constexpr int MAXKEY_WG = 512;
__global__ void __launch_bounds__(NT) k_maxkey(const void* sc, int f64, int64_t n, uint64_t* out) {
  __shared__ uint64_t wm[NT / 64];
  uint64_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const double v = score_at(sc, f64, i);
    if (v == v) m = max(m, okey(v));
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint64_t)__shfl_xor((unsigned long long)m, o, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) m = max(m, wm[w]);
    if (m) atomicMax((unsigned long long*)out, (unsigned long long)m);
  }
}

__global__ void __launch_bounds__(NT) k_mask_thr(const void* sc, int f64, int64_t n, double thr,
                                                 const uint64_t* maxkey, double tau, uint32_t* bits) {
  const int64_t wq = (int64_t)blockIdx.x * NT + threadIdx.x;    // one 32-pixel word per thread
  if (wq * 32 >= n) return;
  const double t = maxkey ? tau * from_okey(*maxkey) : thr;
  uint32_t word = 0;
  for (int j = 0; j < 32; ++j) {
    const int64_t p = wq * 32 + j;
    if (p < n && score_at(sc, f64, p) > t) word |= 1u << j;
  }
  bits[wq] = word;
}

__global__ void k_clear_key(uint64_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

__global__ void k_topk_init(TopkState* st, int64_t k, uint32_t* hist) {
  if (threadIdx.x == 0) { st->prefix = 0; st->mask = 0; st->remaining = k; st->ties = 0; st->all = 0; }
  hist[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(NT) k_topk_hist(const void* sc, int f64, int64_t n, const TopkState* st,
                                                  int shift, uint32_t* hist) {
  __shared__ uint32_t lh[256];
  lh[threadIdx.x] = 0;
  __syncthreads();
  if (!st->all) {
    const uint64_t pre = st->prefix, msk = st->mask;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
      const double v = score_at(sc, f64, i);
      if (!(v == v)) continue;
      const uint64_t key = okey(v);
      if ((key & msk) == pre) atomicAdd(&lh[(key >> shift) & 255], 1u);
    }
  }
  __syncthreads();
  if (lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

__global__ void k_topk_select(TopkState* st, int shift, uint32_t* hist) {
  if (threadIdx.x == 0 && !st->all) {
    int64_t cum = 0;
    int found = 0;
    for (int bin = 255; bin >= 0; --bin) {
      const int64_t c = hist[bin];
      if (cum + c >= st->remaining) {
        st->prefix |= (uint64_t)bin << shift;
        st->mask |= (uint64_t)0xFF << shift;
        st->remaining -= cum;
        st->ties = c;
        found = 1;
        break;
      }
      cum += c;
    }
    if (!found) st->all = 1;           // fewer valid scores than k: every valid score is marked
  }
  __syncthreads();
  hist[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(NT) k_mask_topk(const void* sc, int f64, int64_t n, const TopkState* st,
                                                  uint32_t* bits) {
  const int64_t wq = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (wq * 32 >= n) return;
  const uint64_t kstar = st->prefix;
  const bool all = st->all, take_ties = st->ties == st->remaining;
  uint32_t word = 0;
  for (int j = 0; j < 32; ++j) {
    const int64_t p = wq * 32 + j;
    if (p >= n) break;
    const double v = score_at(sc, f64, p);
    if (!(v == v)) continue;
    const uint64_t key = okey(v);
    if (all || key > kstar || (take_ties && key == kstar)) word |= 1u << j;
  }
  bits[wq] = word;
}

// Ties at the k-th score beyond the quota: the lowest pixel indices win.
// One workgroup scans in pixel order with a block-wide prefix count.
__global__ void __launch_bounds__(NT) k_topk_ties(const void* sc, int f64, int64_t n, const TopkState* st,
                                                  uint32_t* bits) {
  if (st->all || st->ties == st->remaining) return;
  __shared__ int cnt[NT];
  const uint64_t kstar = st->prefix;
  int64_t taken = 0;
  const int64_t quota = st->remaining;
  for (int64_t base = 0; base < n && taken < quota; base += NT) {
    const int64_t p = base + threadIdx.x;
    const int f = (p < n) && [&] { const double v = score_at(sc, f64, p); return v == v && okey(v) == kstar; }();
    cnt[threadIdx.x] = f;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {
      const int add = threadIdx.x >= o ? cnt[threadIdx.x - o] : 0;
      __syncthreads();
      cnt[threadIdx.x] += add;
      __syncthreads();
    }
    const int excl = cnt[threadIdx.x] - f;
    if (f && taken + excl < quota) atomicOr(&bits[p >> 5], 1u << (p & 31));
    taken += cnt[NT - 1];
    __syncthreads();
  }
}

// Byte copy and word fill used by the allocation-free mask (kernels, so the
// sequence can be captured into a HIP graph: no memset or memcpy nodes).
__global__ void __launch_bounds__(NT) k_copy_bytes(const uint8_t* a, uint8_t* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) b[i] = a[i];
}
__global__ void __launch_bounds__(NT) k_zero_words(uint32_t* w, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) w[i] = 0u;
}

// Working memory of the allocation-free mask entry point, one copy per GPU
// (each device's code object holds its own), kept until the process ends:
// the maximum key, the top-k state and histogram in the first 4 KiB, then
// the mask words of up to 2^23 pixels.  Host code never passes this name to
// a kernel: it takes the device address from rxk_noalloc_scratch.
constexpr size_t kNoallocHead = 4096;
constexpr size_t kNoallocBytes = kNoallocHead + (size_t(1) << 20);
static __device__ __attribute__((aligned(256))) uint8_t scratch[kNoallocBytes];

}  // namespace rxk

// The current device's address of the allocation-free mask's working memory
// and its size (the header part first, then the mask words).
extern "C" hipError_t rxk_noalloc_scratch(void** ptr, size_t* head, size_t* bytes) {
  *head = rxk::kNoallocHead;
  *bytes = rxk::kNoallocBytes;
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(rxk::scratch));
}

extern "C" hipError_t rxk_launch_copy_bytes(const void* a, void* b, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + rxk::NT - 1) / rxk::NT;
  hipLaunchKernelGGL(rxk::k_copy_bytes, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(rxk::NT), 0, st,
                     static_cast<const uint8_t*>(a), static_cast<uint8_t*>(b), n);
  return hipGetLastError();
}

extern "C" hipError_t rxk_launch_zero_words(uint32_t* w, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + rxk::NT - 1) / rxk::NT;
  hipLaunchKernelGGL(rxk::k_zero_words, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(rxk::NT), 0, st, w, n);
  return hipGetLastError();
}

extern "C" hipError_t rxk_launch_whiten(int in_type, int wprec, const rxk::LaunchSet* ls, int wg, int Bw,
                                        hipStream_t st) {
  using namespace rxk;
  if (wg <= 0) return hipSuccess;
  if (in_type == IN_U16 && (wprec == P_BF16 || wprec == P_F16 || wprec == P_FP8) && Bw % 32 == 0 && Bw >= 32 &&
      Bw <= 32 * MAXS) {
    // batches of 16-bit rows with S % 4 == 0 and 8-byte aligned starts
    // (vec8_ok: a lane's G <= 4 samples are one aligned load) take the tile
    // kernel, the others the chunk kernel; the choice is per batch (both
    // give the same scores, bit for bit)
    const int ns = Bw / 32;                                  // the launch shares Bw = 32 ceil(nT / 2)
    const int G = w2_groups(wprec, ns);
    LaunchSet t, o;
    t.nb = o.nb = 0;
    t.wg0[0] = o.wg0[0] = 0;
    for (int i = 0; i < ls->nb; ++i) {
      const BatchDesc& d = ls->d[i];
      const int64_t tpl = (d.S + 16 * G - 1) / (16 * G);
      const int64_t tiles = ((int64_t)(d.nblk - 1) * d.blk_lines + d.last_lines) * tpl;
      if (d.vec8_ok && (int64_t)t.wg0[t.nb] + tiles <= INT32_MAX) {
        t.d[t.nb] = d;
        t.wg0[t.nb + 1] = t.wg0[t.nb] + (int)tiles;
        ++t.nb;
      } else {
        o.d[o.nb] = d;
        o.wg0[o.nb + 1] = o.wg0[o.nb] + (ls->wg0[i + 1] - ls->wg0[i]);
        ++o.nb;
      }
    }
    if (t.nb > 0) {
      static int cus[64] = {0};
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess) return hipGetLastError();
      if (dev < 64 && cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return hipGetLastError();
        cus[dev] = c;
      }
      const int ncu = (dev < 64 && cus[dev] > 0) ? cus[dev] : 256;
      const int64_t ntile = t.wg0[t.nb];
      // one persistent workgroup per CU fills a CU's registers and most of
      // its LDS; leaving W2_FREE_CUS CUs out lets the next batch's merge and
      // factorisation (queued on another HIP stream) run beside the whitening
      const int navail = ncu > 4 * W2_FREE_CUS ? ncu - W2_FREE_CUS : ncu;
      const int g = (int)std::max<int64_t>(1, std::min<int64_t>(navail, ntile / W2W));   // a tile per wave at least
      switch ((wprec * 16 + ns) * 8 + G) {
#define RXK_W2(PV, N, GG)                                                                              \
  case (PV * 16 + N) * 8 + GG:                                                                         \
    hipLaunchKernelGGL((k_whiten2<PV, N, GG>), dim3(g), dim3(W2NT), 0, st, t, Bw, ntile);              \
    break;
#define RXK_W2P(PV, GG) RXK_W2(PV, 1, GG) RXK_W2(PV, 2, GG) RXK_W2(PV, 3, GG) RXK_W2(PV, 4, GG) RXK_W2(PV, 5, GG) \
                        RXK_W2(PV, 6, GG) RXK_W2(PV, 7, GG) RXK_W2(PV, 8, GG) RXK_W2(PV, 9, GG)
        RXK_W2P(P_BF16, 4) RXK_W2P(P_F16, 4) RXK_W2(P_BF16, 10, 2) RXK_W2(P_F16, 10, 2)
        RXK_W2(P_FP8, 1, 4) RXK_W2(P_FP8, 2, 4) RXK_W2(P_FP8, 3, 4) RXK_W2(P_FP8, 4, 4) RXK_W2(P_FP8, 5, 4)
        RXK_W2(P_FP8, 6, 2) RXK_W2(P_FP8, 7, 2) RXK_W2(P_FP8, 8, 2) RXK_W2(P_FP8, 9, 2) RXK_W2(P_FP8, 10, 2)
#undef RXK_W2P
#undef RXK_W2
        default: return hipErrorInvalidValue;
      }
      if (wprec == P_FP8) {
        LaunchSet c = t;                                        // one workgroup per line
        for (int i = 0; i < c.nb; ++i)
          c.wg0[i + 1] = c.wg0[i] + (c.d[i].nblk - 1) * c.d[i].blk_lines + c.d[i].last_lines;
        hipLaunchKernelGGL(k_fp8_clips, dim3(c.wg0[c.nb]), dim3(NT), 0, st, c);
      }
    }
    if (o.nb == 0) return hipGetLastError();
    if (wprec == P_BF16) hipLaunchKernelGGL((k_whiten<IN_U16, P_BF16>), dim3(o.wg0[o.nb]), dim3(NT), 0, st, o, Bw);
    else if (wprec == P_F16) hipLaunchKernelGGL((k_whiten<IN_U16, P_F16>), dim3(o.wg0[o.nb]), dim3(NT), 0, st, o, Bw);
    else hipLaunchKernelGGL((k_whiten<IN_U16, P_FP8>), dim3(o.wg0[o.nb]), dim3(NT), 0, st, o, Bw);
    return hipGetLastError();
  }
#define RXK_W(INV, PV)                                                                          \
  if (in_type == INV && wprec == PV) {                                                          \
    hipLaunchKernelGGL((k_whiten<INV, PV>), dim3(wg), dim3(NT), 0, st, *ls, Bw);                \
    return hipGetLastError();                                                                   \
  }
  RXK_W(IN_U16, P_F64) RXK_W(IN_U16, P_F32) RXK_W(IN_U16, P_BF16) RXK_W(IN_U16, P_F16) RXK_W(IN_U16, P_FP8)
  RXK_W(IN_F32, P_F64) RXK_W(IN_F32, P_F32) RXK_W(IN_F32, P_BF16) RXK_W(IN_F32, P_F16) RXK_W(IN_F32, P_FP8)
  RXK_W(IN_F64, P_F64) RXK_W(IN_F64, P_F32) RXK_W(IN_F64, P_BF16) RXK_W(IN_F64, P_F16) RXK_W(IN_F64, P_FP8)
#undef RXK_W
  return hipErrorInvalidValue;
}

// mode 0: absolute threshold; 1: relative to the maximum; 2: top-k.
// bits: device words, (n + 31) / 32 of them.  scratch: >= 64 bytes + 1 KiB.
extern "C" hipError_t rxk_launch_mask(const void* sc, int f64, int64_t n, int mode, double tau, int64_t k,
                                      uint32_t* bits, void* scratch, hipStream_t st) {
  using namespace rxk;
  if (n <= 0) return hipSuccess;
  const int64_t words = (n + 31) / 32;
  const int gw = (int)((words + NT - 1) / NT);
  const int gs = (int)(((n + NT - 1) / NT) < 2048 ? ((n + NT - 1) / NT) : 2048);
  uint64_t* maxkey = static_cast<uint64_t*>(scratch);
  TopkState* tk = reinterpret_cast<TopkState*>(static_cast<char*>(scratch) + 64);
  uint32_t* hist = reinterpret_cast<uint32_t*>(static_cast<char*>(scratch) + 128);
  if (mode == 0) {
    hipLaunchKernelGGL(k_mask_thr, dim3(gw), dim3(NT), 0, st, sc, f64, n, tau, (const uint64_t*)nullptr, 0.0, bits);
  } else if (mode == 1) {
    hipLaunchKernelGGL(k_clear_key, dim3(1), dim3(64), 0, st, maxkey);
    hipLaunchKernelGGL(k_maxkey, dim3(gs < MAXKEY_WG ? gs : MAXKEY_WG), dim3(NT), 0, st, sc, f64, n, maxkey);
    hipLaunchKernelGGL(k_mask_thr, dim3(gw), dim3(NT), 0, st, sc, f64, n, 0.0, (const uint64_t*)maxkey, tau, bits);
  } else {
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, st, tk, k, hist);
    for (int shift = 56; shift >= 0; shift -= 8) {
      hipLaunchKernelGGL(k_topk_hist, dim3(gs), dim3(NT), 0, st, sc, f64, n, (const TopkState*)tk, shift, hist);
      hipLaunchKernelGGL(k_topk_select, dim3(1), dim3(256), 0, st, tk, shift, hist);
    }
    hipLaunchKernelGGL(k_mask_topk, dim3(gw), dim3(NT), 0, st, sc, f64, n, (const TopkState*)tk, bits);
    hipLaunchKernelGGL(k_topk_ties, dim3(1), dim3(NT), 0, st, sc, f64, n, (const TopkState*)tk, bits);
  }
  return hipGetLastError();
}
