// Streaming window statistics: band mean and scatter matrix of every pixel
// in the window (paper, Section "System Implementation / Detection
// Algorithm": mean per band, covariance over all pixels of the set).
//
// Per block of lines:
//   k_valid  -- float input only: marks the pixels whose bands are all finite
//               and counts the others per line; those pixels stay out of
//               every sum below (and score NaN)
//   k_shift  -- centring shift c = mean of the block's first line per band
//               (rounded to FP32 on mixed paths, so it is exact in both the
//               FP32 centring and the FP64 merge).
//   k_syrk   -- C = sum_p (x_p - c)(x_p - c)^T on matrix cores, lower 64x64
//               super-tiles x split-K over pixel chunks, FP32 (or FP64)
//               partials; diagonal super-tiles also emit exact raw band sums.
//   k_merge_vec / k_merge_red / k_merge_rec -- fixed-order FP64 reduction of the
//               partials, exact shift correction M2_b = C - n e e^T
//               (e = m_b - c), then the pairwise (Chan-Golub-LeVeque) update
//               of the window (N, S1, M2), snapshotting it after every block.
#include <atomic>
#include <type_traits>

#include "rx_dev.h"

namespace rxk {

// ---------------------------------------------------------------------------- validity (float input)
// One workgroup per line of the batch; a thread walks the band rows of its
// samples (coalesced across the wave), so the line is read once.
template <int IN>
__global__ void __launch_bounds__(NT) k_valid(LaunchSet ls) {
  int line;
  const int bi = find_batch(ls, blockIdx.x, line);
  const BatchDesc& d = ls.d[bi];
  using T = typename InT<IN>::T;
  const T* xl = static_cast<const T*>(d.x) + (int64_t)line * d.B * d.S;
  __shared__ uint32_t red[NT / 64];
  uint32_t bad = 0;
  for (int s = threadIdx.x; s < d.S; s += NT) {
    bool ok = true;
#pragma unroll 8
    for (int k = 0; k < d.B; ++k) ok &= finite_val(xl[(int64_t)k * d.S + s]);
    d.valid[(int64_t)line * d.S + s] = ok ? 1 : 0;
    bad += ok ? 0u : 1u;
  }
  bad = wave_sum(bad);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    d.nbadl[line] = (int)t;
    if (t) atomicAdd(d.cnt64, (unsigned long long)t);
  }
}

// ---------------------------------------------------------------------------- shift
// The shift is the mean of the block's first line (of its finite pixels for
// float input; 0 when there are none): any finite value is exact in the
// merge's correction, a close one keeps the centred products small.
template <int IN, int P>
__global__ void __launch_bounds__(NT) k_shift(LaunchSet ls) {
  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  using T = typename InT<IN>::T;
  const int nbg = d.Bp / 4;
  const int b = local / nbg;
  const int band = 4 * (local % nbg) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double c = 0.0;
  if (band < d.B) {
    const T* row = static_cast<const T*>(d.x) + ((int64_t)b * d.blk_lines * d.B + band) * d.S;
    double s = 0.0;
    if constexpr (IN == IN_U16) {
      for (int i = lane; i < d.S; i += 64) s += to_d(row[i]);
      s = wave_sum(s);
      c = s / (double)d.S;
    } else {
      const uint8_t* vl = d.valid + (int64_t)b * d.blk_lines * d.S;
      double cnt = 0.0;
      for (int i = lane; i < d.S; i += 64) {
        const bool ok = vl[i] != 0;
        s += ok ? to_d(row[i]) : 0.0;
        cnt += ok ? 1.0 : 0.0;
      }
      s = wave_sum(s);
      cnt = wave_sum(cnt);
      c = cnt > 0.0 ? s / cnt : 0.0;
    }
    if (P != P_F64) c = (double)(float)c;
  }
  if (lane == 0) d.shift[(int64_t)b * d.Bp + band] = c;
  if constexpr (P == P_FP8) {
    // FP8 operand band scale 2^-e: the first line's largest deviation from
    // the shift lands at or below 224, half of E4M3's largest value (448),
    // leaving a factor of two for the rest of the block; values beyond 448
    // saturate and are counted
    float sc = 0.0f;
    if (band < d.B) {
      const T* row = static_cast<const T*>(d.x) + ((int64_t)b * d.blk_lines * d.B + band) * d.S;
      const float cf = (float)c;
      float m = 0.0f;
      for (int i = lane; i < d.S; i += 64) {
        bool ok = true;
        if constexpr (IN != IN_U16) ok = d.valid[(int64_t)b * d.blk_lines * d.S + i] != 0;
        const float v = ok ? __builtin_fabsf((float)row[i] - cf) : 0.0f;
        m = v > m ? v : m;
      }
      for (int o = 32; o > 0; o >>= 1) {
        const float t = __shfl_xor(m, o, 64);
        m = t > m ? t : m;
      }
      int e = 0;
      if (m > 0.0f) {
        int ex;
        (void)frexpf(m / 224.0f, &ex);           // m / 224 in [2^(ex-1), 2^ex)
        e = ex;                                  // m 2^-e <= 224
      }
      sc = ldexpf(1.0f, -e);
    }
    if (lane == 0 && band < d.Bp) d.sscale[(int64_t)b * d.Bp + band] = sc;
  }
}

// ---------------------------------------------------------------------------- covariance product
// One workgroup = (block b, split s, lower super-tile (I, J)).  Each pixel
// chunk (KC samples of one line) of the split is centred by the shift,
// converted to the operand precision and staged in LDS as [row][k]:
// rows 0..63 are bands 64I.., rows 64..127 bands 64J.. (off-diagonal only).
// Wave w computes the 32x32 sub-block (w>>1, w&1) as 2x2 matrix-core tiles.
template <int IN, int P>
__global__ void __launch_bounds__(NT) k_syrk(LaunchSet ls) {
  using M = MM<P>;
  using S = typename M::storage;
  using T = typename InT<IN>::T;
  using C = typename M::accs;
  constexpr int PADK = 16 / (int)sizeof(S);
  constexpr int LDP = KC + PADK;
  __shared__ S tile[128 * LDP];

  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  const int sup = local % d.nsup;
  const int rest = local / d.nsup;
  int b = rest / d.ks, split = rest % d.ks;
  if (b >= d.nblk - 1) { b = d.nblk - 1; split = rest - (d.nblk - 1) * d.ks; }
  const int ksb = ks_of(d, b);
  int I, J;
  sup_ij(sup, I, J);
  const bool diag = (I == J);
  const int nrows = diag ? 64 : 128;
  const int coloff = diag ? 0 : 64;

  const int lines_b = blk_lines_of(d, b);
  const int64_t nch = (int64_t)lines_b * d.cpl;
  const int64_t c0 = nch * split / ksb, c1 = nch * (split + 1) / ksb;

  const int tid = threadIdx.x;
  const int tpr = NT / nrows;            // threads per staged row: 2 or 4
  const int r = tid / tpr;               // staged row of this thread
  const int segs = 8 / tpr;              // 8-sample segments per thread
  const int seg0 = (tid % tpr) * segs;
  const int band = r < 64 ? 64 * I + r : 64 * J + (r - 64);
  const bool bvalid = band < d.B;
  const double shd = bvalid ? d.shift[(int64_t)b * d.Bp + band] : 0.0;
  const float shf = (float)shd;
  const T* xb = static_cast<const T*>(d.x) + (int64_t)b * d.blk_lines * d.B * d.S;
  double rawsum = 0.0;

  const int w = tid >> 6, lane = tid & 63;
  const int wr = w >> 1, wc = w & 1;
  const bool skip = (diag && wr < wc) || (64 * I + 32 * wr >= d.B) || (64 * J + 32 * wc >= d.B);
  typename M::acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = typename M::acc{};

  const int lr = lane & 15, lk = (lane >> 4) * M::KV;
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int line = (int)(ch / d.cpl);
    const int s0 = (int)(ch % d.cpl) * KC;
    const int nvalid = min(KC, d.S - s0);
    // ---- stage the chunk
    if (r < nrows) {
      const T* row = xb + ((int64_t)line * d.B + band) * d.S + s0;
      const uint8_t* vrow = (IN == IN_U16) ? nullptr : d.valid + ((int64_t)b * d.blk_lines + line) * d.S + s0;
      for (int sg = 0; sg < segs; ++sg) {
        const int k0 = 8 * (seg0 + sg);
        T v[8];
        if (bvalid && d.vec_ok && k0 + 8 <= nvalid) {
          load8(row + k0, v);
        } else if (IN == IN_U16 && bvalid && d.vec8_ok && k0 + 8 <= nvalid) {
          load8_a8(row + k0, v);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = (bvalid && k0 + j < nvalid) ? row[k0 + j] : T(0);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ok = bvalid && (k0 + j < nvalid) && (IN == IN_U16 || vrow[k0 + j] != 0);
          S o;
          if constexpr (P == P_F64) {
            o = ok ? (to_d(v[j]) - shd) : 0.0;
          } else {
            float dv;
            if constexpr (IN == IN_F64) dv = (float)(v[j] - shd);
            else dv = (float)v[j] - shf;
            o = to_storage<P>(ok ? dv : 0.0f);
          }
          tile[r * LDP + k0 + j] = o;
          if (ok) rawsum += to_d(v[j]);
        }
      }
    }
    __syncthreads();
    // ---- matrix-core products over the chunk
    if (!skip) {
#pragma unroll
      for (int st = 0; st < KC / M::KK; ++st) {
        const int kk = st * M::KK + lk;
        typename M::frag a0 = load_frag<P>(&tile[(32 * wr + lr) * LDP + kk]);
        typename M::frag a1 = load_frag<P>(&tile[(32 * wr + 16 + lr) * LDP + kk]);
        typename M::frag b0 = load_frag<P>(&tile[(coloff + 32 * wc + lr) * LDP + kk]);
        typename M::frag b1 = load_frag<P>(&tile[(coloff + 32 * wc + 16 + lr) * LDP + kk]);
        acc[0][0] = M::mma(a0, b0, acc[0][0]);
        acc[0][1] = M::mma(a0, b1, acc[0][1]);
        acc[1][0] = M::mma(a1, b0, acc[1][0]);
        acc[1][1] = M::mma(a1, b1, acc[1][1]);
      }
    }
    __syncthreads();
  }

  // ---- write the partial scatter into the split's Bp x Bp matrix (lower part)
  const int64_t slot = (int64_t)b * d.ks + split;
  if (!skip) {
    C* out = static_cast<C*>(d.part) + slot * d.Bp * d.Bp;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gi = 64 * I + 32 * wr + 16 * ti + M::out_row(lane >> 4, j);
          const int gj = 64 * J + 32 * wc + 16 * tj + lr;
          if (gi < d.Bp && gj < d.Bp) out[(int64_t)gi * d.Bp + gj] = acc[ti][tj][j];
        }
  }
  // ---- raw band sums (diagonal super-tiles cover every band exactly once)
  if (diag) {
    for (int o = 1; o < tpr; o <<= 1) rawsum += __shfl_xor(rawsum, o, 64);
    if ((tid % tpr) == 0 && band < d.Bp) d.psum[slot * d.Bp + band] = bvalid ? rawsum : 0.0;
  }
}

// ---------------------------------------------------------------------------- covariance product, 8-value formats
// One 1024-thread workgroup = (block b, split s) owns the WHOLE lower triangle
// for its pixel range, so every input element is read from memory once and
// the split partial is one Bp x Bp matrix.  Chunks of KC pixels (one line
// segment) are centred, rounded to the operand format and staged in LDS as
// [band][k] (double-buffered, the next chunk's loads in flight while the
// current one is multiplied).  Wave w owns a rectangle of at most 4 x 4
// 16-band tiles (rect table from the host; at most 15 rectangles for
// B <= 320): per 32-pixel step it reads its row fragments once and each
// column fragment once from LDS.  Raw band sums ride along in the staging.
constexpr int S2NT = 1024;
constexpr int S2LDK = KC + 8;              // LDS row pitch (elements)
constexpr int S2IT = (16 * MAXT * 8 + S2NT - 1) / S2NT;   // staging items per thread

template <int IN, int P>
__global__ void __launch_bounds__(S2NT) k_syrk2(LaunchSet ls) {
  using M = MM<P>;
  using S = typename M::storage;
  using T = typename InT<IN>::T;
  static_assert(M::KV == 8, "8-value operand formats only");
  __shared__ __attribute__((aligned(16))) S tile[2][16 * MAXT * S2LDK];

  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  int b = local / d.ks, split = local % d.ks;
  if (b >= d.nblk - 1) { b = d.nblk - 1; split = local - (d.nblk - 1) * d.ks; }
  const int ksb = ks_of(d, b);
  const int lines_b = blk_lines_of(d, b);
  const int64_t nch = (int64_t)lines_b * d.cpl;
  const int64_t c0 = nch * split / ksb, c1 = nch * (split + 1) / ksb;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const T* xb = static_cast<const T*>(d.x) + (int64_t)b * d.blk_lines * d.B * d.S;

  // staging items: item = row * 8 + segment of 8 samples, fixed per thread.
  // Raw sums are exact: uint32 for 16-bit input (a split has at most 8192
  // chunks, and a thread adds 8 values of at most 65535 per chunk to each
  // sum: below 2^32), FP64 otherwise.
  using RS = typename std::conditional<IN == IN_U16, uint32_t, double>::type;
  float shf[S2IT], bsc[S2IT];               // shift, and the FP8 operand's band scale
  RS rawsum[S2IT];
  uint32_t nclip = 0;                         // FP8: operand values beyond the format's range
#pragma unroll
  for (int q = 0; q < S2IT; ++q) {
    const int r = (tid + S2NT * q) >> 3;
    shf[q] = (r < d.B) ? (float)d.shift[(int64_t)b * d.Bp + r] : 0.0f;
    bsc[q] = (P == P_FP8 && r < d.B) ? d.sscale[(int64_t)b * d.Bp + r] : 1.0f;
    rawsum[q] = RS(0);
  }
  auto row_of = [&](int q) { const int it = tid + S2NT * q; return (it < d.Bp * 8) ? (it >> 3) : -1; };
  const int k0 = 8 * (tid & 7);
  constexpr int RW = 8 * (int)sizeof(T) / 16;     // 16-byte words per 8 input values
  uint4 raw[S2IT][RW];                              // next chunk, kept packed until it is staged
  auto load = [&](int64_t ch) {
    const int line = (int)(ch / d.cpl);
    const int s0 = (int)(ch % d.cpl) * KC;
    const int nvalid = min(KC, d.S - s0);
#pragma unroll
    for (int q = 0; q < S2IT; ++q) {
      const int r = row_of(q);
      if (r >= 0 && r < d.B) {
        const T* row = xb + ((int64_t)line * d.B + r) * d.S + s0;
        if (d.vec_ok && k0 + 8 <= nvalid) {
#pragma unroll
          for (int w = 0; w < RW; ++w) raw[q][w] = reinterpret_cast<const uint4*>(row + k0)[w];
        } else if (IN == IN_U16 && d.vec8_ok && k0 + 8 <= nvalid) {
          const uint2 h0 = reinterpret_cast<const uint2*>(row + k0)[0];
          const uint2 h1 = reinterpret_cast<const uint2*>(row + k0)[1];
          raw[q][0] = uint4{h0.x, h0.y, h1.x, h1.y};
        } else {
          T t[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) t[j] = (k0 + j < nvalid) ? row[k0 + j] : T(0);
          pack8(t, raw[q]);
        }
      }
    }
    if constexpr (IN == IN_U16) {
      return nvalid;
    } else {
      // float input: bits 16.. carry which of this thread's 8 samples are valid
      const uint8_t* vl = d.valid + ((int64_t)b * d.blk_lines + line) * d.S + s0;
      int vm = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) vm |= (k0 + j < nvalid && vl[k0 + j] != 0) ? (1 << j) : 0;
      return nvalid | (vm << 16);
    }
  };
  auto store = [&](int buf, int packed) {
    const int nvalid = (IN == IN_U16) ? packed : (packed & 0xffff);
#pragma unroll
    for (int q = 0; q < S2IT; ++q) {
      const int r = row_of(q);
      if (r < 0) continue;
      T vv[8];
      unpack8(raw[q], vv);
      S o[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool ok = (r < d.B) && (k0 + j < nvalid) && (IN == IN_U16 || ((packed >> (16 + j)) & 1));
        float dv;
        if constexpr (IN == IN_F64) dv = (float)(vv[j] - (double)d.shift[(int64_t)b * d.Bp + r]);
        else dv = (float)vv[j] - shf[q];
        if constexpr (P == P_FP8) {
          dv *= bsc[q];                       // a power of two: exact
          nclip += ok ? e4m3_clips(dv) : 0u;
        }
        o[j] = to_storage<P>(ok ? dv : 0.0f);
        if (ok) rawsum[q] += (RS)vv[j];
      }
      if constexpr (sizeof(S) == 1) {
        uint2 ow;
        ow.x = (uint32_t)o[0] | ((uint32_t)o[1] << 8) | ((uint32_t)o[2] << 16) | ((uint32_t)o[3] << 24);
        ow.y = (uint32_t)o[4] | ((uint32_t)o[5] << 8) | ((uint32_t)o[6] << 16) | ((uint32_t)o[7] << 24);
        *reinterpret_cast<uint2*>(&tile[buf][r * S2LDK + k0]) = ow;
      } else {
        uint4 ow;
        ow.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16); ow.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
        ow.z = (uint32_t)o[4] | ((uint32_t)o[5] << 16); ow.w = (uint32_t)o[6] | ((uint32_t)o[7] << 16);
        *reinterpret_cast<uint4*>(&tile[buf][r * S2LDK + k0]) = ow;
      }
    }
  };

  // this wave's rectangle
  const int rr0 = (wv < d.nrect) ? d.rect[wv][0] : 0, rc0 = (wv < d.nrect) ? d.rect[wv][1] : 0;
  const int rnr = (wv < d.nrect) ? d.rect[wv][2] : 0, rnc = (wv < d.nrect) ? d.rect[wv][3] : 0;
  typename M::acc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = typename M::acc{};
  const int lr = lane & 15, lk = (lane >> 4) * 8;

  int buf = 0;
  if (c0 < c1) {
    const int nv = load(c0);
    store(0, nv);
  }
  __syncthreads();
  for (int64_t ch = c0; ch < c1; ++ch) {
    int nvn = 0;
    const bool more = ch + 1 < c1;
    if (more) nvn = load(ch + 1);             // next chunk's loads in flight during the products
    const S* tb = tile[buf];
#pragma unroll
    for (int st = 0; st < KC / 32; ++st) {
      const int kk = 32 * st + lk;
      typename M::frag a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < rnr) a[i] = load_frag<P>(&tb[(16 * (rr0 + i) + lr) * S2LDK + kk]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j < rnc) {
          const typename M::frag bf = load_frag<P>(&tb[(16 * (rc0 + j) + lr) * S2LDK + kk]);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (i < rnr && rr0 + i >= rc0 + j) acc[i][j] = M::mma(a[i], bf, acc[i][j]);
        }
      }
    }
    if (more) store(buf ^ 1, nvn);
    __syncthreads();
    buf ^= 1;
  }

  // partial scatter of this split: lower tiles of the rectangle into the Bp x Bp matrix
  const int64_t slot = (int64_t)b * d.ks + split;
  using C = typename M::accs;
  C* out = static_cast<C*>(d.part) + slot * d.Bp * d.Bp;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (i < rnr && j < rnc && rr0 + i >= rc0 + j) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gi = 16 * (rr0 + i) + M::out_row(lane >> 4, e), gj = 16 * (rc0 + j) + lr;
          float v = acc[i][j][e];
          if constexpr (P == P_FP8) {
            // undo the band scales (powers of two): the partial of the unscaled products
            const float si = d.sscale[(int64_t)b * d.Bp + gi], sj = d.sscale[(int64_t)b * d.Bp + gj];
            v = (si > 0.0f && sj > 0.0f) ? (v / si) / sj : 0.0f;
          }
          out[(int64_t)gi * d.Bp + gj] = v;
        }
      }
  if constexpr (P == P_FP8) wave_count(d.cnt64 + 2, nclip);
  // raw band sums: the 8 segments of a row are 8 adjacent lanes
#pragma unroll
  for (int q = 0; q < S2IT; ++q) {
    double t = (double)rawsum[q];
    t += __shfl_xor(t, 1, 64);
    t += __shfl_xor(t, 2, 64);
    t += __shfl_xor(t, 4, 64);
    const int r = row_of(q);
    if ((tid & 7) == 0 && r >= 0) d.psum[slot * d.Bp + r] = t;
  }
}

// ---------------------------------------------------------------------------- covariance product, 16-bit input, direct-to-LDS staging
// As k_syrk2, for 16-bit input with 16-byte aligned rows: the raw chunks are
// loaded straight into a three-deep LDS ring (global_load_lds_dwordx4, no
// registers), two chunks ahead of the one being multiplied.  Row r's eight
// 16-byte segments are stored XOR-swizzled (slot = segment ^ (r & 7)) so
// the 16-row fragment reads hit distinct banks; each thread converts its own
// slots in place (centred in FP32, rounded to the operand format) and keeps
// the exact raw band sums.  Every wave issues exactly S2IT loads per chunk,
// also for rounds past the band count, so waiting for a chunk is a fixed
// count of outstanding loads that the compiler can follow slot by slot.
constexpr int S3ROWS = 16 * MAXT;          // band rows (shift table)
constexpr int S3RING = 128 * S2IT;         // rows per ring buffer: S2IT rounds of 128


// R > 1 (launches with few splits, e.g. a lone block): R workgroups share a
// split, all staging every chunk of it; workgroup r of the R multiplies only
// the fragment columns j = r (mod R) of each super-tile.  Every output
// fragment sees the same MFMA sequence (chunk order, then the two 32-sample
// steps) as with R = 1, so the partials are bit-identical whatever R is.
template <int P, int R>
__global__ void __launch_bounds__(S2NT) k_syrk3(LaunchSet ls) {
  static_assert(R == 1 || R == 2 || R == 4, "fragment columns per super-tile split evenly");
  constexpr int NJ = 4 / R;                      // fragment columns per wave
  using M = MM<P>;
  using S = typename M::storage;
  static_assert(M::KV == 8 && sizeof(S) == 2, "16-bit operand formats only");
  // three distinct LDS objects, used in a statically known rotation, so the
  // compiler tracks the in-flight direct loads of each one separately
  __shared__ __attribute__((aligned(16))) uint16_t ring0[S3RING * KC];
  __shared__ __attribute__((aligned(16))) uint16_t ring1[S3RING * KC];
  __shared__ __attribute__((aligned(16))) uint16_t ring2[S3RING * KC];
  __shared__ float shl[S3ROWS];

  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  const int cgrp = local % R;                    // this workgroup's fragment columns
  local /= R;
  int b = local / d.ks, split = local % d.ks;
  if (b >= d.nblk - 1) { b = d.nblk - 1; split = local - (d.nblk - 1) * d.ks; }
  const int ksb = ks_of(d, b);
  const int lines_b = blk_lines_of(d, b);
  // chunk indices of one block fit in 32 bits (a block is a few thousand lines)
  const int nch = lines_b * d.cpl;
  const int c0 = (int)((int64_t)nch * split / ksb), c1 = (int)((int64_t)nch * (split + 1) / ksb);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint16_t* xb = static_cast<const uint16_t*>(d.x) + (int64_t)b * d.blk_lines * d.B * d.S;
  const int lrow = lane >> 3, lslot = lane & 7;

  // Round q of a chunk: wave wv loads rows 128 q + 8 wv + lrow, lane slot
  // lslot holding segment lslot ^ lrow (r & 7 == lrow).  Addresses are a
  // wave-uniform line base plus a 32-bit per-lane offset; lanes past the band
  // count or the row end load the line's first word (in bounds).  Rows below
  // the padded band count get zeros from the conversion; rows past it are
  // read only by products whose tiles are never stored.
  // The descriptor fields live in registers for the whole loop, and chunk
  // positions advance one chunk at a time (no division per chunk): a chunk
  // is KC samples of one line, at sample s0 of the line starting at lb.
  const int nB = d.B, nBp = d.Bp, nS = d.S;
  const int64_t line_bytes = 2 * (int64_t)nB * nS;
  struct Pos { const char* lb; int s0; };
  auto advance = [&](Pos& p) {
    p.s0 += KC;
    if (p.s0 >= nS) { p.s0 = 0; p.lb += line_bytes; }
  };
  const int segc = lslot ^ lrow;
  uint32_t offq[S2IT];                           // lane offsets of a whole chunk, per round
#pragma unroll
  for (int q = 0; q < S2IT; ++q)
    offq[q] = (128 * q + 8 * wv + lrow < nB)
                  ? 2u * ((uint32_t)(128 * q + 8 * wv + lrow) * (uint32_t)nS + 8u * (uint32_t)segc) : 0u;
  auto issue = [&](const Pos& p, uint16_t* buf) {
    const char* lb = p.lb + 2 * p.s0;
    const bool ragged = nS - p.s0 < KC;          // wave-uniform
#pragma unroll
    for (int q = 0; q < S2IT; ++q) {
      uint32_t off = offq[q];
      if (ragged) off = (8 * segc < nS - p.s0) ? off : 0u;
      __builtin_amdgcn_global_load_lds((const void*)(lb + off),
                                       (__attribute__((address_space(3))) void*)(buf + (128 * q + 8 * wv) * KC),
                                       16, 0, 0);
    }
  };

  uint32_t rawsum[S2IT];
#pragma unroll
  for (int q = 0; q < S2IT; ++q) rawsum[q] = 0u;
  for (int r = tid; r < nBp; r += S2NT) shl[r] = (r < nB) ? (float)d.shift[(int64_t)b * nBp + r] : 0.0f;
  // The direct path runs only when the sample count is a multiple of 8, so an
  // 8-sample segment is either wholly inside the row or wholly past its end.
  // Per 32-bit word (two samples): two conversions and two subtractions in
  // FP32 (exact for any 16-bit count), one packed rounding to the operand
  // format, and the exact raw sum by a 16-bit dot product with (1, 1).
  // Rounds whose 8 rows all lie inside the band count, in chunks without a
  // ragged end, need no masking (a wave-uniform test); elsewhere items
  // outside become raw 0 with shift 0 and so convert to +0.
  auto convert = [&](int s0, uint16_t* buf) {
    const int nvalid = min(KC, nS - s0);
#pragma unroll
    for (int q = 0; q < S2IT; ++q) {
      const int rb = 128 * q + 8 * wv;           // first row of the wave's round (uniform)
      if (rb >= nBp) continue;
      const int r = rb + lrow;
      uint4* p = reinterpret_cast<uint4*>(buf + r * KC + 8 * lslot);
      uint4 wv4 = *p;
      float sh = shl[r];
      if (!(rb + 8 <= nB && nvalid == KC)) {
        const bool ok = (r < nB) && (8 * segc < nvalid);
        wv4 = ok ? wv4 : uint4{0u, 0u, 0u, 0u};
        sh = ok ? sh : 0.0f;
      }
      const uint32_t wd[4] = {wv4.x, wv4.y, wv4.z, wv4.w};
      uint32_t o[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        rawsum[q] = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, wd[h]), u16x2{1, 1}, rawsum[q], false);
        o[h] = cvt_pack2<P>((float)(wd[h] & 0xffffu) - sh, (float)(wd[h] >> 16) - sh);
      }
      *p = uint4{o[0], o[1], o[2], o[3]};
    }
  };

  // wave wv owns the 64x64 super-tile (I, J), I >= J, of the lower triangle
  // (at most 15 of them for 320 bands); it multiplies the fragment rows of it
  // that hold a stored tile and keeps the lower tiles.  Rows past the band
  // count read ring rows that are either zero or never written out.
  int I = 0, J = 0;
  {
    int t = wv;
    while (t > I) { t -= I + 1; ++I; }
    J = t;
  }
  const int nsup = (nBp + 63) >> 6;
  const bool active = I < nsup;
  typename M::acc acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = typename M::acc{};
  const int lr = lane & 15, lkg = lane >> 4;
  // fragment rows that hold no stored fragment (past the padded band count,
  // or wholly above the diagonal) are not multiplied; the stored fragments'
  // MFMA sequences are unchanged
  uint32_t rowm = 0;
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int jc = cgrp + R * j;
      if (64 * I + 16 * ii < nBp && 64 * J + 16 * jc < nBp && (I > J || ii >= jc)) rowm |= 1u << ii;
    }
  rowm = __builtin_amdgcn_readfirstlane(rowm);

  auto multiply = [&](const uint16_t* tb) {
    if (!active) return;
#pragma unroll
    for (int st = 0; st < KC / 32; ++st) {
      const int g = 4 * st + lkg;               // 8-value k-group within the chunk
      const int off = lr * KC + 8 * (g ^ (lr & 7));
      typename M::frag a[4], bq[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        bq[j] = load_frag<P>(reinterpret_cast<const S*>(tb + (64 * J + 16 * (cgrp + R * j)) * KC + off));
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
        if ((rowm >> ii) & 1u) {
          a[ii] = load_frag<P>(reinterpret_cast<const S*>(tb + (64 * I + 16 * ii) * KC + off));
#pragma unroll
          for (int j = 0; j < NJ; ++j) acc[ii][j] = M::mma(a[ii], bq[j], acc[ii][j]);
        }
    }
  };
  // Each lane converts exactly the 16 bytes it loaded itself (same row and
  // slot mapping in issue and convert), so converting a chunk needs only the
  // wave's own load count, not a barrier.  One barrier per chunk: after it,
  // every wave has converted chunk ch (the products may read any row) and
  // finished multiplying chunk ch - 1 (its slot takes chunk ch + 2).  Then the
  // wave queues ch + 2, multiplies ch and converts its own rows of ch + 1,
  // whose loads were queued two products earlier; one wave's conversion
  // overlaps the products of another on the same SIMD.
  // Steady state: every step queues exactly S2IT loads, and waiting for the
  // previous chunk leaves exactly those in flight.
  static_assert(S2IT <= 15, "vmcnt immediate");
  // ip: next chunk to queue; cs0: first sample of the next chunk to convert
  Pos ip;
  {
    const int line = c0 / d.cpl;
    ip = Pos{reinterpret_cast<const char*>(xb) + line * line_bytes, (c0 - line * d.cpl) * KC};
  }
  int cs0 = ip.s0;
  auto conv_next = [&](uint16_t* buf) {
    convert(cs0, buf);
    cs0 += KC;
    if (cs0 >= nS) cs0 = 0;
  };
  auto queue_next = [&](uint16_t* buf) {
    issue(ip, buf);
    advance(ip);
  };
  auto full = [&](uint16_t* cur, uint16_t* nxt, uint16_t* ahead) {
    lds_barrier();
    queue_next(ahead);
    multiply(cur);
    __builtin_amdgcn_s_waitcnt(0x0F70 | S2IT);
    conv_next(nxt);
  };
  // the last steps: nothing or only the final chunk left to queue
  auto last = [&](int ch, uint16_t* cur, uint16_t* nxt, uint16_t* ahead) {
    lds_barrier();
    if (ch + 2 < c1) queue_next(ahead);
    multiply(cur);
    if (ch + 2 < c1) {
      __builtin_amdgcn_s_waitcnt(0x0F70 | S2IT);
      conv_next(nxt);
    } else if (ch + 1 < c1) {
      __builtin_amdgcn_s_waitcnt(0x0F70);
      conv_next(nxt);
    }
  };

  // the shifts in shl are written by other threads than the ones reading
  // them; publish them before the first conversion (nothing in flight yet)
  __syncthreads();
  if (c0 + 1 < c1) {
    queue_next(ring0);
    queue_next(ring1);
    __builtin_amdgcn_s_waitcnt(0x0F70 | S2IT);
    conv_next(ring0);
  } else if (c0 < c1) {
    queue_next(ring0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    conv_next(ring0);
  }
  int ch = c0;
  for (; ch + 4 < c1; ch += 3) {
    full(ring0, ring1, ring2);
    full(ring1, ring2, ring0);
    full(ring2, ring0, ring1);
  }
  // at most four chunks remain, continuing the rotation at ring0
  if (ch < c1) last(ch, ring0, ring1, ring2);
  if (ch + 1 < c1) last(ch + 1, ring1, ring2, ring0);
  if (ch + 2 < c1) last(ch + 2, ring2, ring0, ring1);
  if (ch + 3 < c1) last(ch + 3, ring0, ring1, ring2);

  const int64_t slot = (int64_t)b * d.ks + split;
  using C = typename M::accs;
  C* out = static_cast<C*>(d.part) + slot * d.Bp * d.Bp;
  if (active) {
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int ti = 4 * I + ii, tj = 4 * J + cgrp + R * j;
        if (16 * ti < d.Bp && ti >= tj) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gi = 16 * ti + M::out_row(lane >> 4, e), gj = 16 * tj + lr;
            out[(int64_t)gi * d.Bp + gj] = acc[ii][j][e];
          }
        }
      }
  }
  if (cgrp != 0) return;                         // one workgroup of the R writes the band sums
#pragma unroll
  for (int q = 0; q < S2IT; ++q) {
    double t = (double)rawsum[q];
    t += __shfl_xor(t, 1, 64);
    t += __shfl_xor(t, 2, 64);
    t += __shfl_xor(t, 4, 64);
    const int r = (tid + S2NT * q) >> 3;
    if ((tid & 7) == 0 && r < d.Bp) d.psum[slot * d.Bp + r] = t;
  }
}

// ---------------------------------------------------------------------------- merge
constexpr int MB = 64;      // elements (bands, or matrix entries) per merge workgroup
constexpr int MW = 4;       // waves per merge workgroup
constexpr int MAXBLK = 64;  // blocks per batch (reset bits are a 64-bit mask)

// Vector part: one workgroup per 64 bands.  The four waves share out the
// blocks and form every block's exact raw band sum (fixed-order sum over its
// splits) into LDS, then one wave runs the sequential recurrence over blocks:
// block mean m_b, e = m_b - shift, d = m_b - window mean before the block,
// window sums after it, and per block the pairwise-update weight
// N n_b / (N + n_b) (0 when the window was empty: the block's scatter
// replaces the window's; -1 when the block has no finite pixel: the window
// is left as it was).  n_b counts the block's finite pixels; the window
// count N travels with the window sums (entry Bp).
__global__ void __launch_bounds__(MB * MW) k_merge_vec(LaunchSet ls) {
  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  __shared__ double sb[MAXBLK][MB];
  __shared__ double shb[MAXBLK][MB];
  const int lane = threadIdx.x & (MB - 1), w = threadIdx.x / MB;
  const int k = MB * local + lane;
  const bool in = k < d.B;
  for (int b = w; b < d.nblk; b += MW) {
    const int ksb = ks_of(d, b);
    double t = 0.0;
    if (in) {
      // eight loads in flight, added in split order
      const double* ps = d.psum + (int64_t)b * d.ks * d.Bp + k;
      int s = 0;
      for (; s + 8 <= ksb; s += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = ps[(int64_t)(s + u) * d.Bp];
#pragma unroll
        for (int u = 0; u < 8; ++u) t += a[u];
      }
      for (; s < ksb; ++s) t += ps[(int64_t)s * d.Bp];
    }
    sb[b][lane] = t;
    shb[b][lane] = (k < d.Bp) ? d.shift[(int64_t)b * d.Bp + k] : 0.0;
  }
  __syncthreads();
  if (w != 0 || k >= d.Bp) return;
  double N = d.s1_in[d.Bp];
  double s1 = in ? d.s1_in[k] : 0.0;
  if (d.causal == 1) {                   // slot nblk: the window before the batch
    const bool r0 = d.reset_bits & 1ull;
    const int64_t o = (int64_t)d.nblk * d.Bp + k;
    d.mu_snap[o] = (in && !r0 && N > 0.0) ? s1 / N : 0.0;
    if (k == 0) d.n_snap[d.nblk] = r0 ? 0.0 : N;
  }
  for (int b = 0; b < d.nblk; ++b) {
    const int lb = blk_lines_of(d, b);
    double nb = (double)lb * d.S;
    if (d.nbadl) {
      int bad = 0;
      for (int l = 0; l < lb; ++l) bad += d.nbadl[b * d.blk_lines + l];
      nb -= (double)bad;
    }
    if ((d.reset_bits >> b) & 1ull) { N = 0.0; s1 = 0.0; }
    const int64_t o = (int64_t)b * d.Bp + k;
    if (k == 0) d.nbv[b] = nb;
    if (nb > 0.0) {
      const double mb = sb[b][lane] / nb;
      d.ev[o] = in ? mb - shb[b][lane] : 0.0;
      d.dv[o] = (in && N > 0.0) ? mb - s1 / N : 0.0;
      if (k == 0) d.coef[b] = N > 0.0 ? N * nb / (N + nb) : 0.0;
      s1 += sb[b][lane];
      N += nb;
    } else {
      d.ev[o] = 0.0;
      d.dv[o] = 0.0;
      if (k == 0) d.coef[b] = -1.0;
    }
    d.mu_snap[o] = (in && N > 0.0) ? s1 / N : 0.0;
    if (k == 0) d.n_snap[b] = N;
  }
  d.s1_out[k] = in ? s1 : 0.0;
  if (k == 0) d.s1_out[d.Bp] = N;
}

// Matrix part, by row strips: a workgroup owns 4 consecutive rows and 64
// consecutive columns at or below the diagonal; wave w takes row 4g + w and
// lane l column 64c + l, so every load of a split partial is one contiguous
// 256-byte row segment.  Two launches, so the per-block sums over the split
// partials (the bulk of the reads) run in parallel over blocks instead of
// inside the recurrence over blocks:
//   k_merge_red: one workgroup per (block, row strip): C_b = fixed-order FP64
//     sum of the block's split partials, M2_b = C_b - n_b e e^T, written over
//     the block's snapshot slot;
//   k_merge_rec: one workgroup per row strip: the pairwise recurrence over
//     the blocks in order (M <- M + M2_b + w d d^T; M <- M2_b for an empty
//     window; M unchanged for a block with no finite pixel), each block's
//     M2_b read back from its slot (loads independent of the recurrence,
//     eight blocks ahead) and replaced by the window's scatter matrix after
//     the block.
__device__ __forceinline__ bool strip_entry(const BatchDesc& d, int q, int& gi, int& gj) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int g = 0;
  while (q >= (4 * g + 67) / 64) { q -= (4 * g + 67) / 64; ++g; }
  gi = 4 * g + w;
  gj = 64 * q + lane;
  return gi < d.B && gj <= gi;
}

template <typename PT>
__global__ void __launch_bounds__(MB * MW) k_merge_red(LaunchSet ls) {
  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  int strips = 0;
  for (int g = 0; g < d.Bp / 4; ++g) strips += (4 * g + 67) / 64;
  const int b = local / strips, q = local % strips;
  int gi, gj;
  if (!strip_entry(d, q, gi, gj)) return;
  const int64_t bp2 = (int64_t)d.Bp * d.Bp, e = (int64_t)gi * d.Bp + gj;
  const double nb = d.nbv[b];
  const int ksb = ks_of(d, b);
  const PT* pb = static_cast<const PT*>(d.part) + (int64_t)b * d.ks * bp2 + e;
  double c = 0.0;
  int sp = 0;
  for (; sp + 8 <= ksb; sp += 8) {             // eight loads in flight, summed in order
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = (double)pb[(sp + u) * bp2];
#pragma unroll
    for (int u = 0; u < 8; ++u) c += a[u];
  }
  for (; sp < ksb; ++sp) c += (double)pb[sp * bp2];
  const int64_t o = (int64_t)b * d.Bp;
  d.m2_snap[b * bp2 + e] = c - nb * d.ev[o + gi] * d.ev[o + gj];
}

__global__ void __launch_bounds__(MB * MW) k_merge_rec(LaunchSet ls) {
  int q;
  const int bi = find_batch(ls, blockIdx.x, q);
  const BatchDesc& d = ls.d[bi];
  int gi, gj;
  if (!strip_entry(d, q, gi, gj)) return;
  const int64_t bp2 = (int64_t)d.Bp * d.Bp, e = (int64_t)gi * d.Bp + gj;
  double m2 = d.m2_in[e];
  if (d.causal == 1) d.m2_snap[d.nblk * bp2 + e] = (d.reset_bits & 1ull) ? 0.0 : m2;   // window before the batch
  constexpr int PF = 8;                            // blocks whose M2_b are loaded ahead
  for (int b0 = 0; b0 < d.nblk; b0 += PF) {
    double mbv[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t) mbv[t] = (b0 + t < d.nblk) ? d.m2_snap[(b0 + t) * bp2 + e] : 0.0;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int b = b0 + t;
      if (b >= d.nblk) break;
      const int64_t o = (int64_t)b * d.Bp;
      if ((d.reset_bits >> b) & 1ull) m2 = 0.0;
      const double wgt = d.coef[b];
      if (wgt >= 0.0) m2 = (wgt > 0.0) ? m2 + mbv[t] + wgt * d.dv[o + gi] * d.dv[o + gj] : mbv[t];
      d.m2_snap[b * bp2 + e] = m2;
    }
  }
  d.m2_out[e] = m2;
}

// Workgroups per split of the direct-load covariance kernel: the largest of
// 4, 2, 1 that keeps the launch within the device's CU count (one workgroup
// per CU).  The choice only spreads work; it never changes a partial.
static int syrk3_share(int wg) {
  static std::atomic<int> cus[64];
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1;
  n = cus[dev].load(std::memory_order_relaxed);
  if (n == 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 1;
    cus[dev].store(n, std::memory_order_relaxed);
  }
  return (4 * wg <= n) ? 4 : ((2 * wg <= n) ? 2 : 1);
}

}  // namespace rxk

// Host entry used by the runtime: phase 3 validity (float input, before
// the others), 0 centring shift, 1 covariance product, 2 merge (vector then
// matrix part).  wg: workgroups of the phase
// (for phase 2: wg = vector workgroups, wg2 = matrix workgroups).
extern "C" hipError_t rxk_launch_stats(int in_type, int prec, int phase, const rxk::LaunchSet* ls, int wg,
                                       const rxk::LaunchSet* ls2, int wg2, hipStream_t st) {
  using namespace rxk;
  if (phase == 3) {
    if (wg <= 0) return hipSuccess;
    if (in_type == IN_F32) hipLaunchKernelGGL(k_valid<IN_F32>, dim3(wg), dim3(NT), 0, st, *ls);
    else if (in_type == IN_F64) hipLaunchKernelGGL(k_valid<IN_F64>, dim3(wg), dim3(NT), 0, st, *ls);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (phase == 2) {
    if (wg > 0) hipLaunchKernelGGL(k_merge_vec, dim3(wg), dim3(MB * MW), 0, st, *ls);
    if (wg2 > 0) {
      LaunchSet r = *ls2;                     // the strips of every block of each batch
      r.wg0[0] = 0;
      for (int i = 0; i < r.nb; ++i) r.wg0[i + 1] = r.wg0[i] + (ls2->wg0[i + 1] - ls2->wg0[i]) * r.d[i].nblk;
      if (prec == P_F64) hipLaunchKernelGGL((k_merge_red<double>), dim3(r.wg0[r.nb]), dim3(MB * MW), 0, st, r);
      else hipLaunchKernelGGL((k_merge_red<float>), dim3(r.wg0[r.nb]), dim3(MB * MW), 0, st, r);
      hipLaunchKernelGGL(k_merge_rec, dim3(wg2), dim3(MB * MW), 0, st, *ls2);
    }
    return hipGetLastError();
  }
  if (wg <= 0) return hipSuccess;
  if (prec == P_FP8) {                       // FP8 operands with band scales: the register-staged kernels
    if (phase == 0) {
      if (in_type == IN_U16) hipLaunchKernelGGL((k_shift<IN_U16, P_FP8>), dim3(wg), dim3(NT), 0, st, *ls);
      else if (in_type == IN_F32) hipLaunchKernelGGL((k_shift<IN_F32, P_FP8>), dim3(wg), dim3(NT), 0, st, *ls);
      else hipLaunchKernelGGL((k_shift<IN_F64, P_FP8>), dim3(wg), dim3(NT), 0, st, *ls);
    } else {
      if (in_type == IN_U16) hipLaunchKernelGGL((k_syrk2<IN_U16, P_FP8>), dim3(wg), dim3(S2NT), 0, st, *ls);
      else if (in_type == IN_F32) hipLaunchKernelGGL((k_syrk2<IN_F32, P_FP8>), dim3(wg), dim3(S2NT), 0, st, *ls);
      else hipLaunchKernelGGL((k_syrk2<IN_F64, P_FP8>), dim3(wg), dim3(S2NT), 0, st, *ls);
    }
    return hipGetLastError();
  }
  if (phase == 1 && in_type == IN_U16 && (prec == P_BF16 || prec == P_F16)) {
    // aligned 16-bit batches take the direct-load kernel, the others the
    // register-staged one; the choice is per batch, so a block's partials
    // never depend on what else shares the launch
    LaunchSet a, o;
    a.nb = o.nb = 0;
    a.wg0[0] = o.wg0[0] = 0;
    for (int i = 0; i < ls->nb; ++i) {
      LaunchSet& t = ls->d[i].vec_ok ? a : o;
      t.d[t.nb] = ls->d[i];
      t.wg0[t.nb + 1] = t.wg0[t.nb] + (ls->wg0[i + 1] - ls->wg0[i]);
      ++t.nb;
    }
    if (a.nb > 0) {
      // few splits in the launch (a lone block has about 11): share each
      // split among R workgroups so the launch still covers most CUs
      const int R = syrk3_share(a.wg0[a.nb]);
      for (int i = 0; i <= a.nb; ++i) a.wg0[i] *= R;
      const dim3 g(a.wg0[a.nb]);
      if (prec == P_BF16) {
        if (R == 4) hipLaunchKernelGGL((k_syrk3<P_BF16, 4>), g, dim3(S2NT), 0, st, a);
        else if (R == 2) hipLaunchKernelGGL((k_syrk3<P_BF16, 2>), g, dim3(S2NT), 0, st, a);
        else hipLaunchKernelGGL((k_syrk3<P_BF16, 1>), g, dim3(S2NT), 0, st, a);
      } else {
        if (R == 4) hipLaunchKernelGGL((k_syrk3<P_F16, 4>), g, dim3(S2NT), 0, st, a);
        else if (R == 2) hipLaunchKernelGGL((k_syrk3<P_F16, 2>), g, dim3(S2NT), 0, st, a);
        else hipLaunchKernelGGL((k_syrk3<P_F16, 1>), g, dim3(S2NT), 0, st, a);
      }
    }
    if (o.nb > 0) {
      if (prec == P_BF16) hipLaunchKernelGGL((k_syrk2<IN_U16, P_BF16>), dim3(o.wg0[o.nb]), dim3(S2NT), 0, st, o);
      else hipLaunchKernelGGL((k_syrk2<IN_U16, P_F16>), dim3(o.wg0[o.nb]), dim3(S2NT), 0, st, o);
    }
    return hipGetLastError();
  }
#define RXK_CASE(INV, PV)                                                                      \
  if (in_type == INV && prec == PV) {                                                          \
    if (phase == 0) hipLaunchKernelGGL((k_shift<INV, PV>), dim3(wg), dim3(NT), 0, st, *ls);    \
    else if (MM<PV>::KV == 8) hipLaunchKernelGGL((k_syrk2<INV, (MM<PV>::KV == 8 ? PV : P_BF16)>), dim3(wg), dim3(S2NT), 0, st, *ls); \
    else hipLaunchKernelGGL((k_syrk<INV, PV>), dim3(wg), dim3(NT), 0, st, *ls);                \
    return hipGetLastError();                                                                  \
  }
  RXK_CASE(IN_U16, P_F64) RXK_CASE(IN_U16, P_F32) RXK_CASE(IN_U16, P_BF16) RXK_CASE(IN_U16, P_F16)
  RXK_CASE(IN_F32, P_F64) RXK_CASE(IN_F32, P_F32) RXK_CASE(IN_F32, P_BF16) RXK_CASE(IN_F32, P_F16)
  RXK_CASE(IN_F64, P_F64) RXK_CASE(IN_F64, P_F32) RXK_CASE(IN_F64, P_BF16) RXK_CASE(IN_F64, P_F16)
#undef RXK_CASE
  return hipErrorInvalidValue;
}
