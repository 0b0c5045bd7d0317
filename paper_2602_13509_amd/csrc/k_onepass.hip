// One-pass scoring: the covariance product of a block and the scores of its
// pixels from a single read of its lines (Eq. 1 of the paper, Section
// "System Implementation / Detection Algorithm", scored with the window as
// it stood before the push: the line-based reading of Section "Discussion /
// Performance").
//
// k_onepass: one 1024-thread workgroup per (block, covariance split), as the
// covariance kernels.  A chunk is 32 samples of one line, all bands:
//  * Raw 16-bit rows are loaded straight into a two-deep LDS ring
//    (global_load_lds, 16 bytes a lane); each lane reads back only the 16
//    bytes it loaded, so the ring needs no barrier of its own.
//  * The loading lane centres its 8 samples in FP32 (mean split hi + lo,
//    the band's power-of-two scale), rounds them once to BF16 and scatters
//    them into a double-buffered operand tile laid out [sample][band]; it
//    also keeps the exact raw band sum.  Both products read this one tile:
//      - covariance: 16-band fragments with 32 samples as the contraction
//        index (8 two-byte reads per lane), lower super-tiles of 4 x 4
//        fragments per wave as in the two-pass covariance kernel;
//      - whitening: W fragments (row scale folded in) staged once in LDS,
//        and 8 consecutive bands of one sample per lane (one 16-byte read).
//    Each wave whitens one or two out-band tiles of both 16-sample groups;
//    the squares of its tile rows go to LDS and are added in wave order
//    into the score after the next barrier.
//  * One barrier per chunk: after it every wave has converted chunk c and
//    finished chunk c - 1's products; the wave then queues chunk c + 2 into
//    the ring slot chunk c came from, multiplies chunk c and converts chunk
//    c + 1, whose loads were queued one chunk earlier.
// Sample s = 8 q + t of a chunk (q the 16-byte segment) sits in operand row
// 4 t + q, and band k of row r at ((k / 8) ^ ((r / 4) & 1)) * 8 + k % 8: the
// scattered stores and both products' reads then touch distinct LDS banks.
// The covariance partials are those of the centred, scaled operand, scaled
// back by the band scales (powers of two: exact); the block's centring
// (the mean before the push) is written as its shift for the merge.  A
// block without an earlier window is centred on its shift, unscaled, and
// scores NaN.
#include "rx_dev.h"

namespace rxk {

constexpr int OPNT = 1024;                 // 16 waves
constexpr int OPW = OPNT / 64;
constexpr int OPKC = 32;                   // samples per chunk
constexpr int OPT = 17;                    // 16-band tiles: at most 272 bands
constexpr int OPROWS = 16 * OPT;
constexpr int OPCVP = OPROWS;              // operand row pitch (halfwords)
constexpr int OPFR = fr_off(OPT);          // whitening operand fragments
static_assert((2 * OPCVP) % 128 == 32, "four consecutive operand rows start in distinct bank quarters");
static_assert((2 * OPCVP) % 16 == 0, "16-byte reads of 8 bands");

__device__ __forceinline__ int cv_idx(int r, int k) {
  return r * OPCVP + ((((k >> 3) ^ ((r >> 2) & 1)) << 3) | (k & 7));
}

// NL: direct-load rounds of 16 band rows per wave and chunk (1 when the
// padded band count is at most 256, else 2; rounds past the last tile load
// the line's first word into a scratch slot, so every wave issues NL loads
// per chunk and waiting for a chunk is a fixed count).
template <int NL>
__global__ void __launch_bounds__(OPNT) k_onepass(LaunchSet ls, int Bw) {
  using M = MM<P_BF16>;
  using F = typename M::frag;
  __shared__ __attribute__((aligned(16))) uint16_t raw0[OPROWS * OPKC];
  __shared__ __attribute__((aligned(16))) uint16_t raw1[OPROWS * OPKC];
  __shared__ __attribute__((aligned(16))) uint16_t rawx[16 * OPKC];
  __shared__ __attribute__((aligned(16))) uint16_t cv0[OPKC * OPCVP];
  __shared__ __attribute__((aligned(16))) uint16_t cv1[OPKC * OPCVP];
  __shared__ __attribute__((aligned(16))) uint8_t wf[OPFR * 64 * 16];
  __shared__ float part[2][OPW][OPKC];
  __shared__ float nqh[OPROWS], nql[OPROWS], iss[OPROWS];

  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  int b = local / d.ks, split = local % d.ks;
  if (b >= d.nblk - 1) { b = d.nblk - 1; split = local - (d.nblk - 1) * d.ks; }
  const int ksb = ks_of(d, b);
  const int lines_b = blk_lines_of(d, b);
  const int nB = d.B, nBp = d.Bp, nS = d.S, T = nBp / 16;
  const int cpl = (nS + OPKC - 1) / OPKC;
  const int nch = lines_b * cpl;
  const int c0 = (int)((int64_t)nch * split / ksb), c1 = (int)((int64_t)nch * (split + 1) / ksb);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int sb = d.nblk;                               // slot: the window before the push
  const bool has_w = !causal_empty(d, b) && d.status[sb] == 0;

  // ---- per-block constants: centring, band scale; the whitening operand
  for (int k = tid; k < OPROWS; k += OPNT) {
    float mh = 0.0f, ml = 0.0f, is = 0.0f;
    if (k < nB) {
      const double m = has_w ? d.mu_snap[(int64_t)sb * nBp + k] : d.shift[(int64_t)b * nBp + k];
      mh = (float)m;
      ml = (float)(m - (double)mh);
      is = has_w ? d.iscale[(int64_t)sb * nBp + k] : 1.0f;
    }
    // the scale is a power of two: fma(v, s, -mh s) - ml s = ((v - mh) - ml) s
    nqh[k] = -(mh * is);
    nql[k] = -(ml * is);
    iss[k] = is;
  }
  if (has_w && split == 0)
    for (int k = tid; k < nBp; k += OPNT) d.shift[(int64_t)b * nBp + k] = k < nB ? d.mu_snap[(int64_t)sb * nBp + k] : 0.0;
  if (has_w) {
    const uint16_t* wl = static_cast<const uint16_t*>(d.wlp) + (int64_t)sb * nBp * Bw;
    const int nfr = fr_off(T);
    for (int it = tid; it < nfr * 64; it += OPNT) {
      const int f = it >> 6, l = it & 63;
      int i = 0;
      while (fr_off(i + 1) <= f) ++i;
      const int st = f - fr_off(i);
      const uint16_t* src = wl + (int64_t)(16 * i + (l & 15)) * Bw + 32 * st + 8 * (l >> 4);
      // BF16 keeps FP32's exponent range: the row's power-of-two output
      // scale folds into the operand exactly
      const float o = d.oscale[(int64_t)sb * nBp + 16 * i + (l & 15)];
      uint4 w = *reinterpret_cast<const uint4*>(src);
      uint32_t* q = reinterpret_cast<uint32_t*>(&w);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const float lo = __builtin_bit_cast(float, q[h] << 16) * o;
        const float hi = __builtin_bit_cast(float, q[h] & 0xffff0000u) * o;
        q[h] = (__builtin_bit_cast(uint32_t, lo) >> 16) | (__builtin_bit_cast(uint32_t, hi) & 0xffff0000u);
      }
      *reinterpret_cast<uint4*>(wf + it * 16) = w;
    }
  }
  __syncthreads();

  // ---- direct loads: round q of wave wv holds band rows 16 (wv + 16 q) + lane / 4,
  // lane % 4 the 16-byte segment; rows past the band count, segments past the
  // row end and rounds past the last tile load the chunk's first word
  const int lrow = lane >> 2, lseg = lane & 3;
  const int64_t line_bytes = 2 * (int64_t)nB * nS;
  const char* xb = static_cast<const char*>(d.x) + (int64_t)b * d.blk_lines * line_bytes;
  uint32_t off[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int r = 16 * (wv + 16 * q) + lrow;
    off[q] = (r < nB) ? 2u * ((uint32_t)r * (uint32_t)nS + 8u * (uint32_t)lseg) : 0u;
  }
  struct Pos { const char* lb; int s0; };
  auto advance = [&](Pos& p) {
    p.s0 += OPKC;
    if (p.s0 >= nS) { p.s0 = 0; p.lb += line_bytes; }
  };
  auto issue = [&](const Pos& p, uint16_t* buf) {
    const char* lb = p.lb + 2 * p.s0;
    const bool ragged = nS - p.s0 < OPKC;                       // wave-uniform
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      uint32_t o = off[q];
      if (ragged) o = (8 * lseg < nS - p.s0) ? o : 0u;
      const int round = wv + 16 * q;
      uint16_t* dst = round < OPT ? buf + round * 16 * OPKC : rawx;
      __builtin_amdgcn_global_load_lds((const void*)(lb + o), (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };

  // ---- conversion of one chunk by the lanes that loaded it; the raw sums
  // are exact in 32 bits: 8 values of at most 65535 per chunk, and the host
  // gives a split at most 8191 chunks
  uint32_t rsum[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) rsum[q] = 0u;
  auto convert = [&](int s0, const uint16_t* rb, uint16_t* cvb) {
    const int nvalid = min(OPKC, nS - s0);
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int round = wv + 16 * q;
      if (round >= OPT) continue;                               // scratch slot
      const int r = 16 * round + lrow;
      uint4 w4 = *reinterpret_cast<const uint4*>(rb + r * OPKC + 8 * lseg);
      const bool ok = r < nB && 8 * lseg < nvalid;
      if (!ok) w4 = uint4{0u, 0u, 0u, 0u};
      const float is = iss[r], qh = nqh[r], ql = nql[r];
      const uint32_t wd[4] = {w4.x, w4.y, w4.z, w4.w};
      // sample 2 h sits in operand row 8 h + lseg (band group r / 8), sample
      // 2 h + 1 in row 8 h + 4 + lseg (band group r / 8 ^ 1)
      uint16_t* e0 = cvb + cv_idx(lseg, r);
      uint16_t* e1 = cvb + cv_idx(4 + lseg, r);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        rsum[q] = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, wd[h]), u16x2{1, 1}, rsum[q], false);
        float c0v = __builtin_fmaf((float)(wd[h] & 0xffffu), is, qh) + ql;
        float c1v = __builtin_fmaf((float)(wd[h] >> 16), is, qh) + ql;
        c0v = ok ? c0v : 0.0f;
        c1v = ok ? c1v : 0.0f;
        const uint32_t pk = cvt_pack2<P_BF16>(c0v, c1v);
        e0[8 * h * OPCVP] = (uint16_t)(pk & 0xffffu);
        e1[8 * h * OPCVP] = (uint16_t)(pk >> 16);
      }
    }
  };

  // ---- covariance product: wave wv owns lower super-tile (I, J) of 4 x 4
  // fragments and multiplies the fragment rows of it that hold a stored tile
  int I = 0, J = 0;
  {
    int t = wv;
    while (t > I) { t -= I + 1; ++I; }
    J = t;
  }
  const int nsup = (nBp + 63) >> 6;
  const bool active = I < nsup;
  typename M::acc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = typename M::acc{};
  const int lr = lane & 15, lkg = lane >> 4;
  uint32_t rowm = 0;
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (64 * I + 16 * ii < nBp && 64 * J + 16 * j < nBp && (I > J || ii >= j)) rowm |= 1u << ii;
  rowm = __builtin_amdgcn_readfirstlane(rowm);
  // fragment of bands kb..kb+15 (kb a multiple of 16): lane (lr, lkg) holds
  // samples 8 lkg + t of band kb + lr, which sit in operand row 4 t + lkg;
  // even t in band group kb / 8 + lr / 8, odd t in the other of the pair.
  // kb is passed through an opaque copy so that the per-fragment addresses
  // are formed where they are used, not held for the whole loop.
  const int fb0 = cv_idx(lkg, lr), fb1 = cv_idx(4 + lkg, lr);
  auto frag_cov = [&](const uint16_t* cvb, int kb) -> F {
    asm volatile("" : "+s"(kb));
    const uint16_t* p0 = cvb + fb0 + kb;
    const uint16_t* p1 = cvb + fb1 + kb;
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 8; t += 2) {
      const uint32_t lo = p0[4 * t * OPCVP];
      const uint32_t hi = p1[4 * t * OPCVP];
      w[t / 2] = lo | (hi << 16);
    }
    return __builtin_bit_cast(F, uint4{w[0], w[1], w[2], w[3]});
  };
  auto multiply = [&](const uint16_t* cvb) {
    if (!active) return;
    F bq[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bq[j] = (64 * J + 16 * j < nBp) ? frag_cov(cvb, 64 * J + 16 * j) : F{};
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
      if ((rowm >> ii) & 1u) {
        const F a = frag_cov(cvb, 64 * I + 16 * ii);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[ii][j] = M::mma(a, bq[j], acc[ii][j]);
      }
  };

  // ---- whitening: out-band tiles i0 (and i1) of both 16-sample groups
  const int i0 = d.wrow[wv][0], i1 = d.wrow[wv][1];
  const int n = lane & 15, kg = lane >> 4;
  auto whiten = [&](const uint16_t* cvb, float* pw) {
    float dl[2] = {0.0f, 0.0f};
    if (has_w && i0 != 0xff) {
      // 8 bands 32 st + 8 kg.. of sample row 16 g + n: band group 4 st + kg,
      // swapped in pairs when (n / 4) is odd
      const uint16_t* xp = cvb + cv_idx(n, 8 * kg);
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = r ? i1 : i0;
        if (i == 0xff) break;
        typename M::acc a[2] = {typename M::acc{}, typename M::acc{}};
        const uint8_t* wp = wf + (fr_off(i) * 64 + lane) * 16;
        for (int st = 0; st <= (i >> 1); ++st) {
          const int k0 = 32 * st + 8 * kg;
          const F w = *reinterpret_cast<const F*>(wp + st * 1024);
#pragma unroll
          for (int g = 0; g < 2; ++g) {
            const F x = (k0 < nBp) ? *reinterpret_cast<const F*>(xp + 16 * g * OPCVP + 32 * st) : F{};
            a[g] = M::mma(w, x, a[g]);
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int g = 0; g < 2; ++g) dl[g] = __builtin_fmaf(a[g][e], a[g][e], dl[g]);
      }
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        dl[g] += __shfl_xor(dl[g], 16, 64);
        dl[g] += __shfl_xor(dl[g], 32, 64);
      }
    }
    if (kg == 0) {
      pw[wv * OPKC + n] = dl[0];
      pw[wv * OPKC + 16 + n] = dl[1];
    }
  };

  // ---- scores of a chunk: the waves' squares added in wave order
  float* out = static_cast<float*>(d.scores);
  const int64_t line0 = (int64_t)b * d.blk_lines;               // block's first line in the batch
  auto store_scores = [&](const float* pw, int ch) {
    if (wv != OPW - 1 || lane >= OPKC) return;
    const int line = ch / cpl;
    const int smp = (ch - line * cpl) * OPKC + 8 * (lane & 3) + (lane >> 2);
    if (smp >= nS) return;
    float v = __builtin_nanf("");
    if (has_w) {
      v = 0.0f;
#pragma unroll
      for (int w = 0; w < OPW; ++w) v += pw[w * OPKC + lane];
    }
    out[(line0 + line) * nS + smp] = v;
  };

  // ---- the chunk loop
  Pos ip;
  {
    const int line = c0 / cpl;
    ip = Pos{xb + line * line_bytes, (c0 - line * cpl) * OPKC};
  }
  int cs0 = ip.s0;                                              // first sample of the next chunk to convert
  auto conv_next = [&](const uint16_t* rb, uint16_t* cvb) {
    convert(cs0, rb, cvb);
    cs0 += OPKC;
    if (cs0 >= nS) cs0 = 0;
  };
  if (c0 < c1) {
    issue(ip, raw0);
    advance(ip);
    if (c0 + 1 < c1) {
      issue(ip, raw1);
      advance(ip);
      __builtin_amdgcn_s_waitcnt(0x0F70 | NL);
    } else {
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    conv_next(raw0, cv0);
  }
  // chunk c sits in cvc; chunk c + 1 arrives in rawn and is converted into
  // cvn; chunk c + 2 is queued into rawf (the slot chunk c came from)
  auto step = [&](int c, const uint16_t* cvc, uint16_t* cvn, const uint16_t* rawn, uint16_t* rawf, float* pc,
                  const float* pp) {
    lds_barrier();
    if (c > c0) store_scores(pp, c - 1);
    if (c + 2 < c1) {
      issue(ip, rawf);
      advance(ip);
    }
    multiply(cvc);
    whiten(cvc, pc);
    if (c + 1 < c1) {
      if (c + 2 < c1) __builtin_amdgcn_s_waitcnt(0x0F70 | NL);
      else __builtin_amdgcn_s_waitcnt(0x0F70);
      conv_next(rawn, cvn);
    }
  };
  int c = c0;
  for (; c + 1 < c1; c += 2) {
    step(c, cv0, cv1, raw1, raw0, &part[0][0][0], &part[1][0][0]);
    step(c + 1, cv1, cv0, raw0, raw1, &part[1][0][0], &part[0][0][0]);
  }
  if (c < c1) step(c, cv0, cv1, raw1, raw0, &part[0][0][0], &part[1][0][0]);
  lds_barrier();
  if (c1 > c0) store_scores(&part[(c1 - 1 - c0) & 1][0][0], c1 - 1);

  // ---- covariance partial of this split (lower tiles), scaled back by the
  // band scales, and the exact raw band sums
  const int64_t slot = (int64_t)b * d.ks + split;
  float* pout = static_cast<float*>(d.part) + slot * nBp * nBp;
  auto unscale = [&](int k) -> float { return (k < nB && iss[k] > 0.0f) ? 1.0f / iss[k] : 0.0f; };
  if (active) {
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ti = 4 * I + ii, tj = 4 * J + j;
        if (16 * ti < nBp && ti >= tj) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gi = 16 * ti + M::out_row(lkg, e), gj = 16 * tj + lr;
            pout[(int64_t)gi * nBp + gj] = acc[ii][j][e] * unscale(gi) * unscale(gj);
          }
        }
      }
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int round = wv + 16 * q;
    double t = (double)rsum[q];
    t += __shfl_xor(t, 1, 64);
    t += __shfl_xor(t, 2, 64);
    const int r = 16 * round + lrow;
    if (round < OPT && lseg == 0 && r < nBp) d.psum[slot * nBp + r] = t;
  }
}

}  // namespace rxk

// One-pass launch: ls->wg0 holds the prefix of (block, split) workgroups per
// batch; every batch has at most 272 padded bands, BF16 operands, 16-bit
// input with 16-byte aligned rows and S % 8 == 0, and its slot nblk (the
// window before the push) in place.  Bw: the whitening operand's row pitch.
extern "C" hipError_t rxk_launch_onepass(const rxk::LaunchSet* ls, int wg, int Bw, hipStream_t st) {
  using namespace rxk;
  if (wg <= 0) return hipSuccess;
  int T = 0;
  for (int i = 0; i < ls->nb; ++i) T = T > ls->d[i].Bp / 16 ? T : ls->d[i].Bp / 16;
  if (T > OPT) return hipErrorInvalidValue;
  if (T <= 16) hipLaunchKernelGGL((k_onepass<1>), dim3(wg), dim3(OPNT), 0, st, *ls, Bw);
  else hipLaunchKernelGGL((k_onepass<2>), dim3(wg), dim3(OPNT), 0, st, *ls, Bw);
  return hipGetLastError();
}
