// Streaming window statistics: band mean and scatter matrix of every pixel
// in the window (paper, Section "System Implementation / Detection
// Algorithm": mean per band, covariance over all pixels of the set).
//
// Per block of lines:
//   k_shift  -- centring shift c = mean of the block's first line per band
//               (rounded to FP32 on mixed paths, so it is exact in both the
//               FP32 centring and the FP64 merge).
//   k_syrk   -- C = sum_p (x_p - c)(x_p - c)^T on matrix cores, lower 64x64
//               super-tiles x split-K over pixel chunks, FP32 (or FP64)
//               partials; diagonal super-tiles also emit exact raw band sums.
//   k_merge_vec / k_merge_mat -- fixed-order FP64 reduction of the
//               partials, exact shift correction M2_b = C - n e e^T
//               (e = m_b - c), then the pairwise (Chan-Golub-LeVeque) update
//               of the window (N, S1, M2), snapshotting it after every block.
#include "rx_dev.h"

namespace rxk {

// ---------------------------------------------------------------------------- shift
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
    for (int i = lane; i < d.S; i += 64) s += to_d(row[i]);
    s = wave_sum(s);
    c = s / (double)d.S;
    if (P != P_F64) c = (double)(float)c;
  }
  if (lane == 0) d.shift[(int64_t)b * d.Bp + band] = c;
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
      for (int sg = 0; sg < segs; ++sg) {
        const int k0 = 8 * (seg0 + sg);
        T v[8];
        if (bvalid && d.vec_ok && k0 + 8 <= nvalid) {
          load8(row + k0, v);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = (bvalid && k0 + j < nvalid) ? row[k0 + j] : T(0);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ok = bvalid && (k0 + j < nvalid);
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

// ---------------------------------------------------------------------------- merge
// Vector part, one workgroup per batch, sequential over its blocks: per band
// the exact raw block sum (fixed-order sum over splits), block mean m_b,
// e = m_b - shift, d = m_b - window mean before the block, window sums after
// the block; per block the pairwise-update weight N n_b / (N + n_b) (0 when
// the window was empty: the block's scatter replaces the window's).
__global__ void __launch_bounds__(NT) k_merge_vec(LaunchSet ls) {
  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  for (int k = threadIdx.x; k < d.Bp; k += NT) {
    double N = (double)d.n_in;
    double s1 = (k < d.B) ? d.s1_in[k] : 0.0;
    for (int b = 0; b < d.nblk; ++b) {
      const double nb = (double)blk_lines_of(d, b) * d.S;
      const int ksb = ks_of(d, b);
      if ((d.reset_bits >> b) & 1ull) { N = 0.0; s1 = 0.0; }
      double sb = 0.0;
      if (k < d.B)
        for (int s = 0; s < ksb; ++s) sb += d.psum[((int64_t)b * d.ks + s) * d.Bp + k];
      const double mb = sb / nb;
      const int64_t o = (int64_t)b * d.Bp + k;
      d.ev[o] = (k < d.B) ? mb - d.shift[o] : 0.0;
      d.dv[o] = (k < d.B && N > 0.0) ? mb - s1 / N : 0.0;
      if (k == 0) d.coef[b] = N > 0.0 ? N * nb / (N + nb) : 0.0;
      s1 += sb;
      N += nb;
      d.mu_snap[o] = (k < d.B) ? s1 / N : 0.0;
      if (k == 0) d.n_snap[b] = N;
    }
    d.s1_out[k] = (k < d.B) ? s1 : 0.0;
  }
}

// Matrix part, one workgroup per lower 16x16 tile, one element per thread:
// C_b = fixed-order FP64 sum of the split partials, M2_b = C_b - n_b e e^T
// (exact shift correction), then the pairwise update
// M2 <- M2 + M2_b + w d d^T  (or M2 <- M2_b for an empty window), with the
// window's scatter matrix snapshotted after every block.
template <typename PT>
__global__ void __launch_bounds__(NT) k_merge_mat(LaunchSet ls) {
  int t;
  const int bi = find_batch(ls, blockIdx.x, t);
  const BatchDesc& d = ls.d[bi];
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int gi = 16 * ti + (threadIdx.x >> 4), gj = 16 * tj + (threadIdx.x & 15);
  if (!(gi < d.B && gj < d.B && gi >= gj)) return;
  const int64_t bp2 = (int64_t)d.Bp * d.Bp, e = (int64_t)gi * d.Bp + gj;
  double m2 = d.m2_in[e];
  for (int b = 0; b < d.nblk; ++b) {
    const double nb = (double)blk_lines_of(d, b) * d.S;
    const int ksb = ks_of(d, b);
    if ((d.reset_bits >> b) & 1ull) m2 = 0.0;
    const PT* pb = static_cast<const PT*>(d.part) + (int64_t)b * d.ks * bp2 + e;
    double c = 0.0;
    for (int s = 0; s < ksb; ++s) c += (double)pb[s * bp2];
    const int64_t o = (int64_t)b * d.Bp;
    const double m2b = c - nb * d.ev[o + gi] * d.ev[o + gj];
    const double w = d.coef[b];
    m2 = (w > 0.0) ? m2 + m2b + w * d.dv[o + gi] * d.dv[o + gj] : m2b;
    d.m2_snap[b * bp2 + e] = m2;
  }
  d.m2_out[e] = m2;
}

}  // namespace rxk

// Host entry used by the runtime: phase 0 centring shift, 1 covariance
// product, 2 merge (vector then matrix part).  wg: workgroups of the phase
// (for phase 2: wg = vector workgroups, wg2 = matrix workgroups).
extern "C" hipError_t rxk_launch_stats(int in_type, int prec, int phase, const rxk::LaunchSet* ls, int wg,
                                       const rxk::LaunchSet* ls2, int wg2, hipStream_t st) {
  using namespace rxk;
  if (phase == 2) {
    if (wg > 0) hipLaunchKernelGGL(k_merge_vec, dim3(wg), dim3(NT), 0, st, *ls);
    if (wg2 > 0) {
      if (prec == P_F64) hipLaunchKernelGGL((k_merge_mat<double>), dim3(wg2), dim3(NT), 0, st, *ls2);
      else hipLaunchKernelGGL((k_merge_mat<float>), dim3(wg2), dim3(NT), 0, st, *ls2);
    }
    return hipGetLastError();
  }
  if (wg <= 0) return hipSuccess;
#define RXK_CASE(INV, PV)                                                                      \
  if (in_type == INV && prec == PV) {                                                          \
    if (phase == 0) hipLaunchKernelGGL((k_shift<INV, PV>), dim3(wg), dim3(NT), 0, st, *ls);    \
    else hipLaunchKernelGGL((k_syrk<INV, PV>), dim3(wg), dim3(NT), 0, st, *ls);                \
    return hipGetLastError();                                                                  \
  }
  RXK_CASE(IN_U16, P_F64) RXK_CASE(IN_U16, P_F32) RXK_CASE(IN_U16, P_BF16) RXK_CASE(IN_U16, P_F16)
  RXK_CASE(IN_F32, P_F64) RXK_CASE(IN_F32, P_F32) RXK_CASE(IN_F32, P_BF16) RXK_CASE(IN_F32, P_F16)
  RXK_CASE(IN_F64, P_F64) RXK_CASE(IN_F64, P_F32) RXK_CASE(IN_F64, P_BF16) RXK_CASE(IN_F64, P_F16)
#undef RXK_CASE
  return hipErrorInvalidValue;
}
