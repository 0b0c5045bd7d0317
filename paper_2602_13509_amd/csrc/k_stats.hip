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
//   k_merge  -- fixed-order FP64 reduction of the partials, exact shift
//               correction M2_b = C - n e e^T (e = m_b - c), then the
//               pairwise (Chan-Golub-LeVeque) update of the window
//               (N, S1, M2), snapshotting the window after every block.
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

  // ---- write the partial super-tile (row-major 64x64)
  const int64_t slot = (int64_t)b * d.ks + split;
  if (!skip) {
    C* out = static_cast<C*>(d.part) + (slot * d.nsup + sup) * (SUP * SUP);
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = 32 * wr + 16 * ti + M::out_row(lane >> 4, j);
          const int cc = 32 * wc + 16 * tj + lr;
          out[rr * SUP + cc] = acc[ti][tj][j];
        }
  }
  // ---- raw band sums (diagonal super-tiles cover every band exactly once)
  if (diag) {
    for (int o = 1; o < tpr; o <<= 1) rawsum += __shfl_xor(rawsum, o, 64);
    if ((tid % tpr) == 0 && band < d.Bp) d.psum[slot * d.Bp + band] = bvalid ? rawsum : 0.0;
  }
}

// ---------------------------------------------------------------------------- merge
// One workgroup per lower super-tile; it walks the batch's blocks in order.
template <typename PT>
__global__ void __launch_bounds__(NT) k_merge(LaunchSet ls) {
  int sup;
  const int bi = find_batch(ls, blockIdx.x, sup);
  const BatchDesc& d = ls.d[bi];
  int I, J;
  sup_ij(sup, I, J);
  const bool diag = (I == J);
  __shared__ double s1w[128];   // window raw sums: rows 0..63 = bands 64I.., 64..127 = bands 64J..
  __shared__ double ev[128];    // block mean minus shift
  __shared__ double dv[128];    // block mean minus window mean (before the block)
  const int tid = threadIdx.x;
  const int64_t bp2 = (int64_t)d.Bp * d.Bp;

  double m2[16];
  int gi[16], gj[16];
  bool val[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + NT * q;
    gi[q] = 64 * I + idx / 64;
    gj[q] = 64 * J + idx % 64;
    val[q] = gi[q] < d.B && gj[q] < d.B && gi[q] >= gj[q];
    m2[q] = val[q] ? d.m2_in[(int64_t)gi[q] * d.Bp + gj[q]] : 0.0;
  }
  const int myband = tid < 64 ? 64 * I + tid : 64 * J + (tid - 64);
  if (tid < 128) s1w[tid] = (myband < d.B) ? d.s1_in[myband] : 0.0;
  double N = (double)d.n_in;
  __syncthreads();

  for (int b = 0; b < d.nblk; ++b) {
    const double nb = (double)blk_lines_of(d, b) * d.S;
    const int ksb = ks_of(d, b);
    const bool reset = (d.reset_bits >> b) & 1ull;
    if (reset) {
      N = 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) m2[q] = 0.0;
    }
    if (tid < 128) {
      double sb = 0.0;
      if (myband < d.B)
        for (int s = 0; s < ksb; ++s) sb += d.psum[((int64_t)b * d.ks + s) * d.Bp + myband];
      const double sw = reset ? 0.0 : s1w[tid];
      const double mb = sb / nb;
      ev[tid] = (myband < d.B) ? mb - d.shift[(int64_t)b * d.Bp + myband] : 0.0;
      dv[tid] = (myband < d.B && N > 0.0) ? mb - sw / N : 0.0;
      s1w[tid] = sw + sb;
    }
    __syncthreads();
    const double coef = N > 0.0 ? N * nb / (N + nb) : 0.0;
    const PT* pb = static_cast<const PT*>(d.part) + ((int64_t)b * d.ks * d.nsup + sup) * (SUP * SUP);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (!val[q]) continue;
      const int idx = tid + NT * q;
      double c = 0.0;
      for (int s = 0; s < ksb; ++s) c += (double)pb[(int64_t)s * d.nsup * (SUP * SUP) + idx];
      const int ri = idx / 64, cj = idx % 64 + (diag ? 0 : 64);
      const double m2b = c - nb * ev[ri] * ev[cj];
      m2[q] = (N > 0.0) ? m2[q] + m2b + coef * dv[ri] * dv[cj] : m2b;
      d.m2_snap[b * bp2 + (int64_t)gi[q] * d.Bp + gj[q]] = m2[q];
    }
    N += nb;
    if (diag && tid < 64 && myband < d.Bp)
      d.mu_snap[(int64_t)b * d.Bp + myband] = (myband < d.B) ? s1w[tid] / N : 0.0;
    if (sup == 0 && tid == 0) d.n_snap[b] = N;
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (val[q]) d.m2_out[(int64_t)gi[q] * d.Bp + gj[q]] = m2[q];
  if (diag && tid < 64 && myband < d.Bp) d.s1_out[myband] = s1w[tid];
}

}  // namespace rxk

// Host entry used by the runtime: one LaunchSet per kernel phase.  Workgroup
// prefixes differ per kernel, so the runtime passes three copies.
extern "C" hipError_t rxk_launch_stats(int in_type, int prec, const rxk::LaunchSet* ls_shift,
                                       const rxk::LaunchSet* ls_syrk, const rxk::LaunchSet* ls_merge,
                                       int wg_shift, int wg_syrk, int wg_merge, hipStream_t st) {
  using namespace rxk;
#define RXK_CASE(INV, PV)                                                                 \
  if (in_type == INV && prec == PV) {                                                     \
    if (wg_shift > 0) hipLaunchKernelGGL((k_shift<INV, PV>), dim3(wg_shift), dim3(NT), 0, st, *ls_shift); \
    if (wg_syrk > 0) hipLaunchKernelGGL((k_syrk<INV, PV>), dim3(wg_syrk), dim3(NT), 0, st, *ls_syrk);     \
    if (wg_merge > 0) {                                                                   \
      if (PV == P_F64) hipLaunchKernelGGL((k_merge<double>), dim3(wg_merge), dim3(NT), 0, st, *ls_merge); \
      else hipLaunchKernelGGL((k_merge<float>), dim3(wg_merge), dim3(NT), 0, st, *ls_merge);              \
    }                                                                                     \
    return hipGetLastError();                                                             \
  }
  RXK_CASE(IN_U16, P_F64) RXK_CASE(IN_U16, P_F32) RXK_CASE(IN_U16, P_BF16) RXK_CASE(IN_U16, P_F16)
  RXK_CASE(IN_F32, P_F64) RXK_CASE(IN_F32, P_F32) RXK_CASE(IN_F32, P_BF16) RXK_CASE(IN_F32, P_F16)
  RXK_CASE(IN_F64, P_F64) RXK_CASE(IN_F64, P_F32) RXK_CASE(IN_F64, P_BF16) RXK_CASE(IN_F64, P_F16)
#undef RXK_CASE
  return hipErrorInvalidValue;
}
