// FP64 factorisation of the window covariance for Eq. 1 of the paper
// (Section "System Implementation / Detection Algorithm"): the score needs
// Sigma^{-1}; it is applied as delta = |W (x - mu)|^2 with W lower
// triangular and W^T W = (Sigma + lambda I)^{-1}.
//
// One workgroup per block snapshot:
//   Sigma = M2 / (N - ddof);  lambda = rho * tr(Sigma) / B;  Sigma_r = Sigma + lambda I
//   equilibration R = S Sigma_r S with S = diag(Sigma_r,kk^{-1/2})  (unit diagonal)
//   R = L L^T, W = L^{-1} S, built block-row by block-row (16 rows at a time,
//   bordering): with W_K = L_K^{-1} known for the leading K rows,
//     L21 = A21 W_K^T,  L22 L22^T = A22 - L21 L21^T,  Y = L22^{-1},
//     new rows of L^{-1}:  [ -Y L21 W_K , Y ].
//   A non-positive pivot flags the block singular (its scores become NaN).
// The whitening operand in the whitening precision is then formed with
// power-of-two scales: input band scale 2^-e_k (e_k = floor(log2 sigma_k))
// and output row scale 2^f_i chosen so each row fits the format's range.
#include "rx_dev.h"

namespace rxk {

constexpr int MAXBP = 16 * MAXT;

template <int WP>
__global__ void __launch_bounds__(NT) k_factor(LaunchSet ls, int Bw) {
  int b;
  const int bi = find_batch(ls, blockIdx.x, b);
  const BatchDesc& d = ls.d[bi];
  const int B = d.B, Bp = d.Bp;
  const int64_t bp2 = (int64_t)Bp * Bp;
  double* R = d.m2_snap + b * bp2;
  double* W = d.w64 + b * bp2;
  double* WT = d.wt64 + b * bp2;
  __shared__ double A[16 * MAXBP];   // A21, then X = Y L21
  __shared__ double L[16 * MAXBP];   // L21
  __shared__ double sc[MAXBP];       // equilibration scale
  __shared__ double T22[16][17];
  __shared__ double Y[16][17];
  __shared__ double red[NT / 64];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double N = d.n_snap[b];

  if (d.rho == 0.0 && N <= (double)B) {       // window too small: Sigma is singular
    if (tid == 0) d.status[b] = 2;
    return;
  }
  const double den = N - (double)d.ddof;
  if (tid == 0) flag = 0;

  // ---- trace and ridge
  double tr = 0.0;
  for (int k = tid; k < B; k += NT) tr += R[(int64_t)k * Bp + k];
  tr = wave_sum(tr);
  if (lane == 0) red[wv] = tr;
  __syncthreads();
  tr = 0.0;
  for (int i = 0; i < NT / 64; ++i) tr += red[i];
  const double lam = d.rho * (tr / den) / (double)B;
  for (int k = tid; k < Bp; k += NT) {
    double v = 1.0;
    if (k < B) {
      v = R[(int64_t)k * Bp + k] / den + lam;
      if (!(v > 0.0) || !(v < INFINITY)) flag = 1;
    }
    sc[k] = 1.0 / sqrt(v);
  }
  __syncthreads();
  if (flag) {
    if (tid == 0) { d.status[b] = 1; atomicAdd(d.nsing, 1u); }
    return;
  }
  // ---- equilibrate in place (lower triangle); padding becomes identity
  for (int64_t idx = tid; idx < bp2; idx += NT) {
    const int i = (int)(idx / Bp), j = (int)(idx % Bp);
    if (j > i) continue;
    double v;
    if (i < B && j < B) v = (i == j) ? (R[idx] / den + lam) * sc[i] * sc[i] : (R[idx] / den) * sc[i] * sc[j];
    else v = (i == j) ? 1.0 : 0.0;
    R[idx] = v;
  }
  __syncthreads();

  // ---- bordered blocked inverse Cholesky
  for (int K = 0; K < Bp; K += 16) {
    for (int idx = tid; idx < 16 * K; idx += NT) {
      const int r = idx / K, t = idx % K;
      A[r * MAXBP + t] = R[(int64_t)(K + r) * Bp + t];
    }
    {
      const int r = tid >> 4, q = tid & 15;
      T22[r][q] = (q <= r) ? R[(int64_t)(K + r) * Bp + K + q] : R[(int64_t)(K + q) * Bp + K + r];
    }
    __syncthreads();
    // L21 = A21 W_K^T  (column c of L21 needs row c of W_K, i.e. column c of WT)
    for (int c = tid; c < K; c += NT) {
      double acc[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.0;
      for (int t = 0; t <= c; ++t) {
        const double w = WT[(int64_t)t * Bp + c];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] += A[r * MAXBP + t] * w;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) L[r * MAXBP + c] = acc[r];
    }
    __syncthreads();
    {
      const int r = tid >> 4, q = tid & 15;
      double s = T22[r][q];
      for (int c = 0; c < K; ++c) s -= L[r * MAXBP + c] * L[q * MAXBP + c];
      __syncthreads();
      T22[r][q] = s;
    }
    __syncthreads();
    // 16x16 Cholesky in wave 0: lane = (row i, column group cg of 4)
    if (wv == 0) {
      const int i = lane & 15, cg = lane >> 4;
      double v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = T22[i][4 * cg + e];
      bool bad = false;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int je = j & 3, jg = j >> 2;
        const double piv = __shfl(v[je], j + 16 * jg, 64);
        bad |= !(piv > 0.0);
        const double dd = sqrt(piv);
        const double lij = __shfl(v[je], i + 16 * jg, 64) / dd;
        double lkj[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) lkj[e] = __shfl(v[je], (4 * cg + e) + 16 * jg, 64) / dd;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 4 * cg + e;
          if (k > j && i >= k) v[e] -= lij * lkj[e];
        }
        if (cg == jg) v[je] = (i > j) ? lij : (i == j ? dd : 0.0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) T22[i][4 * cg + e] = v[e];
      if (lane == 0 && bad) flag = 1;
    }
    __syncthreads();
    if (flag) break;
    if (tid < 16) {                 // Y = L22^{-1}, one column per thread
      const int q = tid;
      double y[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double s = (i == q) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) s -= T22[i][k] * y[k];
        y[i] = (i >= q) ? s / T22[i][i] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Y[i][q] = y[i];
    }
    __syncthreads();
    // X = Y L21 (overwrites A21)
    for (int c = tid; c < K; c += NT) {
      double l[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) l[q] = L[q * MAXBP + c];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double x = 0.0;
#pragma unroll
        for (int q = 0; q <= r; ++q) x += Y[r][q] * l[q];
        A[r * MAXBP + c] = x;
      }
    }
    __syncthreads();
    // new rows K..K+15 of L^{-1} (full width) and their transpose
    for (int t = tid; t < Bp; t += NT) {
      double acc[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.0;
      if (t < K) {
        // all lanes of a wave walk the same c, so W row c is read coalesced
        for (int c = t & ~63; c < K; ++c) {
          const double w = (c >= t) ? W[(int64_t)c * Bp + t] : 0.0;
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[r] -= A[r * MAXBP + c] * w;
        }
      } else if (t < K + 16) {
        const int q = t - K;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = (q <= r) ? Y[r][q] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        W[(int64_t)(K + r) * Bp + t] = acc[r];
        WT[(int64_t)t * Bp + K + r] = acc[r];
      }
    }
    __syncthreads();
  }
  if (flag) {
    if (tid == 0) { d.status[b] = 1; atomicAdd(d.nsing, 1u); }
    return;
  }

  // ---- W = L^{-1} S (FP64), padding rows/columns zeroed
  for (int64_t idx = tid; idx < bp2; idx += NT) {
    const int i = (int)(idx / Bp), j = (int)(idx % Bp);
    W[idx] = (i < B && j < B && j <= i) ? W[idx] * sc[j] : 0.0;
  }
  __syncthreads();

  // ---- whitening operand in the whitening precision
  if constexpr (WP == P_F32) {
    float* wl = static_cast<float*>(d.wlp) + (int64_t)b * Bp * Bw;
    for (int64_t idx = tid; idx < (int64_t)Bp * Bw; idx += NT) {
      const int i = (int)(idx / Bw), j = (int)(idx % Bw);
      wl[idx] = (j < Bp) ? (float)W[(int64_t)i * Bp + j] : 0.0f;
    }
    for (int k = tid; k < Bp; k += NT) {
      d.iscale[(int64_t)b * Bp + k] = 1.0f;
      d.oscale[(int64_t)b * Bp + k] = 1.0f;
    }
  } else if constexpr (WP != P_F64) {
    using S = typename MM<WP>::storage;
    S* wl = static_cast<S*>(d.wlp) + (int64_t)b * Bp * Bw;
    constexpr int top = (WP == P_FP8) ? 7 : 14;     // row max lands in [2^top, 2^(top+1))
    __shared__ int ek[MAXBP];
    __shared__ int fi[MAXBP];
    for (int k = tid; k < Bp; k += NT) {
      const int e = (k < B) ? ilogb(1.0 / sc[k]) : 0;   // 2^e <= sigma_k < 2^(e+1)
      ek[k] = e;
      d.iscale[(int64_t)b * Bp + k] = (float)ldexp(1.0, -e);
    }
    __syncthreads();
    for (int i = tid; i < Bp; i += NT) {
      double m = 0.0;
      for (int j = 0; j <= i && j < B; ++j) m = fmax(m, fabs(ldexp(W[(int64_t)i * Bp + j], ek[j])));
      const int f = (m > 0.0) ? ilogb(m) - top : 0;
      fi[i] = f;
      d.oscale[(int64_t)b * Bp + i] = (float)ldexp(1.0, f);
    }
    __syncthreads();
    for (int64_t idx = tid; idx < (int64_t)Bp * Bw; idx += NT) {
      const int i = (int)(idx / Bw), j = (int)(idx % Bw);
      float v = 0.0f;
      if (j < Bp) v = (float)ldexp(W[(int64_t)i * Bp + j], ek[j] - fi[i]);
      wl[idx] = to_storage<WP>(v);
    }
  }
  if (tid == 0) d.status[b] = 0;
}

}  // namespace rxk

extern "C" hipError_t rxk_launch_factor(int wprec, const rxk::LaunchSet* ls, int wg, int Bw,
                                        hipStream_t st) {
  using namespace rxk;
  if (wg <= 0) return hipSuccess;
  switch (wprec) {
    case P_F64: hipLaunchKernelGGL((k_factor<P_F64>), dim3(wg), dim3(NT), 0, st, *ls, Bw); break;
    case P_F32: hipLaunchKernelGGL((k_factor<P_F32>), dim3(wg), dim3(NT), 0, st, *ls, Bw); break;
    case P_BF16: hipLaunchKernelGGL((k_factor<P_BF16>), dim3(wg), dim3(NT), 0, st, *ls, Bw); break;
    case P_F16: hipLaunchKernelGGL((k_factor<P_F16>), dim3(wg), dim3(NT), 0, st, *ls, Bw); break;
    case P_FP8: hipLaunchKernelGGL((k_factor<P_FP8>), dim3(wg), dim3(NT), 0, st, *ls, Bw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
