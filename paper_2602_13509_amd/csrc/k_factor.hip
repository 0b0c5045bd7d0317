// FP64 factorisation of the window covariance for Eq. 1 of the paper
// (Section "System Implementation / Detection Algorithm"): the score needs
// Sigma^{-1}; it is applied as delta = |W (x - mu)|^2 with W lower
// triangular and W^T W = (Sigma + lambda I)^{-1}.
//
// One 512-thread workgroup per block snapshot:
//   Sigma = M2 / (N - ddof);  lambda = rho * tr(Sigma) / B;  Sigma_r = Sigma + lambda I
//   equilibration R = S Sigma_r S with S = diag(Sigma_r,kk^{-1/2})  (unit diagonal)
//   R = L L^T and W = L^{-1} S in one right-looking sweep over 16x16 tiles
//   held in registers, FP64 matrix-core products (details below).
//   A non-positive pivot flags the block singular (its scores become NaN).
// The whitening operand in the whitening precision is then formed with
// power-of-two scales: input band scale 2^-e_k (e_k = floor(log2 sigma_k))
// and output row scale 2^f_i chosen so each row fits the format's range.
#include "rx_dev.h"

namespace rxk {

constexpr int MAXBP = 16 * MAXT;
constexpr int FNW = 8;                  // waves per factor workgroup (2 per SIMD: 256 registers each)
constexpr int FNT = 64 * FNW;           // threads per factor workgroup
// lower tiles per wave: a template argument sized to the band count; up to
// 20 tiles (B <= 272) the tiles and the step's temporaries fit in registers
constexpr int ftpw_for(int T) { return (T * (T + 1) / 2 + FNW - 1) / FNW; }
constexpr int FTS = 16 * 17;            // LDS tile: 16 rows, pitch 17 doubles (bank-conflict free)

__device__ __forceinline__ double readlane_d(double x, int l) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = __builtin_amdgcn_readlane(v.x, l);
  v.y = __builtin_amdgcn_readlane(v.y, l);
  return __builtin_bit_cast(double, v);
}

template <int WP, int FTPW>
__global__ void __launch_bounds__(FNT) k_factor(LaunchSet ls) {
  int b;
  const int bi = find_batch(ls, blockIdx.x, b);
  const BatchDesc& d = ls.d[bi];
  const int B = d.B, Bp = d.Bp;
  const int64_t bp2 = (int64_t)Bp * Bp;
  const double* R = d.m2_snap + b * bp2;
  double* W = d.w64 + b * bp2;
  __shared__ double lcol[MAXT * FTS];   // pivot column: R_ik, then L_ik
  __shared__ double prow[MAXT * FTS];   // pivot row: E_kj, then W_kj; Y at k
  __shared__ double ybuf[FTS];          // Y = L_kk^{-1}
  __shared__ double sc[MAXBP];          // equilibration scale
  __shared__ double T22[16][17];
  __shared__ double red[FNW];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const double N = d.n_snap[b];

  if (d.rho == 0.0 && N <= (double)B) {       // window too small: Sigma is singular
    if (tid == 0) d.status[b] = 2;
    return;
  }
  const double den = N - (double)d.ddof;
  if (tid == 0) flag = 0;

  // ---- trace and ridge
  double tr = 0.0;
  for (int k = tid; k < B; k += FNT) tr += R[(int64_t)k * Bp + k];
  tr = wave_sum(tr);
  if (lane == 0) red[wv] = tr;
  __syncthreads();
  tr = 0.0;
  for (int i = 0; i < FNW; ++i) tr += red[i];
  const double lam = d.rho * (tr / den) / (double)B;
  for (int k = tid; k < Bp; k += FNT) {
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

  // ---- one right-looking sweep over 16x16 tiles held in registers:
  // every lower tile (i, j) of R lives in one wave (cyclic ownership).  At
  // step k the diagonal tile is factored (L_kk, Y = L_kk^{-1}); the pivot
  // column becomes L_ik = R_ik Y^T; the pivot row of the eliminated identity
  // becomes final rows of W = L^{-1}: W_kj = Y E_kj (W_kk = Y); every tile
  // below row k is then updated with one 16x16x16 product:
  //   j > k: R_ij -= L_ik L_jk^T     j == k: E_ik = -L_ik Y     j < k: E_ij -= L_ik W_kj
  // so each tile holds R, then L (pivot column), then E, then W.
  const int T = Bp / 16, ntiles = T * (T + 1) / 2;
  const int lr = lane & 15, lg = lane >> 4;
  // LDS tiles are row-major with pitch 17: element (r, c) at r * 17 + c.
  // offA: this lane's element of an A-operand (or transposed B) read, (lr, 4q + lg);
  // offB: of a B-operand read / accumulator write, (lg + 4q, lr).  Per-step reads
  // use these with immediate offsets (4q, 68q).
  const int offA0 = lr * 17 + lg, offB0 = lg * 17 + lr;
  const double rden = 1.0 / den;
  f64x4 tl[FTPW];
  int ti[FTPW], tj[FTPW];
#pragma unroll
  for (int s = 0; s < FTPW; ++s) {
    const int t = s * FNW + wv;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    ti[s] = __builtin_amdgcn_readfirstlane((t < ntiles) ? i : -1);
    tj[s] = __builtin_amdgcn_readfirstlane((t < ntiles) ? t - i * (i + 1) / 2 : -1);
    tl[s] = f64x4{0.0, 0.0, 0.0, 0.0};
    if (ti[s] >= 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // branch-free: every lane loads a valid address, padding is selected away
        const int row = 16 * ti[s] + lg + 4 * r, col = 16 * tj[s] + lr;
        const bool in = (row < B) && (col < B);
        const int hi = in ? (row >= col ? row : col) : 0, lo = in ? (row >= col ? col : row) : 0;
        double v = R[(int64_t)hi * Bp + lo] * rden + ((row == col) ? lam : 0.0);
        v *= sc[row] * sc[col];
        v = in ? v : ((row == col) ? 1.0 : 0.0);
        tl[s][r] = v;
      }
    }
    if ((s & 3) == 3) __builtin_amdgcn_sched_barrier(0);   // at most four tiles of loads in flight
  }
  for (int k = 0; k < T; ++k) {
    int offA = offA0, offB = offB0;
    asm volatile("" : "+v"(offA), "+v"(offB));   // keep derived addresses inside the step
    // stage the tiles this step reads from other waves
#pragma unroll
    for (int s = 0; s < FTPW; ++s) {
      double* dst = nullptr;
      if (ti[s] == k && tj[s] == k) dst = &T22[0][0];
      else if (tj[s] == k && ti[s] > k) dst = lcol + ti[s] * FTS;
      else if (ti[s] == k && tj[s] >= 0 && tj[s] < k) dst = prow + tj[s] * FTS;
      if (dst) {
        double* p = dst + offB;
#pragma unroll
        for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // 16x16 Cholesky of the diagonal tile and Y = L_kk^{-1} together, in wave 0:
    // lane = (row i, column group cg of 4) holds S[i][4cg..4cg+3] and the
    // eliminated identity E[i][4cg..4cg+3].  Column j: pivot d = sqrt(S[j][j]),
    // L[i][j] = S[i][j] / d, Y[j][.] = E[j][.] / d, then S[i][k] -= L[i][j] L[k][j]
    // (j < k <= i) and E[i][.] -= L[i][j] Y[j][.] (i > j).
    if (wv == 0) {
      int i = lane & 15, cg = lane >> 4;
      asm volatile("" : "+v"(i), "+v"(cg));    // shuffle addresses are formed per step, not hoisted
      double v[4], y[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = T22[i][4 * cg + e];
        y[e] = (i == 4 * cg + e) ? 1.0 : 0.0;
      }
      bool bad = false;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int je = j & 3, jg = j >> 2;
        const double piv = readlane_d(v[je], j + 16 * jg);
        bad |= !(piv > 0.0);
        const double rd = 1.0 / sqrt(piv);
        const double lij = __shfl(v[je], i + 16 * jg, 64) * rd;
        double lkj[4], yj[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          lkj[e] = __shfl(v[je], (4 * cg + e) + 16 * jg, 64) * rd;
          yj[e] = __shfl(y[e], j + 16 * cg, 64) * rd;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kk = 4 * cg + e;
          if (kk > j && i >= kk) v[e] -= lij * lkj[e];
          y[e] = (i == j) ? yj[e] : ((i > j) ? y[e] - lij * yj[e] : y[e]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) ybuf[i * 17 + 4 * cg + e] = y[e];
      if (lane == 0 && bad) flag = 1;
    }
    __syncthreads();
    if (flag) break;
    // pivot column L_ik = R_ik Y^T, pivot row W_kj = Y E_kj, W_kk = Y
#pragma unroll
    for (int s = 0; s < FTPW; ++s) {
      if (tj[s] == k && ti[s] > k) {
        double* lc = lcol + ti[s] * FTS;
        const double* la = lc + offA;
        const double* yb = ybuf + offA;
        tl[s] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
          tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(la[4 * q4], yb[4 * q4], tl[s], 0, 0, 0);
        double* p = lc + offB;
#pragma unroll
        for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
      } else if (ti[s] == k && tj[s] >= 0 && tj[s] < k) {
        double* pr = prow + tj[s] * FTS;
        const double* ya = ybuf + offA;
        const double* pb = pr + offB;
        tl[s] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
          tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[4 * q4], pb[68 * q4], tl[s], 0, 0, 0);
        double* p = pr + offB;
#pragma unroll
        for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
      } else if (ti[s] == k && tj[s] == k) {
        const double* yb = ybuf + offB;
        double* p = prow + k * FTS + offB;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tl[s][r] = yb[68 * r];
          p[68 * r] = tl[s][r];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // update every tile below row k
#pragma unroll
    for (int s = 0; s < FTPW; ++s) {
      if (ti[s] > k) {
        const double* la = lcol + ti[s] * FTS + offA;
        if (tj[s] == k) tl[s] = f64x4{0.0, 0.0, 0.0, 0.0};
        if (tj[s] > k) {
          const double* lb = lcol + tj[s] * FTS + offA;
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4)
            tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-la[4 * q4], lb[4 * q4], tl[s], 0, 0, 0);
        } else {
          const double* pb = prow + tj[s] * FTS + offB;
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4)
            tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-la[4 * q4], pb[68 * q4], tl[s], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (flag) {
    if (tid == 0) { d.status[b] = 1; atomicAdd(d.nsing, 1u); }
    return;
  }
  // ---- W = L^{-1} S (FP64, row-major) and the whitening operand in the whitening
  // precision, from the tiles.  Tiles above the diagonal are never written:
  // those parts of both buffers are zeroed once when they are allocated.
  constexpr bool LP = (WP == P_BF16 || WP == P_F16 || WP == P_FP8);
  constexpr int top = (WP == P_FP8) ? 7 : 14;     // scaled row maximum lands in [2^top, 2^(top+1))
  __shared__ int ek[MAXBP];
  __shared__ int fi[MAXBP];
  for (int k = tid; k < Bp; k += FNT) ek[k] = (LP && k < B) ? ilogb(1.0 / sc[k]) : 0;   // 2^e <= sigma_k < 2^(e+1)
#pragma unroll
  for (int s = 0; s < FTPW; ++s) {
    if (ti[s] >= 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti[s] + lg + 4 * r, col = 16 * tj[s] + lr;
        const double v = (row < B && col < B && col <= row) ? tl[s][r] * sc[col] : 0.0;
        tl[s][r] = v;
        W[(int64_t)row * Bp + col] = v;
      }
    }
  }
  if constexpr (WP != P_F64) {
    using S = typename MM<WP>::storage;
    const int Bw = 32 * ((Bp + 31) / 32);           // operand row pitch of this batch
    S* wl = static_cast<S*>(d.wlp) + (int64_t)b * Bp * Bw;
    __syncthreads();
    constexpr int NCC = (MAXBP + 63) / 64;        // 64-column chunks of a row
    if constexpr (LP) {
      // row maxima of |W_ij 2^e_j|: one wave per four rows, lanes over the
      // columns, every load of the four rows independent (the maximum is exact
      // in any order)
      for (int i0 = 4 * wv; i0 < Bp; i0 += 4 * FNW) {
        double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NCC; ++c) {
          const int j = lane + 64 * c;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = i0 + q;
            if (j <= i && j < B) m[q] = fmax(m[q], fabs(ldexp(W[(int64_t)i * Bp + j], ek[j])));
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          for (int o = 32; o > 0; o >>= 1) m[q] = fmax(m[q], __shfl_xor(m[q], o, 64));
          if (lane == 0) fi[i0 + q] = (m[q] > 0.0) ? ilogb(m[q]) - top : 0;
        }
      }
    } else {
      for (int k = tid; k < Bp; k += FNT) fi[k] = 0;
    }
    __syncthreads();
    for (int k = tid; k < Bp; k += FNT) {
      d.iscale[(int64_t)b * Bp + k] = (float)ldexp(1.0, -ek[k]);
      d.oscale[(int64_t)b * Bp + k] = (float)ldexp(1.0, fi[k]);
    }
    // one wave per four rows, lanes over the columns of each row's lower tiles
    for (int i0 = 4 * wv; i0 < Bp; i0 += 4 * FNW) {
#pragma unroll
      for (int c = 0; c < NCC; ++c) {
        const int j = lane + 64 * c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + q;
          if (j < 16 * (i / 16 + 1))
            wl[(int64_t)i * Bw + j] = to_storage<WP>((float)ldexp(W[(int64_t)i * Bp + j], ek[j] - fi[i]));
        }
      }
    }
  }
  if (tid == 0) d.status[b] = 0;
}

}  // namespace rxk

template <int WP>
static void launch_factor_t(const rxk::LaunchSet* ls, int wg, hipStream_t st) {
  using namespace rxk;
  int T = 0;                                // the largest band-tile count of the launch sizes the tile array
  for (int i = 0; i < ls->nb; ++i) T = T > ls->d[i].Bp / 16 ? T : ls->d[i].Bp / 16;
  if (T <= 12) hipLaunchKernelGGL((k_factor<WP, ftpw_for(12)>), dim3(wg), dim3(FNT), 0, st, *ls);
  else if (T <= 17) hipLaunchKernelGGL((k_factor<WP, ftpw_for(17)>), dim3(wg), dim3(FNT), 0, st, *ls);
  else if (T <= 19) hipLaunchKernelGGL((k_factor<WP, ftpw_for(19)>), dim3(wg), dim3(FNT), 0, st, *ls);
  else hipLaunchKernelGGL((k_factor<WP, ftpw_for(MAXT)>), dim3(wg), dim3(FNT), 0, st, *ls);
}

extern "C" hipError_t rxk_launch_factor(int wprec, const rxk::LaunchSet* ls, int wg,
                                        hipStream_t st) {
  using namespace rxk;
  if (wg <= 0) return hipSuccess;
  switch (wprec) {
    case P_F64: launch_factor_t<P_F64>(ls, wg, st); break;
    case P_F32: launch_factor_t<P_F32>(ls, wg, st); break;
    case P_BF16: launch_factor_t<P_BF16>(ls, wg, st); break;
    case P_F16: launch_factor_t<P_F16>(ls, wg, st); break;
    case P_FP8: launch_factor_t<P_FP8>(ls, wg, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
