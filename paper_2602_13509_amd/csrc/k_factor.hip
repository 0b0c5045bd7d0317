// FP64 factorisation of the window covariance for Eq. 1 of the paper
// (Section "System Implementation / Detection Algorithm"): the score needs
// Sigma^{-1}; it is applied as delta = |W (x - mu)|^2 with W lower
// triangular and W^T W = (Sigma + lambda I)^{-1}.
//
// One 512-thread workgroup per block snapshot (causal mode adds one for the
// window before the batch):
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
// tiles per wave, a template argument sized to the band count: wave 0 holds
// the T diagonal tiles, the other waves share the T (T - 1) / 2 tiles below
// the diagonal; up to 20 tiles (B <= 272) they and the step's temporaries fit
// in registers
constexpr int ftpw_for(int T) {
  return T > (T * (T - 1) / 2 + FNW - 2) / (FNW - 1) ? T : (T * (T - 1) / 2 + FNW - 2) / (FNW - 1);
}
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
  __shared__ double ybuf[2][FTS];       // Y_k = L_kk^{-1}, by step parity
  __shared__ double sc[MAXBP];          // equilibration scale
  __shared__ double T22[16][17];
  __shared__ double red[FNW];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const double N = d.n_snap[b];

  if (tid == 0) d.clipflag[b] = 0;             // set by the whitening of this batch
  // the block this slot scores (causal mode: slot b scores block b + 1, the
  // extra slot nblk block 0, the last slot none in this batch); the stream's
  // singular / not-ready counters count scored blocks
  const int sbk = !d.causal ? b : (b == d.nblk ? 0 : (b + 1 < d.nblk ? b + 1 : -1));
  const bool counted = sbk >= 0 && !causal_empty(d, sbk);
  if (tid == 0 && sbk >= 0 && causal_empty(d, sbk)) atomicAdd(d.nsing + 1, 1u);   // no window before it
  // window too small: Sigma is singular (no ridge), or its normaliser is not
  // positive (float input whose non-finite pixels left too few)
  if ((d.rho == 0.0 && N <= (double)B) || !(N - (double)d.ddof > 0.0)) {
    if (tid == 0) { d.status[b] = 2; if (counted) atomicAdd(d.nsing + 1, 1u); }
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
    if (tid == 0) { d.status[b] = 1; if (counted) atomicAdd(d.nsing, 1u); }
    return;
  }

  // ---- one right-looking sweep over 16x16 tiles held in registers.  Wave 0
  // owns the diagonal tiles (slot s holds tile (s, s)); the other waves own
  // the tiles below the diagonal, cyclically in row-major order.  Step k, with
  // Y_k = L_kk^{-1} already known:
  //   P: the pivot column becomes L_ik = R_ik Y_k^T and the pivot row of the
  //      eliminated identity becomes final rows of W = L^{-1}:
  //      W_kj = Y_k E_kj, W_kk = Y_k; each owner forms its own tiles and
  //      publishes them in LDS;
  //   U: every tile below row k takes one 16x16x16 product:
  //      j > k: R_ij -= L_ik L_jk^T   j == k: E_ik = -L_ik Y_k   j < k: E_ij -= L_ik W_kj
  //      and wave 0, once its own updates are done, factors the new diagonal
  //      tile (k + 1, k + 1) into Y_{k+1} while the other waves still update.
  // Two barriers per step; each tile holds R, then L, then E, then W.
  const int T = Bp / 16;
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
    int i = -1, j = -1;
    if (wv == 0) {
      if (s < T) { i = s; j = s; }
    } else {
      const int u = s * (FNW - 1) + (wv - 1);      // index among the tiles below the diagonal
      if (u < T * (T - 1) / 2) {
        i = 1;
        while ((i + 1) * i / 2 <= u) ++i;
        j = u - i * (i - 1) / 2;
      }
    }
    ti[s] = __builtin_amdgcn_readfirstlane(i);
    tj[s] = __builtin_amdgcn_readfirstlane(j);
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

  // 16x16 Cholesky of the diagonal tile staged in T22 and Y = L^{-1} together,
  // in wave 0: lane = (row i, column group cg of 4) holds S[i][4cg..4cg+3] and
  // the eliminated identity E[i][4cg..4cg+3].  Column j: pivot d = sqrt(S[j][j]),
  // L[i][j] = S[i][j] / d, Y[j][.] = E[j][.] / d, then S[i][k] -= L[i][j] L[k][j]
  // (j < k <= i) and E[i][.] -= L[i][j] Y[j][.] (i > j).
  auto diag = [&](double* yout) {
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
      // 1/sqrt(piv): the hardware reciprocal square root, then two Newton
      // steps (each squares the relative error), within a few ulp of the
      // correctly rounded value and far shorter than a square root and a
      // division on this column's critical path
      double rd = __builtin_amdgcn_rsq(piv);
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const double e = __builtin_fma(-piv * rd, rd, 1.0);
        rd = __builtin_fma(0.5 * rd, e, rd);
      }
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
    for (int e = 0; e < 4; ++e) yout[i * 17 + 4 * cg + e] = y[e];
    if (lane == 0 && bad) flag = 1;
  };
  // wave 0 puts its diagonal tile kd into T22 (the same wave reads it back)
  auto stage_diag = [&](int kd) {
#pragma unroll
    for (int s = 0; s < FTPW; ++s) {
      if (ti[s] == kd && tj[s] == kd) {
        double* p = &T22[0][0] + offB0;
#pragma unroll
        for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
      }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  };

  // Step -1 only factors the first diagonal tile, so one copy of the
  // diagonal code serves every step.
  for (int k = -1; k < T && !flag; ++k) {
    if (k >= 0) {
      int offA = offA0, offB = offB0;
      asm volatile("" : "+v"(offA), "+v"(offB));   // keep derived addresses inside the step
      const double* yk = ybuf[k & 1];
      // ---- P: pivot column L_ik = R_ik Y_k^T, pivot row W_kj = Y_k E_kj, W_kk = Y_k
#pragma unroll
      for (int s = 0; s < FTPW; ++s) {
        if (tj[s] == k && ti[s] > k) {
          // R_ik goes through this wave's LDS slot to be read in operand order
          double* lc = lcol + ti[s] * FTS;
          double* p = lc + offB;
#pragma unroll
          for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          const double* la = lc + offA;
          const double* yb = yk + offA;
          tl[s] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4)
            tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(la[4 * q4], yb[4 * q4], tl[s], 0, 0, 0);
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
          for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
        } else if (ti[s] == k && tj[s] >= 0 && tj[s] < k) {
          // E_kj goes through this wave's LDS slot (each lane reads back the
          // elements it wrote), then W_kj replaces it there
          double* pr = prow + tj[s] * FTS;
          double* p = pr + offB;
#pragma unroll
          for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          const double* ya = yk + offA;
          const double* pb = pr + offB;
          tl[s] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4)
            tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[4 * q4], pb[68 * q4], tl[s], 0, 0, 0);
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
          for (int r = 0; r < 4; ++r) p[68 * r] = tl[s][r];
        } else if (ti[s] == k && tj[s] == k) {
          const double* yb = yk + offB;
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
      // ---- U: update every tile below row k
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
    }
    // wave 0: the next diagonal tile is final now; factor it
    if (wv == 0 && k + 1 < T) {
      stage_diag(k + 1);
      diag(ybuf[(k + 1) & 1]);
    }
    __syncthreads();
  }
  if (flag) {
    if (tid == 0) { d.status[b] = 1; if (counted) atomicAdd(d.nsing, 1u); }
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

// Causal mode 2: slot nblk (the window before the batch, which scores block
// 0) is the previous batch's last slot, already factored: copy what the
// whitening reads (mean, operand or FP64 W, band and row scales, status) and
// count block 0 as the factor counts the blocks it scores.  CPWG workgroups
// per batch share the copies in 16-byte strides (every size is a multiple of
// 16 bytes); the first one also moves the status.
__global__ void __launch_bounds__(256) k_copy_slot(LaunchSet ls) {
  int z;
  const int bi = find_batch(ls, blockIdx.x, z);
  const BatchDesc& d = ls.d[bi];
  const int Bp = d.Bp, n = d.nblk;
  auto copy = [&](void* dst, const void* src, int64_t bytes) {
    uint4* o = static_cast<uint4*>(dst);
    const uint4* i = static_cast<const uint4*>(src);
    for (int64_t q = (int64_t)z * 256 + threadIdx.x; q < bytes / 16; q += CPWG * 256) o[q] = i[q];
  };
  copy(d.mu_snap + (int64_t)n * Bp, d.src_mu, (int64_t)Bp * 8);
  if (d.wl_bytes > 0) copy(static_cast<char*>(d.wlp) + n * d.wl_bytes, d.src_wlp, d.wl_bytes);
  else copy(d.w64 + (int64_t)n * Bp * Bp, d.src_w64, (int64_t)Bp * Bp * 8);
  copy(d.iscale + (int64_t)n * Bp, d.src_isc, (int64_t)Bp * 4);
  copy(d.oscale + (int64_t)n * Bp, d.src_osc, (int64_t)Bp * 4);
  if (z == 0 && threadIdx.x == 0) {
    const int st = d.src_status[0];
    d.status[n] = st;
    d.clipflag[n] = 0;
    if (causal_empty(d, 0)) atomicAdd(d.nsing + 1, 1u);
    else if (st == 1) atomicAdd(d.nsing, 1u);
    else if (st == 2) atomicAdd(d.nsing + 1, 1u);
  }
}

}  // namespace rxk

// ls->wg0 must hold the prefix of CPWG workgroups per batch.
extern "C" hipError_t rxk_launch_copy_slot(const rxk::LaunchSet* ls, int nb, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(rxk::k_copy_slot, dim3(nb * rxk::CPWG), dim3(256), 0, st, *ls);
  return hipGetLastError();
}

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
