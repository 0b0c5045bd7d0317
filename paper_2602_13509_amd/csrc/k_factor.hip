// FP64 factorisation of the window covariance for Eq. 1 of the paper
// (Section "System Implementation / Detection Algorithm"): the score needs
// Sigma^{-1}; it is applied as delta = |W (x - mu)|^2 with W lower
// triangular and W^T W = (Sigma + lambda I)^{-1}.  Per block snapshot
// (causal mode adds one for the window before the batch):
//   Sigma = M2 / (N - ddof);  lambda = rho * tr(Sigma) / B;  Sigma_r = Sigma + lambda I
//   equilibration R = S Sigma_r S with S = diag(Sigma_r,kk^{-1/2})  (unit diagonal)
//   R = L L^T (k_chol), W = L^{-1} S (k_trinv), FP64 matrix-core products.
//   A non-positive pivot flags the block singular (its scores become NaN).
// The whitening operand in the whitening precision is then formed (k_wop)
// with power-of-two scales: input band scale 2^-e_k (e_k = floor(log2
// sigma_k)) and output row scale 2^f_i chosen so each row fits the format's
// range.
#include <type_traits>

#include "rx_dev.h"

namespace rxk {

constexpr int MAXBP = 16 * MAXT;
constexpr int FTS = 16 * 17;            // LDS tile: 16 rows, pitch 17 doubles (bank-conflict free)

__device__ __forceinline__ double readlane_d(double x, int l) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = __builtin_amdgcn_readlane(v.x, l);
  v.y = __builtin_amdgcn_readlane(v.y, l);
  return __builtin_bit_cast(double, v);
}

// ============================================================================
// Three-kernel factorisation (up to 320 bands, T <= 20 tiles), all FP64:
//   k_chol   one 1024-thread workgroup per block: conditioning (as above), then
//            the Cholesky factor of the equilibrated R by a right-looking sweep
//            over 16x16 tiles held in registers.  Hands over, per block, the
//            diagonal inverses Y_k = L_kk^{-1} and the tiles L_ik (i > k) in
//            matrix-core operand order, and the equilibration scale.
//   k_trinv  one workgroup per (block, 16-column tile j): column j of
//            W = L^{-1} S by forward substitution,
//              W_jj = Y_j,   W_ij = -Y_i sum_{j <= m < i} L_im W_mj   (i > j),
//            the columns being independent; the sum over m is shared by the
//            four waves and added in a fixed order.
//   k_wop    one workgroup per (block, 16-row tile): the row scales and the
//            whitening operand of those rows (low-precision and FP32 paths).
// The Cholesky kernel holds only R (no eliminated identity): up to 272 bands
// its tiles fit the registers of 16 waves; from 273 bands on, the tiles
// below the diagonal past eleven per wave stay in LDS.  The inverse, which
// is as much arithmetic again, runs on T workgroups per block instead of one.

constexpr int CNW = 16;                 // waves per Cholesky workgroup (4 per SIMD: 128 registers each)
constexpr int CNT = 64 * CNW;
constexpr int CDW = 3;                  // waves owning the diagonal tiles (tile (k, k) -> wave k % CDW)
constexpr int CMAXT = MAXT;             // largest tile count (320 bands)
constexpr int CREG = 11;                // most tiles below the diagonal a wave holds in registers
// tiles per diagonal wave; tiles per other wave, in registers and (past CREG,
// from 273 bands on) in LDS, sized to the tile count T
constexpr int cdiag_for(int T) { return (T + CDW - 1) / CDW; }
constexpr int coff_for(int T) { return (T * (T - 1) / 2 + CNW - CDW - 1) / (CNW - CDW); }
constexpr int creg_for(int T) { return coff_for(T) < CREG ? coff_for(T) : CREG; }
constexpr int clds_for(int T) { return coff_for(T) - creg_for(T); }
// lfac layout per block (doubles): Y_k at 256 k, L_ik at 256 (T + i (i - 1) / 2 + k), then
// the equilibration scale [Bp].  Lane l of a stored tile holds, at 4 l + q, the element
// (row l % 16, column l / 16 + 4 q): the A operand of four v_mfma_f64_16x16x4f64.
__host__ __device__ constexpr int64_t lf_tiles(int T) { return (int64_t)T + (int64_t)T * (T - 1) / 2; }
__device__ __forceinline__ int64_t lf_L(int T, int i, int k) { return 256 * ((int64_t)T + (int64_t)i * (i - 1) / 2 + k); }

// Workgroup barrier ordering LDS accesses only: the sweep's global stores
// (the hand-off, read only by the next kernel) and prefetched global loads
// stay in flight across it, where __syncthreads() would wait for them.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Tiles of the sweep are held in "fragment layout": lane l (lr = l % 16,
// lg = l / 16) keeps, at index q, the element X[lr][lg + 4 q] of a 16x16
// tile X.  That is at once the A operand of X and the B operand of X^T for
// four chained v_mfma_f64_16x16x4f64 (chunk q), and an MFMA whose product is
// C leaves C^T's fragment layout in its accumulator.  So the sweep needs no
// transposes: with F(X) the fragment layout of X,
//   L_ik = R_ik Y_k^T:  acc = Y_k R_ik^T = L_ik^T   (A = F(Y_k), B = F(R_ik))  -> F(L_ik)
//   R_ij -= L_ik L_jk^T: R_ij^T -= L_jk L_ik^T      (A = F(L_jk), B = F(L_ik)) on F(R_ij)
// and tiles travel through LDS as one 32-byte vector per lane.

// What the sweep of every wave shares: LDS, the hand-off pointer and the
// equilibrated covariance's source.
struct CholCtx {
  f64x4* lcol;           // [CMAXT][64] the pivot column F(L_ik), lane-major
  f64x4* ybuf;           // [2][64] F(Y_k), by step parity
  f64x4* ltile;          // [NL][64] this wave's tiles kept in LDS (from 273 bands on)
  double* t22;           // [FTS] this wave's diagonal staging
  const double* sc;      // [Bp] equilibration scale
  int* flag;             // non-positive pivot seen
  const double* R;       // M2 snapshot (lower)
  double* lf;            // hand-off of this block
  double rden, lam;
  int B, Bp, T, wv, lane;
};

// 16x16 Cholesky of the staged diagonal tile (row-major, pitch 17) and its
// inverse together (one wave): lane = (row i, column group cg of 4) holds
// S[i][4cg..4cg+3] and the eliminated identity E[i][4cg..4cg+3].  Column j:
// pivot p = S[j][j], 1/sqrt(p) from the hardware estimate and two Newton
// steps, L[i][j] = S[i][j]/sqrt(p), Y[j][.] = E[j][.]/sqrt(p), then
// S[i][k] -= L[i][j] L[k][j] (i, k > j) and E[i][.] -= L[i][j] Y[j][.]
// (i > j).  S is kept whole and symmetric (it starts from the lower
// triangle, and both halves take the same products), so L[k][j] = S[j][k] /
// sqrt(p) and Y[j][.] sit in the lane's own 16-lane row, at position j: a
// row broadcast (DPP row_newbcast) fetches them; only L[i][j], held in row
// group j / 4, crosses rows.  Y = L^{-1} goes, as F(Y), to yout (LDS) and yg
// (hand-off).
template <int N> __device__ __forceinline__ double row_bcast(double x) {
  const int2 v = __builtin_bit_cast(int2, x);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(0, v.x, 0x150 + N, 0xF, 0xF, false);   // row_newbcast:N
  r.y = __builtin_amdgcn_update_dpp(0, v.y, 0x150 + N, 0xF, 0xF, false);
  return __builtin_bit_cast(double, r);
}

template <int J> using icj = std::integral_constant<int, J>;

__device__ __forceinline__ void chol_diag(const CholCtx& c, f64x4* yout, double* yg) {
  const int lane = c.lane;
  int i = lane & 15, cg = lane >> 4;
  asm volatile("" : "+v"(i), "+v"(cg));    // shuffle addresses are formed per step, not hoisted
  double v[4], y[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int col = 4 * cg + e;
    v[e] = c.t22[(i >= col ? i * 17 + col : col * 17 + i)];
    y[e] = (i == col) ? 1.0 : 0.0;
  }
  bool bad = false;
  auto column = [&](auto J) {
    constexpr int j = decltype(J)::value, je = j & 3, jg = j >> 2;
    const double piv = readlane_d(v[je], j + 16 * jg);
    bad |= !(piv > 0.0);
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
      lkj[e] = row_bcast<j>(v[e]) * rd;
      yj[e] = row_bcast<j>(y[e]) * rd;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = 4 * cg + e;
      if (kk > j && i > j) v[e] -= lij * lkj[e];
      y[e] = (i == j) ? yj[e] : ((i > j) ? y[e] - lij * yj[e] : y[e]);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  column(icj<0>{});  column(icj<1>{});  column(icj<2>{});  column(icj<3>{});
  column(icj<4>{});  column(icj<5>{});  column(icj<6>{});  column(icj<7>{});
  column(icj<8>{});  column(icj<9>{});  column(icj<10>{}); column(icj<11>{});
  column(icj<12>{}); column(icj<13>{}); column(icj<14>{}); column(icj<15>{});
  // Y row-major into the staging tile, then read back as F(Y)
  double* ys = c.t22;
#pragma unroll
  for (int e = 0; e < 4; ++e) ys[i * 17 + 4 * cg + e] = y[e];
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  const double* ya = ys + (lane & 15) * 17 + (lane >> 4);
  const f64x4 fy = f64x4{ya[0], ya[4], ya[8], ya[12]};
  yout[lane] = fy;
  *reinterpret_cast<f64x4*>(yg + 4 * lane) = fy;
  if (lane == 0 && bad) *c.flag = 1;
}

// F(R_ij) of the equilibrated, regularised covariance: element (lr, lg + 4 r);
// branch-free (every lane loads a valid address), padding selected away.
__device__ __forceinline__ f64x4 load_tile(const CholCtx& c, int ti, int tj) {
  const int lr = c.lane & 15, lg = c.lane >> 4;
  f64x4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * ti + lr, col = 16 * tj + lg + 4 * r;
    const bool in = (row < c.B) && (col < c.B);
    const int hi = in ? (row >= col ? row : col) : 0, lo = in ? (row >= col ? col : row) : 0;
    double v = c.R[(int64_t)hi * c.Bp + lo] * c.rden + ((row == col) ? c.lam : 0.0);
    v *= c.sc[row] * c.sc[col];
    t[r] = in ? v : ((row == col) ? 1.0 : 0.0);
  }
  return t;
}

// The sweep of one wave over its NS tiles.  DIAG: the wave owns diagonal
// tiles (k = wv + CDW s) and factors them; otherwise tiles below the
// diagonal (index u = s (CNW - CDW) + wv - CDW in row-major order).  Every
// wave runs the same barriers.  Step k, with Y_k known:
//   P: the owners of column k form F(L_ik) from F(R_ik), publish it in LDS
//      and hand it over;
//   U: every tile with i >= j > k takes R_ij -= L_ik L_jk^T; the owner of
//      (k+1, k+1) updates that tile first and factors it (the next step
//      needs only Y_{k+1}), then its remaining tiles.
template <int NS, int NL, bool DIAG>
__device__ __forceinline__ void chol_sweep(const CholCtx& c) {
  const int lane = c.lane, wv = c.wv, T = c.T, B = c.B, Bp = c.Bp;
  const int lr = lane & 15, lg = lane >> 4;
  f64x4 tl[NS];
  int ti[NS], tj[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    int i = -1, j = -1;
    if (DIAG) {
      const int k = wv + CDW * s;
      if (k < T) { i = k; j = k; }
    } else {
      const int u = s * (CNW - CDW) + (wv - CDW);
      if (u < T * (T - 1) / 2) {
        i = 1;
        while ((i + 1) * i / 2 <= u) ++i;
        j = u - i * (i - 1) / 2;
      }
    }
    ti[s] = __builtin_amdgcn_readfirstlane(i);
    tj[s] = __builtin_amdgcn_readfirstlane(j);
    tl[s] = f64x4{0.0, 0.0, 0.0, 0.0};
    if (ti[s] >= 0) tl[s] = load_tile(c, ti[s], tj[s]);
  }
  // tiles past the register slots (from 273 bands on) live in LDS, each
  // read and written only by its owner wave
  int li[NL > 0 ? NL : 1], lj[NL > 0 ? NL : 1];
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    int i = -1, j = -1;
    const int u = (NS + s) * (CNW - CDW) + (wv - CDW);
    if (u < T * (T - 1) / 2) {
      i = 1;
      while ((i + 1) * i / 2 <= u) ++i;
      j = u - i * (i - 1) / 2;
    }
    li[s] = __builtin_amdgcn_readfirstlane(i);
    lj[s] = __builtin_amdgcn_readfirstlane(j);
    if (li[s] >= 0) c.ltile[s * 64 + lane] = load_tile(c, li[s], lj[s]);
  }
#pragma clang loop unroll(disable)
  for (int k = -1; k < T && !*c.flag; ++k) {
    if (!DIAG && k >= 0) {
      const double* yk = reinterpret_cast<const double*>(c.ybuf + (k & 1) * 64 + lane);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (tj[s] == k && ti[s] > k) {
          f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(yk[q], tl[s][q], acc, 0, 0, 0);
          tl[s] = acc;
          c.lcol[ti[s] * 64 + lane] = acc;
          *reinterpret_cast<f64x4*>(c.lf + lf_L(T, ti[s], k) + 4 * lane) = acc;
        }
      }
#pragma unroll
      for (int s = 0; s < NL; ++s) {
        if (lj[s] == k && li[s] > k) {
          const f64x4 t = c.ltile[s * 64 + lane];
          f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(yk[q], t[q], acc, 0, 0, 0);
          c.lcol[li[s] * 64 + lane] = acc;
          *reinterpret_cast<f64x4*>(c.lf + lf_L(T, li[s], k) + 4 * lane) = acc;
        }
      }
    }
    if (k >= 0) lds_sync();
    const bool dw = DIAG && k + 1 < T && wv == (k + 1) % CDW;
    if (dw) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (ti[s] == k + 1) {
          if (k >= 0) {
            const f64x4 lk = c.lcol[ti[s] * 64 + lane];
#pragma unroll
            for (int q = 0; q < 4; ++q) tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-lk[q], lk[q], tl[s], 0, 0, 0);
          }
          double* p = c.t22 + lr * 17 + lg;       // F(R) -> row-major
#pragma unroll
          for (int r = 0; r < 4; ++r) p[4 * r] = tl[s][r];
        }
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      chol_diag(c, c.ybuf + ((k + 1) & 1) * 64, c.lf + 256 * (int64_t)(k + 1));
    }
    if (k >= 0) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (ti[s] > k && tj[s] > k && !(dw && ti[s] == k + 1)) {
          // element loads, so only the operands of one chunk need registers
          const double* pi = reinterpret_cast<const double*>(c.lcol + ti[s] * 64 + lane);
          const double* pj = reinterpret_cast<const double*>(c.lcol + tj[s] * 64 + lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) tl[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-pj[q], pi[q], tl[s], 0, 0, 0);
        }
      }
#pragma unroll
      for (int s = 0; s < NL; ++s) {
        if (li[s] > k && lj[s] > k) {
          const double* pi = reinterpret_cast<const double*>(c.lcol + li[s] * 64 + lane);
          const double* pj = reinterpret_cast<const double*>(c.lcol + lj[s] * 64 + lane);
          f64x4 t = c.ltile[s * 64 + lane];
#pragma unroll
          for (int q = 0; q < 4; ++q) t = __builtin_amdgcn_mfma_f64_16x16x4f64(-pj[q], pi[q], t, 0, 0, 0);
          c.ltile[s * 64 + lane] = t;
        }
      }
    }
    lds_sync();
  }
}

// One 1024-thread workgroup per block slot: conditioning (trace, ridge,
// equilibration; a window too small or a non-positive variance stops here),
// then the Cholesky sweep; the diagonal inverses and L tiles are handed over
// to k_trinv, the status is set (0: factored, 1: singular, 2: not ready).
template <int T_MAX>
__global__ void __launch_bounds__(CNT) k_chol(LaunchSet ls) {
  int b;
  const int bi = find_batch(ls, blockIdx.x, b);
  const BatchDesc& d = ls.d[bi];
  b += d.fslot0;
  const int B = d.B, Bp = d.Bp;
  const int T = Bp / 16;
  const int64_t bp2 = (int64_t)Bp * Bp;
  const double* R = d.m2_snap + b * bp2;
  double* lf = d.lfac + b * d.lf_stride;
  __shared__ f64x4 lcol[T_MAX * 64];
  __shared__ f64x4 ybuf[2 * 64];
  __shared__ f64x4 ltile[(clds_for(T_MAX) > 0 ? clds_for(T_MAX) * (CNW - CDW) : 1) * 64];
  __shared__ double sc[16 * T_MAX];
  __shared__ double t22[CDW][FTS];
  __shared__ double red[CNW];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double N = d.n_snap[b];

  if (tid == 0) d.clipflag[b] = 0;             // set by the whitening of this batch
  // the blocks this slot scores (causal mode: slot b scores block b + 1, the
  // extra slot nblk block 0, the last slot none in this batch; one-pass
  // mode: slot nblk scores every block); the stream's singular / not-ready
  // counters count scored blocks
  int counted, nostats;
  slot_scores(d, b, counted, nostats);
  if (tid == 0 && nostats > 0) atomicAdd(d.nsing + 1, (unsigned)nostats);
  if ((d.rho == 0.0 && N <= (double)B) || !(N - (double)d.ddof > 0.0)) {
    if (tid == 0) { d.status[b] = 2; if (counted) atomicAdd(d.nsing + 1, (unsigned)counted); }
    return;
  }
  const double den = N - (double)d.ddof;
  if (tid == 0) flag = 0;
  double tr = 0.0;
  for (int k = tid; k < B; k += CNT) tr += R[(int64_t)k * Bp + k];
  tr = wave_sum(tr);
  if (lane == 0) red[wv] = tr;
  __syncthreads();
  tr = 0.0;
  for (int i = 0; i < CNW; ++i) tr += red[i];
  const double lam = d.rho * (tr / den) / (double)B;
  for (int k = tid; k < Bp; k += CNT) {
    double v = 1.0;
    if (k < B) {
      v = R[(int64_t)k * Bp + k] / den + lam;
      if (!(v > 0.0) || !(v < INFINITY)) flag = 1;
    }
    const double s = 1.0 / sqrt(v);
    sc[k] = s;
    lf[256 * lf_tiles(T) + k] = s;
  }
  __syncthreads();
  if (flag) {
    if (tid == 0) { d.status[b] = 1; if (counted) atomicAdd(d.nsing, (unsigned)counted); }
    return;
  }
  CholCtx c;
  c.lcol = lcol; c.ybuf = ybuf; c.t22 = t22[wv < CDW ? wv : 0]; c.sc = sc; c.flag = &flag;
  c.ltile = ltile + (wv >= CDW ? (wv - CDW) * clds_for(T_MAX) * 64 : 0);
  c.R = R; c.lf = lf; c.rden = 1.0 / den; c.lam = lam;
  c.B = B; c.Bp = Bp; c.T = T; c.wv = wv; c.lane = lane;
  if (wv < CDW) chol_sweep<cdiag_for(T_MAX), 0, true>(c);
  else chol_sweep<creg_for(T_MAX), clds_for(T_MAX), false>(c);
  if (flag) {
    if (tid == 0) { d.status[b] = 1; if (counted) atomicAdd(d.nsing, (unsigned)counted); }
    return;
  }
  if (tid == 0) d.status[b] = 0;
}

// Column tile j of W = L^{-1} S for one block (256 threads).  Tiles of W
// are held as G_mj = F(W_mj^T) (lane (lr, lg) keeps W_mj[lg + 4 q][lr]),
// which is the B operand of W_mj and also what an MFMA producing W_mj
// leaves in its accumulator:
//   S_ij = sum_m L_im W_mj      (A = F(L_im) from the hand-off, B = G_mj)
//   W_ij = -Y_i S_ij            (A = F(Y_i), B = the reduced S_ij accumulator)
// Row i takes the four waves' partial sums over m = j + w, j + w + 4, ...
// (added in wave order), then W_ij on wave 0.  The L tiles of the next
// row are loaded while the current row is reduced.  Rows and columns past
// the band count are written as zeros.
constexpr int VW = 4;                   // waves per inverse workgroup
constexpr int VMT = (CMAXT + VW - 1) / VW;   // most m terms per wave and row
__global__ void __launch_bounds__(64 * VW) k_trinv(LaunchSet ls) {
  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  const int B = d.B, Bp = d.Bp, T = Bp / 16;
  const int b = d.fslot0 + local / T, j = local % T;
  if (d.status[b] != 0) return;
  const double* lf = d.lfac + b * d.lf_stride;
  const double* scg = lf + 256 * lf_tiles(T);
  double* W = d.w64 + (int64_t)b * Bp * Bp;
  __shared__ f64x4 wcol[CMAXT * 64];     // G_mj, m >= j, lane-major
  __shared__ f64x4 red[VW * 64];         // per-wave partial sums of the current row
  __shared__ double yt[FTS];             // Y_j row-major (its transpose read)
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lg = lane >> 4;
  const int col = 16 * j + lr;
  const double scol = col < B ? scg[col] : 0.0;

  // W_jj = Y_j: G_jj[q] = Y_j[lg + 4 q][lr], from F(Y_j) through LDS
  if (wv == 0) {
    const f64x4 y = *reinterpret_cast<const f64x4*>(lf + 256 * (int64_t)j + 4 * lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) yt[lr * 17 + lg + 4 * q] = y[q];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    f64x4 g;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      g[r] = yt[(lg + 4 * r) * 17 + lr];
      const int row = 16 * j + lg + 4 * r;
      W[(int64_t)row * Bp + col] = (row < B && col < B) ? g[r] * scol : 0.0;
    }
    wcol[j * 64 + lane] = g;
  }
  __syncthreads();
  // F(L_im) of this wave's terms for row i: m = j + wv + 4 t
  f64x4 cur[VMT], nxt[VMT];
  auto load_row = [&](int i, f64x4* dst) {
#pragma unroll
    for (int t = 0; t < VMT; ++t) {
      const int m = j + wv + VW * t;
      if (m < i) dst[t] = *reinterpret_cast<const f64x4*>(lf + lf_L(T, i, m) + 4 * lane);
    }
  };
  if (j + 1 < T) load_row(j + 1, cur);
  for (int i = j + 1; i < T; ++i) {
    f64x4 yi = f64x4{0.0, 0.0, 0.0, 0.0};
    if (wv == 0) yi = *reinterpret_cast<const f64x4*>(lf + 256 * (int64_t)i + 4 * lane);
    if (i + 1 < T) load_row(i + 1, nxt);
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < VMT; ++t) {
      const int m = j + wv + VW * t;
      if (m < i) {
        const f64x4 g = wcol[m * 64 + lane];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[t][q], g[q], acc, 0, 0, 0);
      }
    }
    red[wv * 64 + lane] = acc;
    lds_sync();
    if (wv == 0) {
      const f64x4 s0 = red[lane], s1 = red[64 + lane], s2 = red[128 + lane], s3 = red[192 + lane];
      f64x4 w = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) w = __builtin_amdgcn_mfma_f64_16x16x4f64(yi[q], ((s0[q] + s1[q]) + s2[q]) + s3[q], w, 0, 0, 0);
      w = -w;
      wcol[i * 64 + lane] = w;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + lg + 4 * r;
        W[(int64_t)row * Bp + col] = (row < B && col < B) ? w[r] * scol : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < VMT; ++t) cur[t] = nxt[t];
    lds_sync();
  }
}

// Row tile t of the whitening operand for one block (256 threads): row
// maxima of |W_ij 2^e_j| (exact in any order), the row scales 2^f_i, the band
// scales 2^-e_k of the tile's bands, and the operand rows in the whitening
// format, read from the W that k_trinv wrote.
template <int WP>
__global__ void __launch_bounds__(256) k_wop(LaunchSet ls) {
  using S = typename MM<WP>::storage;
  int local;
  const int bi = find_batch(ls, blockIdx.x, local);
  const BatchDesc& d = ls.d[bi];
  const int B = d.B, Bp = d.Bp, T = Bp / 16;
  const int b = d.fslot0 + local / T, t = local % T;
  if (d.status[b] != 0) return;
  constexpr bool LP = (WP == P_BF16 || WP == P_F16 || WP == P_FP8);
  constexpr int top = (WP == P_FP8) ? 7 : 14;   // scaled row maximum lands in [2^top, 2^(top+1))
  const double* scg = d.lfac + b * d.lf_stride + 256 * lf_tiles(T);
  const double* W = d.w64 + (int64_t)b * Bp * Bp;
  const int Bw = 32 * ((Bp + 31) / 32);
  S* wl = static_cast<S*>(d.wlp) + (int64_t)b * Bp * Bw;
  __shared__ int ek[16 * MAXT];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ncol = 16 * (t + 1);                 // columns of the row tile's lower part
  for (int k = tid; k < ncol; k += 256) ek[k] = (LP && k < B) ? ilogb(1.0 / scg[k]) : 0;
  if (tid < 16) {
    const int k = 16 * t + tid;
    d.iscale[(int64_t)b * Bp + k] = (float)ldexp(1.0, -((LP && k < B) ? ilogb(1.0 / scg[k]) : 0));
  }
  __syncthreads();
  constexpr int NCC = (16 * MAXT + 63) / 64;
  // the wave's four rows, read once (loads of all four in flight together)
  double w[4][NCC];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 16 * t + 4 * wv + q;
#pragma unroll
    for (int c = 0; c < NCC; ++c) {
      const int jj = lane + 64 * c;
      w[q][c] = jj < ncol ? W[(int64_t)i * Bp + jj] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 16 * t + 4 * wv + q;
    double m = 0.0;
    if (LP) {
#pragma unroll
      for (int c = 0; c < NCC; ++c) {
        const int jj = lane + 64 * c;
        if (jj <= i && jj < B) m = fmax(m, fabs(ldexp(w[q][c], ek[jj])));
      }
      for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    }
    const int fi = (LP && m > 0.0) ? ilogb(m) - top : 0;
    if (lane == 0) d.oscale[(int64_t)b * Bp + i] = (float)ldexp(1.0, fi);
#pragma unroll
    for (int c = 0; c < NCC; ++c) {
      const int jj = lane + 64 * c;
      if (jj < ncol) wl[(int64_t)i * Bw + jj] = to_storage<WP>((float)ldexp(w[q][c], ek[jj] - fi));
    }
  }
}

// Causal mode 2: slot nblk (the window before the batch, which scores block
// 0, or every block in one-pass mode) is a slot of the previous batch,
// already factored: copy what the whitening reads (mean, operand or FP64 W,
// band and row scales, status) and count the blocks it scores as the factor
// counts them.  CPWG workgroups
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
    int with, without;
    slot_scores(d, n, with, without);
    if (without) atomicAdd(d.nsing + 1, (unsigned)without);
    if (with && st == 1) atomicAdd(d.nsing, (unsigned)with);
    else if (with && st == 2) atomicAdd(d.nsing + 1, (unsigned)with);
  }
}

}  // namespace rxk

// ls->wg0 must hold the prefix of CPWG workgroups per batch.
extern "C" hipError_t rxk_launch_copy_slot(const rxk::LaunchSet* ls, int nb, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(rxk::k_copy_slot, dim3(nb * rxk::CPWG), dim3(256), 0, st, *ls);
  return hipGetLastError();
}

// k_chol (sized to the launch's largest tile count), then k_trinv and
// (except on the FP64 path) k_wop, each with T workgroups per block.
template <int WP>
static hipError_t launch_factor3(const rxk::LaunchSet* ls, int wg, int T, hipStream_t st) {
  using namespace rxk;
  if (T <= 8) hipLaunchKernelGGL((k_chol<8>), dim3(wg), dim3(CNT), 0, st, *ls);
  else if (T <= 12) hipLaunchKernelGGL((k_chol<12>), dim3(wg), dim3(CNT), 0, st, *ls);
  else if (T <= 17) hipLaunchKernelGGL((k_chol<17>), dim3(wg), dim3(CNT), 0, st, *ls);
  else hipLaunchKernelGGL((k_chol<CMAXT>), dim3(wg), dim3(CNT), 0, st, *ls);
  LaunchSet c = *ls;                        // T workgroups per block slot
  c.wg0[0] = 0;
  for (int i = 0; i < c.nb; ++i) c.wg0[i + 1] = c.wg0[i] + (ls->wg0[i + 1] - ls->wg0[i]) * (c.d[i].Bp / 16);
  const int n = c.wg0[c.nb];
  hipLaunchKernelGGL(k_trinv, dim3(n), dim3(64 * VW), 0, st, c);
  if constexpr (WP != P_F64) hipLaunchKernelGGL((k_wop<WP>), dim3(n), dim3(256), 0, st, c);
  return hipGetLastError();
}

extern "C" hipError_t rxk_launch_factor(int wprec, const rxk::LaunchSet* ls, int wg,
                                        hipStream_t st) {
  using namespace rxk;
  if (wg <= 0) return hipSuccess;
  int T = 0;
  for (int i = 0; i < ls->nb; ++i) T = T > ls->d[i].Bp / 16 ? T : ls->d[i].Bp / 16;
  if (T > CMAXT) return hipErrorInvalidValue;
  switch (wprec) {
    case P_F64: return launch_factor3<P_F64>(ls, wg, T, st);
    case P_F32: return launch_factor3<P_F32>(ls, wg, T, st);
    case P_BF16: return launch_factor3<P_BF16>(ls, wg, T, st);
    case P_F16: return launch_factor3<P_F16>(ls, wg, T, st);
    case P_FP8: return launch_factor3<P_FP8>(ls, wg, T, st);
    default: return hipErrorInvalidValue;
  }
}
