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
  const int b = min(lineb / d.blk_lines, d.nblk - 1);
  const int s0 = (g % d.cpl) * KC;
  const int nvalid = min(KC, d.S - s0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int n = lane & 15, kg = lane >> 4;
  const T* xl = static_cast<const T*>(d.x) + (int64_t)lineb * B * d.S + s0;
  const double* mu = d.mu_snap + (int64_t)b * Bp;
  constexpr bool F64OUT = (P == P_F64);
  const int64_t out0 = (int64_t)lineb * d.S + s0;

  if (d.status[b] != 0) {                              // singular / not ready: NaN scores
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
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) dv[j] = 0.0f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) dt[(k0 + j) * LDB + k] = to_storage<P>(dv[j]);
    }
    __syncthreads();
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
        dl += y * y;
      }
    }
  }
  dl += __shfl_xor(dl, 16, 64);
  dl += __shfl_xor(dl, 32, 64);
  if (kg == 0 && 16 * w + n < nvalid) {
    if constexpr (F64OUT) static_cast<double*>(d.scores)[out0 + 16 * w + n] = dl;
    else static_cast<float*>(d.scores)[out0 + 16 * w + n] = dl;
  }
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

__global__ void __launch_bounds__(NT) k_maxkey(const void* sc, int f64, int64_t n, uint64_t* out) {
  uint64_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const double v = score_at(sc, f64, i);
    if (v == v) m = max(m, okey(v));
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint64_t)__shfl_xor((unsigned long long)m, o, 64));
  if ((threadIdx.x & 63) == 0 && m) atomicMax((unsigned long long*)out, (unsigned long long)m);
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

}  // namespace rxk

extern "C" hipError_t rxk_launch_whiten(int in_type, int wprec, const rxk::LaunchSet* ls, int wg, int Bw,
                                        hipStream_t st) {
  using namespace rxk;
  if (wg <= 0) return hipSuccess;
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
    hipLaunchKernelGGL(k_maxkey, dim3(gs), dim3(NT), 0, st, sc, f64, n, maxkey);
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
