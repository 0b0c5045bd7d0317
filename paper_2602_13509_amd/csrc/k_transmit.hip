// Transmission encoding of the scores and its receive-side inverse (paper,
// Section "System Implementation / Data Transmission", and the ground
// station's unpacking in Section "Ground Control Station").
//
// Sender: the square root of every score is taken in FP32, normalised by the
// largest of them (so the cube's highest score codes as 1) and rounded to
// IEEE binary16; the maximum m = sqrt(max delta) travels beside the codes.
// Receiver: the normalisation is undone and the value squared,
// delta^ = (h m)^2 in FP32, and the paper's relative threshold marks
// h^2 > tau (the normalised squared score against e.g. 0.110).
//
//   k_tx_clear / k_tx_maxkey / k_tx_finalize -- m = sqrt(max delta) over the
//       finite scores, through an order-preserving 32-bit key held in the
//       caller's max slot (one atomic per workgroup); m = 0 when there is none
//   k_tx_encode -- one score per thread: sqrt, divide by m, RNE to binary16
//   k_tx_decode -- one 32-pixel mask word per thread
#include "rx_dev.h"

namespace rxk {

constexpr int TXNT = 256;
constexpr int TX_MAXWG = 1024;

// order-preserving key of an FP32 value: larger value, larger key; 0 = none
__device__ __forceinline__ uint32_t fkey(float v) {
  const uint32_t u = __builtin_bit_cast(uint32_t, v);
  return (u >> 31) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_fkey(uint32_t k) {
  const uint32_t u = (k >> 31) ? (k & 0x7FFFFFFFu) : ~k;
  return __builtin_bit_cast(float, u);
}

template <typename T>
__device__ __forceinline__ float score_f32(const T* sc, int64_t i) {
  return (float)sc[i];
}

__global__ void k_tx_clear(uint32_t* key) {
  if (threadIdx.x == 0) *key = 0u;
}

template <typename T>
__global__ void __launch_bounds__(TXNT) k_tx_maxkey(const T* sc, int64_t n, uint32_t* key) {
  __shared__ uint32_t wm[TXNT / 64];
  uint32_t m = 0u;
  for (int64_t i = (int64_t)blockIdx.x * TXNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * TXNT) {
    const float v = score_f32(sc, i);
    if (v == v) m = max(m, fkey(v));
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < TXNT / 64; ++w) m = max(m, wm[w]);
    if (m) atomicMax(key, m);
  }
}

// key -> m = sqrt(max delta), in place (the slot becomes the FP32 maximum)
__global__ void k_tx_finalize(float* slot) {
  if (threadIdx.x == 0) {
    const uint32_t k = *reinterpret_cast<uint32_t*>(slot);
    const float mx = k ? from_fkey(k) : 0.0f;
    *slot = sqrtf(mx);
  }
}

template <typename T>
__global__ void __launch_bounds__(TXNT) k_tx_encode(const T* sc, int64_t n, const float* mslot, uint16_t* codes) {
  const int64_t i = (int64_t)blockIdx.x * TXNT + threadIdx.x;
  if (i >= n) return;
  const float m = *mslot;
  const float s = sqrtf(score_f32(sc, i));
  // correctly rounded FP32 square root and division, then one RNE rounding
  const float q = (m > 0.0f) ? s / m : (s == s ? 0.0f : s);
  codes[i] = __builtin_bit_cast(uint16_t, (_Float16)q);
}

__global__ void __launch_bounds__(TXNT) k_tx_decode(const uint16_t* codes, int64_t n, const float* mslot,
                                                    float tau, float* delta, uint32_t* bits) {
  const int64_t wq = (int64_t)blockIdx.x * TXNT + threadIdx.x;   // one 32-pixel word per thread
  if (wq * 32 >= n) return;
  const float m = *mslot;
  uint32_t word = 0u;
  for (int j = 0; j < 32; ++j) {
    const int64_t p = wq * 32 + j;
    if (p >= n) break;
    const float h = (float)__builtin_bit_cast(_Float16, codes[p]);
    // h has 11 significant bits, so h * h is exact in FP32
    if (h * h > tau) word |= 1u << j;
    if (delta) {
      const float u = h * m;
      delta[p] = u * u;
    }
  }
  if (bits) bits[wq] = word;
}

}  // namespace rxk

extern "C" hipError_t rxk_launch_tx_encode(const void* sc, int f64, int64_t n, uint16_t* codes, float* mslot,
                                           hipStream_t st) {
  using namespace rxk;
  uint32_t* key = reinterpret_cast<uint32_t*>(mslot);
  hipLaunchKernelGGL(k_tx_clear, dim3(1), dim3(64), 0, st, key);
  if (n > 0) {
    const int wg = (int)std::min<int64_t>(TX_MAXWG, (n + TXNT - 1) / TXNT);
    if (f64) hipLaunchKernelGGL((k_tx_maxkey<double>), dim3(wg), dim3(TXNT), 0, st, static_cast<const double*>(sc), n, key);
    else hipLaunchKernelGGL((k_tx_maxkey<float>), dim3(wg), dim3(TXNT), 0, st, static_cast<const float*>(sc), n, key);
  }
  hipLaunchKernelGGL(k_tx_finalize, dim3(1), dim3(64), 0, st, mslot);
  if (n > 0) {
    const int64_t wg = (n + TXNT - 1) / TXNT;
    if (f64) hipLaunchKernelGGL((k_tx_encode<double>), dim3(wg), dim3(TXNT), 0, st, static_cast<const double*>(sc), n, mslot, codes);
    else hipLaunchKernelGGL((k_tx_encode<float>), dim3(wg), dim3(TXNT), 0, st, static_cast<const float*>(sc), n, mslot, codes);
  }
  return hipGetLastError();
}

extern "C" hipError_t rxk_launch_tx_decode(const uint16_t* codes, int64_t n, const float* mslot, float tau,
                                           float* delta, uint32_t* bits, hipStream_t st) {
  using namespace rxk;
  if (n <= 0) return hipSuccess;
  const int64_t words = (n + 31) / 32;
  hipLaunchKernelGGL(k_tx_decode, dim3((words + TXNT - 1) / TXNT), dim3(TXNT), 0, st, codes, n, mslot, tau, delta, bits);
  return hipGetLastError();
}
