// Band selection and spectral binning of 16-bit counts at ingest (paper,
// Section "System Implementation / Data Acquisition": the out-of-range bands
// are discarded, 300 -> 280, and four consecutive bands are summed into one,
// 280 -> 70).  BIL in and out:
//   out[l][j][s] = sum_{t < k} in[l][b0 + j k + t][s],   j < nb / k,
// exact in 32-bit integers; the caller guarantees the sums fit 16 bits.
// Streaming and HBM-bound: each thread owns eight consecutive samples of one
// output band (one 16-byte load per input band, one 16-byte store), so every
// load and store of a wave is a contiguous run of the row.
#include "rx_dev.h"

namespace rxk {

constexpr int BINNT = 256;

// 16-byte path: samples % 8 == 0 and 16-byte aligned rows
__global__ void __launch_bounds__(BINNT) k_bin_vec(const uint16_t* in, uint16_t* out, int64_t lines, int bands,
                                                   int samples, int b0, int nbo, int k) {
  const int s8 = samples / 8;
  const int64_t g = (int64_t)blockIdx.x * BINNT + threadIdx.x;   // (line, out band, 8-sample group)
  const int64_t total = lines * nbo * s8;
  if (g >= total) return;
  const int q = (int)(g % s8);
  const int64_t lj = g / s8;
  const int j = (int)(lj % nbo);
  const int64_t l = lj / nbo;
  const uint16_t* src = in + (l * bands + b0 + (int64_t)j * k) * samples + 8 * q;
  uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  for (int t = 0; t < k; ++t) {
    const uint4 w = *reinterpret_cast<const uint4*>(src + (int64_t)t * samples);
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      acc[2 * h] += v[h] & 0xffffu;
      acc[2 * h + 1] += v[h] >> 16;
    }
  }
  uint4 o;
  o.x = acc[0] | (acc[1] << 16);
  o.y = acc[2] | (acc[3] << 16);
  o.z = acc[4] | (acc[5] << 16);
  o.w = acc[6] | (acc[7] << 16);
  *reinterpret_cast<uint4*>(out + (l * nbo + j) * samples + 8 * q) = o;
}

// any shape: one sample per thread
__global__ void __launch_bounds__(BINNT) k_bin_any(const uint16_t* in, uint16_t* out, int64_t lines, int bands,
                                                   int samples, int b0, int nbo, int k) {
  const int64_t g = (int64_t)blockIdx.x * BINNT + threadIdx.x;
  const int64_t total = lines * nbo * samples;
  if (g >= total) return;
  const int s = (int)(g % samples);
  const int64_t lj = g / samples;
  const int j = (int)(lj % nbo);
  const int64_t l = lj / nbo;
  const uint16_t* src = in + (l * bands + b0 + (int64_t)j * k) * samples + s;
  uint32_t acc = 0u;
  for (int t = 0; t < k; ++t) acc += src[(int64_t)t * samples];
  out[(l * nbo + j) * samples + s] = (uint16_t)acc;
}

}  // namespace rxk

extern "C" hipError_t rxk_launch_bin(const uint16_t* in, uint16_t* out, int64_t lines, int bands, int samples, int b0,
                                     int nbo, int k, hipStream_t st) {
  using namespace rxk;
  if (lines <= 0 || nbo <= 0) return hipSuccess;
  const bool vec = samples % 8 == 0 && (reinterpret_cast<uintptr_t>(in) & 15u) == 0 &&
                   (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
  const int64_t items = lines * nbo * (vec ? samples / 8 : samples);
  const int64_t wg = (items + BINNT - 1) / BINNT;
  if (vec) hipLaunchKernelGGL(k_bin_vec, dim3(wg), dim3(BINNT), 0, st, in, out, lines, bands, samples, b0, nbo, k);
  else hipLaunchKernelGGL(k_bin_any, dim3(wg), dim3(BINNT), 0, st, in, out, lines, bands, samples, b0, nbo, k);
  return hipGetLastError();
}
