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

// 8-byte path: samples % 4 == 0 and 8-byte aligned rows (the imager's
// 900-sample lines): four samples per thread, one 8-byte load per input band
__global__ void __launch_bounds__(BINNT) k_bin_v4(const uint16_t* in, uint16_t* out, int64_t lines, int bands,
                                                  int samples, int b0, int nbo, int k) {
  const int s4 = samples / 4;
  const int64_t g = (int64_t)blockIdx.x * BINNT + threadIdx.x;   // (line, out band, 4-sample group)
  const int64_t total = lines * nbo * s4;
  if (g >= total) return;
  const int q = (int)(g % s4);
  const int64_t lj = g / s4;
  const int j = (int)(lj % nbo);
  const int64_t l = lj / nbo;
  const uint16_t* src = in + (l * bands + b0 + (int64_t)j * k) * samples + 4 * q;
  uint32_t acc[4] = {0u, 0u, 0u, 0u};
  for (int t = 0; t < k; ++t) {
    const uint2 w = *reinterpret_cast<const uint2*>(src + (int64_t)t * samples);
    acc[0] += w.x & 0xffffu;
    acc[1] += w.x >> 16;
    acc[2] += w.y & 0xffffu;
    acc[3] += w.y >> 16;
  }
  *reinterpret_cast<uint2*>(out + (l * nbo + j) * samples + 4 * q) = uint2{acc[0] | (acc[1] << 16), acc[2] | (acc[3] << 16)};
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

// Band-interleaved-by-pixel lines ([line][sample][band]) to the BIL layout
// the scoring kernels read ([line][band][sample]): per line a samples x
// bands transpose through a 32 x 33 LDS tile, so both the loads (along
// bands) and the stores (along samples) are contiguous runs.  A pure copy:
// the BIL values are the BIP values bit for bit.
template <typename T>
__global__ void __launch_bounds__(256) k_bip_to_bil(const T* in, T* out, int bands, int samples) {
  __shared__ T tile[32][33];
  const int64_t l = blockIdx.z;
  const int s0 = 32 * blockIdx.x, b0 = 32 * blockIdx.y;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;      // 32 x 8
  const T* src = in + l * (int64_t)bands * samples;
  T* dst = out + l * (int64_t)bands * samples;
#pragma unroll
  for (int r = ty; r < 32; r += 8) {                           // rows = samples, columns = bands
    const int smp = s0 + r, b = b0 + tx;
    if (smp < samples && b < bands) tile[r][tx] = src[(int64_t)smp * bands + b];
  }
  __syncthreads();
#pragma unroll
  for (int r = ty; r < 32; r += 8) {                           // rows = bands, columns = samples
    const int b = b0 + r, smp = s0 + tx;
    if (smp < samples && b < bands) dst[(int64_t)b * samples + smp] = tile[tx][r];
  }
}

}  // namespace rxk

// lines of BIP [lines][samples][bands] with esz-byte values -> BIL [lines][bands][samples]
extern "C" hipError_t rxk_launch_bip_to_bil(const void* in, void* out, int64_t lines, int bands, int samples, int esz,
                                            hipStream_t st) {
  using namespace rxk;
  if (lines <= 0) return hipSuccess;
  if (lines > 65535) {                                          // grid z limit: in pieces of 65535 lines
    const int64_t stride = (int64_t)bands * samples * esz;
    for (int64_t l0 = 0; l0 < lines; l0 += 65535) {
      const int64_t n = lines - l0 < 65535 ? lines - l0 : 65535;
      hipError_t e = rxk_launch_bip_to_bil(static_cast<const char*>(in) + l0 * stride,
                                           static_cast<char*>(out) + l0 * stride, n, bands, samples, esz, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const dim3 grid((samples + 31) / 32, (bands + 31) / 32, (unsigned)lines);
  if (esz == 2) hipLaunchKernelGGL(k_bip_to_bil<uint16_t>, grid, dim3(256), 0, st, static_cast<const uint16_t*>(in),
                                   static_cast<uint16_t*>(out), bands, samples);
  else if (esz == 4) hipLaunchKernelGGL(k_bip_to_bil<float>, grid, dim3(256), 0, st, static_cast<const float*>(in),
                                        static_cast<float*>(out), bands, samples);
  else if (esz == 8) hipLaunchKernelGGL(k_bip_to_bil<double>, grid, dim3(256), 0, st, static_cast<const double*>(in),
                                        static_cast<double*>(out), bands, samples);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

extern "C" hipError_t rxk_launch_bin(const uint16_t* in, uint16_t* out, int64_t lines, int bands, int samples, int b0,
                                     int nbo, int k, hipStream_t st) {
  using namespace rxk;
  if (lines <= 0 || nbo <= 0) return hipSuccess;
  const uintptr_t al = reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out);
  const bool vec = samples % 8 == 0 && (al & 15u) == 0;
  const bool v4 = !vec && samples % 4 == 0 && (al & 7u) == 0;
  const int64_t items = lines * nbo * (vec ? samples / 8 : v4 ? samples / 4 : samples);
  const int64_t wg = (items + BINNT - 1) / BINNT;
  if (vec) hipLaunchKernelGGL(k_bin_vec, dim3(wg), dim3(BINNT), 0, st, in, out, lines, bands, samples, b0, nbo, k);
  else if (v4) hipLaunchKernelGGL(k_bin_v4, dim3(wg), dim3(BINNT), 0, st, in, out, lines, bands, samples, b0, nbo, k);
  else hipLaunchKernelGGL(k_bin_any, dim3(wg), dim3(BINNT), 0, st, in, out, lines, bands, samples, b0, nbo, k);
  return hipGetLastError();
}
