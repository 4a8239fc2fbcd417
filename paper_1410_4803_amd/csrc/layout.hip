// Layout kernels: turn the caller's variant-major .bed selection into the
// operand layouts of the pair kernels.  All are single passes over the input,
// bound by HBM traffic.  Padding positions are written as missing calls, so
// they contribute nothing to any count.
#include "pg_internal.h"

namespace pg {

// ---- sample-major 2-bit words (IBS, matrix-core path) -----------------------
// A block owns 64 samples x 64 words (1024 variants).  Each thread packs 16
// words of one sample from byte reads (a wave reads 16 consecutive bytes per
// variant row), parks them in LDS, and the block then writes each sample's 64
// words as one contiguous 256-byte run.
constexpr int kSmSamples = 64;
constexpr int kSmWords = 64;

__global__ __launch_bounds__(256) void k_sample_major_2bit(Sel s, uint32_t* __restrict__ T,
                                                           int64_t rows_pad, int64_t wp) {
  __shared__ uint32_t tile[kSmSamples][kSmWords + 1];
  const int t = threadIdx.x;
  const int64_t nbi = ceil_div(rows_pad, kSmSamples);
  const int64_t i0 = ((int64_t)blockIdx.x % nbi) * kSmSamples;
  const int64_t w0 = ((int64_t)blockIdx.x / nbi) * kSmWords;
  {
    const int li = t % kSmSamples;
    const int lw0 = (t / kSmSamples) * 16;
    const int64_t i = i0 + li;
    for (int q = 0; q < 16; ++q) {
      const int64_t w = w0 + lw0 + q;
      uint32_t word = kAllMissing16;
      if (w < wp) {
        word = 0;
        for (int b = 0; b < 16; ++b) word |= code_at(s, w * 16 + b, i) << (2 * b);
      }
      tile[li][lw0 + q] = word;
    }
  }
  __syncthreads();
  const int r = t / 4;
  const int c0 = (t % 4) * 16;
  const int64_t i = i0 + r;
  if (i < rows_pad) {
    uint32_t* dst = T + i * wp + w0 + c0;
    for (int q = 0; q < 16; ++q)
      if (w0 + c0 + q < wp) dst[q] = tile[r][c0 + q];
  }
}

int launch_sample_major_2bit(const Sel& s, uint32_t* T, int64_t rows_pad, int64_t wp,
                             hipStream_t st) {
  dim3 grid((unsigned)(ceil_div(rows_pad, kSmSamples) * ceil_div(wp, kSmWords)));
  hipLaunchKernelGGL(k_sample_major_2bit, grid, dim3(256), 0, st, s, T, rows_pad, wp);
  return check_launch("sample_major_2bit");
}

// ---- sample-major bit planes (IBS, popcount path) ---------------------------
__global__ __launch_bounds__(256) void k_ibs_planes(Sel s, uint32_t* __restrict__ P,
                                                    int64_t rows_pad, int64_t words_pad) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = g % rows_pad;
  const int64_t w = g / rows_pad;
  if (w >= words_pad) return;
  uint32_t hi = 0, lo = 0, nm = 0;
  for (int b = 0; b < 32; ++b) {
    const uint32_t c = code_at(s, w * 32 + b, i);
    hi |= (c >> 1) << b;
    lo |= (c & 1u) << b;
    nm |= (uint32_t)(c != 1u) << b;
  }
  P[(w * 3 + 0) * rows_pad + i] = hi;
  P[(w * 3 + 1) * rows_pad + i] = lo;
  P[(w * 3 + 2) * rows_pad + i] = nm;
}

int launch_ibs_planes(const Sel& s, uint32_t* P, int64_t rows_pad, int64_t words_pad,
                      hipStream_t st) {
  dim3 grid((unsigned)ceil_div(rows_pad * words_pad, 256));
  hipLaunchKernelGGL(k_ibs_planes, grid, dim3(256), 0, st, s, P, rows_pad, words_pad);
  return check_launch("ibs_planes");
}

// ---- variant-major 2-bit words (LD) -----------------------------------------
__global__ __launch_bounds__(256) void k_variant_major_2bit(Sel s, uint32_t* __restrict__ D,
                                                            int64_t rows_pad, int64_t wn) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t w = g % wn;
  const int64_t v = g / wn;
  if (v >= rows_pad) return;
  uint32_t word = 0;
  for (int b = 0; b < 16; ++b) word |= code_at(s, v, w * 16 + b) << (2 * b);
  D[v * wn + w] = word;
}

int launch_variant_major_2bit(const Sel& s, uint32_t* D, int64_t rows_pad, int64_t wn,
                              hipStream_t st) {
  dim3 grid((unsigned)ceil_div(rows_pad * wn, 256));
  hipLaunchKernelGGL(k_variant_major_2bit, grid, dim3(256), 0, st, s, D, rows_pad, wn);
  return check_launch("variant_major_2bit");
}

}  // namespace pg
