// Layout kernels: turn the caller's variant-major .bed selection into the
// operand layouts of the pair kernels.  All are single passes over the input,
// bound by HBM traffic.  Padding positions are written as missing calls, so
// they contribute nothing to any count.
#include "tiles.h"

namespace pg {

// ---- helpers for whole-matrix selections (no sample list) -------------------
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
  // bit k -> bit 2k, for the low 16 bits
  x &= 0xFFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// Word g of selected variant v: sixteen consecutive samples of the row as a
// 2-bit word (sample 16g + k at bits 2k), with the missing mask applied and
// samples >= m (and variants >= nv) forced to missing.  This reads the words
// of N (v, g) pairs and issues every load before any result is used (a reader
// that branches per word waits on each load in turn).  Dword-aligned rows take
// one dword per word, other rows two aligned dwords, shifted; a word whose
// dwords would leave the selected rows (a row's last partial dword, the edges
// of the selection) is read byte by byte afterwards.  Words read in place of
// those come from the first dwords of the selection and are discarded.
template <int N>
__device__ __forceinline__ void row_words16(const Sel& s, const int64_t (&v)[N],
                                            const int64_t (&g)[N], bool aligned,
                                            uint32_t (&w)[N]) {
  const uint8_t* first = s.bed + s.v0 * s.bpv;
  const uint8_t* end = first + s.nv * s.bpv;
  const uint8_t* safe =
      reinterpret_cast<const uint8_t*>((reinterpret_cast<uintptr_t>(first) + 3) & ~(uintptr_t)3);
  const bool loads = aligned ? s.nv > 0 && s.bpv >= 4 : safe + 8 <= end;   // same for all lanes
  bool fast[N];
  uint32_t lo[N], hi[N];
  if (loads && aligned) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const uint8_t* p = first + v[r] * s.bpv + 4 * g[r];
      fast[r] = v[r] < s.nv && s.bpv - 4 * g[r] >= 4;
      lo[r] = *reinterpret_cast<const uint32_t*>(fast[r] ? p : first);
      hi[r] = 0;
    }
  } else if (loads) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const uint8_t* p = first + v[r] * s.bpv + 4 * g[r];
      const uint8_t* pa =
          reinterpret_cast<const uint8_t*>(reinterpret_cast<uintptr_t>(p) & ~(uintptr_t)3);
      fast[r] = v[r] < s.nv && s.bpv - 4 * g[r] >= 4 && pa >= first && pa + 8 <= end;
      const uint32_t* q = reinterpret_cast<const uint32_t*>(fast[r] ? pa : safe);
      lo[r] = q[0];
      hi[r] = q[1];
    }
  } else {
#pragma unroll
    for (int r = 0; r < N; ++r) { fast[r] = false; lo[r] = hi[r] = 0; }
  }
  uint64_t mw[N];
  if (s.mask) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const bool in = v[r] < s.nv && s.m - 16 * g[r] > 0;
      mw[r] = s.mask[in ? (s.v0 + v[r]) * s.wpm + ((16 * g[r]) >> 6) : 0];
    }
  }
#pragma unroll
  for (int r = 0; r < N; ++r) {
    uint32_t x;
    if (fast[r]) {
      const uintptr_t p = reinterpret_cast<uintptr_t>(first + v[r] * s.bpv + 4 * g[r]);
      x = aligned ? lo[r] : (uint32_t)((((uint64_t)hi[r] << 32) | lo[r]) >> (8 * (p & 3)));
    } else if (v[r] >= s.nv) {
      x = kAllMissing16;
    } else {
      const uint8_t* p = first + v[r] * s.bpv + 4 * g[r];
      const int64_t avail = s.bpv - 4 * g[r];
      x = 0;
      for (int b = 0; b < 4; ++b)
        if (b < avail) x |= (uint32_t)p[b] << (8 * b);
    }
    const int64_t valid = s.m - 16 * g[r];
    if (valid < 16) {
      const uint32_t keep = valid <= 0 ? 0u : ((1u << (2 * valid)) - 1u);
      x = (x & keep) | (kAllMissing16 & ~keep);
    }
    if (s.mask && valid > 0 && v[r] < s.nv) {
      const uint32_t lanes = spread16((uint32_t)(mw[r] >> ((16 * g[r]) & 63)));
      x = (x & ~(lanes | (lanes << 1))) | lanes;  // masked calls -> code 01
    }
    w[r] = x;
  }
}

// Sample-major 2-bit words without a sample list, 512 samples x 256 variants
// per block: lanes read consecutive words of one .bed row (whole lines), the
// 16x16 transposes land in LDS, and the block writes 64-byte runs of T rows.
// The block's 34 KB of LDS let four blocks share a CU (512 x 512 blocks, 68
// KB: two per CU, 17% slower at 10,000 x 100,000).
// Samples past the matrix and variants past the selection are missing calls.
constexpr int kSmTG = 32;            // sample groups (16 samples) per block
constexpr int kSmTW = 16;            // T words (16 variants) per block
constexpr int kSmTS = kSmTW + 1;     // LDS row stride (words)

// Block `bid` of the tiled layout of one operand.
__device__ __forceinline__ void sample_major_tiled_block(const Sel& s, uint32_t* __restrict__ T,
                                                         int64_t rows_pad, int64_t wp,
                                                         int aligned, int64_t bid,
                                                         uint32_t* s_out) {
  const int64_t nb_g = ceil_div(rows_pad / 16, kSmTG);
  const int64_t g0 = (bid % nb_g) * kSmTG;   // sample group (16 samples)
  const int64_t a0 = (bid / nb_g) * kSmTW;   // T word (16 variants)
  const int t = threadIdx.x;
  const int gl = t % kSmTG;
#pragma unroll 1
  for (int i = 0; i < kSmTW / 8; ++i) {
    const int al = t / kSmTG + 8 * i;
    const int64_t a = a0 + al, g = g0 + gl;
    int64_t vr[16], gr[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) { vr[r] = 16 * a + r; gr[r] = g; }   // (16 wp >= nv)
    uint32_t x[16];
    row_words16(s, vr, gr, aligned != 0, x);
    transpose16_2bit(x);
#pragma unroll
    for (int c = 0; c < 16; ++c) s_out[(c * kSmTG + gl) * kSmTS + al] = x[c];
  }
  __syncthreads();
  for (int e = t; e < 16 * kSmTG * kSmTW; e += 256) {
    const int row = e / kSmTW, col = e % kSmTW;
    const int64_t k = 16 * g0 + row, a = a0 + col;
    if (k < rows_pad && a < wp)   // T row 16 gl + c is LDS row c * kSmTG + gl
      T[k * wp + a] = s_out[((row & 15) * kSmTG + (row >> 4)) * kSmTS + col];
  }
}

__global__ __launch_bounds__(256) void k_sample_major_tiled(Sel s, uint32_t* __restrict__ T,
                                                            int64_t rows_pad, int64_t wp,
                                                            int aligned) {
  __shared__ uint32_t s_out[16 * kSmTG * kSmTS];
  // blocks of one XCD take consecutive sample groups of the same variants, so
  // the row pieces that straddle two blocks' reads meet in that XCD's L2
  sample_major_tiled_block(s, T, rows_pad, wp, aligned, xcd_swizzle(blockIdx.x, gridDim.x),
                           s_out);
}

// Many operands in one launch: block b lays out block b - block_begin of the
// job whose block range holds b (jobs in increasing block_begin).
__global__ __launch_bounds__(256) void k_sample_major_jobs(const LayoutJob* __restrict__ jobs,
                                                           int n_jobs) {
  __shared__ uint32_t s_out[16 * kSmTG * kSmTS];
  const int64_t b = blockIdx.x;
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {   // the last job with block_begin <= b
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  const LayoutJob j = jobs[lo];
  sample_major_tiled_block(j.s, j.T, j.rows_pad, j.wp, j.aligned, b - j.block_begin, s_out);
}

int64_t sample_major_job_blocks(int64_t rows_pad, int64_t wp) {
  return ceil_div(wp, kSmTW) * ceil_div(rows_pad, 16 * kSmTG);
}

int launch_sample_major_jobs(const LayoutJob* jobs, int n_jobs, int64_t total_blocks,
                             hipStream_t st) {
  if (n_jobs <= 0 || total_blocks <= 0) return PG_OK;
  hipLaunchKernelGGL(k_sample_major_jobs, dim3((unsigned)total_blocks), dim3(256), 0, st, jobs,
                     n_jobs);
  return check_launch("sample_major_jobs");
}

// Every other bit (bits 0, 2, 4, ... of x) packed into the low 16 bits.
__device__ __forceinline__ uint32_t compact_even_bits(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  x = (x | (x >> 8)) & 0x0000FFFFu;
  return x;
}

// Bit planes without a sample list: a thread owns 16 samples x 32 variants
// (two 16x16 transposes), then splits each sample's 32 codes into the high
// bit, low bit and non-missing planes; it writes 16 consecutive samples of
// each plane word.
__global__ __launch_bounds__(256) void k_ibs_planes_fast(Sel s, uint32_t* __restrict__ P,
                                                         int64_t rows_pad, int64_t words_pad,
                                                         int aligned) {
  const int64_t groups = rows_pad / 16;
  const int64_t total = groups * words_pad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = e % groups;
    const int64_t w = e / groups;
    uint32_t lo16[16], hi16[16];
    int64_t vr[16], gr[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) { vr[r] = 32 * w + r; gr[r] = g; }
    row_words16(s, vr, gr, aligned != 0, lo16);
#pragma unroll
    for (int r = 0; r < 16; ++r) vr[r] += 16;
    row_words16(s, vr, gr, aligned != 0, hi16);
    transpose16_2bit(lo16);
    transpose16_2bit(hi16);
    uint32_t H[16], L[16], M[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const uint32_t a = lo16[c], b = hi16[c];   // variants 0-15 and 16-31 of sample c
      const uint32_t miss_a = a & ~(a >> 1) & 0x55555555u;   // code 01
      const uint32_t miss_b = b & ~(b >> 1) & 0x55555555u;
      H[c] = compact_even_bits(a >> 1) | (compact_even_bits(b >> 1) << 16);
      L[c] = compact_even_bits(a) | (compact_even_bits(b) << 16);
      M[c] = ~(compact_even_bits(miss_a) | (compact_even_bits(miss_b) << 16));
    }
    uint32_t* dst = P + (w * 3) * rows_pad + 16 * g;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<uint4*>(dst + 4 * q) = make_uint4(H[4 * q], H[4 * q + 1], H[4 * q + 2], H[4 * q + 3]);
      *reinterpret_cast<uint4*>(dst + rows_pad + 4 * q) =
          make_uint4(L[4 * q], L[4 * q + 1], L[4 * q + 2], L[4 * q + 3]);
      *reinterpret_cast<uint4*>(dst + 2 * rows_pad + 4 * q) =
          make_uint4(M[4 * q], M[4 * q + 1], M[4 * q + 2], M[4 * q + 3]);
    }
  }
}

// Variant-major bit planes for the popcount LD path: for 32-sample word w,
// plane p (0 = homozygous A2, 1 = homozygous A1, 2 = non-missing) of selected
// variant v at P[(w*3 + p)*rows_pad + v].  One plane word per thread.
__device__ __forceinline__ void ld_planes_of(uint32_t x, uint32_t& hom2, uint32_t& hom1,
                                             uint32_t& nonmiss) {
  const uint32_t lo = x & 0x55555555u, hi = (x >> 1) & 0x55555555u;
  hom2 = compact_even_bits(lo & hi);
  hom1 = compact_even_bits(~(lo | hi) & 0x55555555u);
  nonmiss = compact_even_bits(~(lo & ~hi) & 0x55555555u);
}

__global__ __launch_bounds__(256) void k_ld_planes(Sel s, uint32_t* __restrict__ P, int64_t rows_pad,
                                                   int64_t words_pad) {
  const int64_t total = rows_pad * words_pad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = e % rows_pad;
    const int64_t w = e / rows_pad;
    uint32_t x0 = 0, x1 = 0;
    for (int b = 0; b < 16; ++b) {
      x0 |= code_at(s, v, 32 * w + b) << (2 * b);
      x1 |= code_at(s, v, 32 * w + 16 + b) << (2 * b);
    }
    uint32_t p0, q0, m0, p1, q1, m1;
    ld_planes_of(x0, p0, q0, m0);
    ld_planes_of(x1, p1, q1, m1);
    P[(w * 3 + 0) * rows_pad + v] = p0 | (p1 << 16);
    P[(w * 3 + 1) * rows_pad + v] = q0 | (q1 << 16);
    P[(w * 3 + 2) * rows_pad + v] = m0 | (m1 << 16);
  }
}

// Replicated fp4 operand: for each sample and each group of 8 variants, two
// words.  HR holds each code's high bit at nibble bits 1 and 3; LR holds its
// low bit at nibble bits 1 and 3 and ones at nibble bits 0 and 2.  Missing
// positions (and padding) are HR = 0, LR = ~0.  With this layout every fp4
// feature nibble is one three-input bit function of (HR, LR, bit-1 mask).
__device__ __forceinline__ void rep_pair(uint32_t codes8, uint32_t& hr, uint32_t& lr) {
  // codes8: 8 codes in the low 16 bits, code t at bits 2t -> code t at bits 4t (nibbles)
  uint32_t x = codes8 & 0xFFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  const uint32_t hi = (x >> 1) & 0x11111111u, lo = x & 0x11111111u;
  hr = (hi << 1) | (hi << 3);
  lr = (lo << 1) | (lo << 3) | 0x55555555u;
}

// Replicated operand without a sample list: a thread owns 16 samples x 64
// variants (four 16x16 transposes) and writes 16 words per sample row.
__global__ __launch_bounds__(256) void k_sample_major_rep(Sel s, uint32_t* __restrict__ R,
                                                          int64_t rows_pad, int64_t rp,
                                                          int aligned) {
  const int64_t groups = rows_pad / 16;
  const int64_t quads = rp / 16;               // 64 variants = 16 words per sample
  const int64_t total = groups * quads;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = e % groups;
    const int64_t q = e / groups;
    uint32_t out[4][16];
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
      const int64_t w = 4 * q + ww;
      int64_t vr[16], gr[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) { vr[r] = 16 * w + r; gr[r] = g; }
      row_words16(s, vr, gr, aligned != 0, out[ww]);
      transpose16_2bit(out[ww]);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      uint32_t v[16];
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        rep_pair(out[ww][c], v[4 * ww + 0], v[4 * ww + 1]);
        rep_pair(out[ww][c] >> 16, v[4 * ww + 2], v[4 * ww + 3]);
      }
      uint4* dst = reinterpret_cast<uint4*>(R + (16 * g + c) * rp + 16 * q);
#pragma unroll
      for (int k = 0; k < 4; ++k) dst[k] = make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    }
  }
}

// Replicated operand with a sample list: one 8-variant group per thread.
__global__ __launch_bounds__(256) void k_sample_major_rep_gather(Sel s, uint32_t* __restrict__ R,
                                                                 int64_t rows_pad, int64_t rp) {
  const int64_t ngroups = rp / 2;
  const int64_t total = rows_pad * ngroups;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ngroups;
    const int64_t q = e % ngroups;
    uint32_t codes = 0;
    for (int b = 0; b < 8; ++b) codes |= code_at(s, 8 * q + b, i) << (2 * b);
    uint32_t hr, lr;
    rep_pair(codes, hr, lr);
    R[i * rp + 2 * q] = hr;
    R[i * rp + 2 * q + 1] = lr;
  }
}

// Variant-major 2-bit words without a sample list: a wave owns 64 * kVmU
// consecutive words of D (rows run on into each other), with their loads in
// flight together.
constexpr int kVmU = 8;

__global__ __launch_bounds__(256) void k_variant_major_fast(Sel s, uint32_t* __restrict__ D,
                                                            int64_t rows_pad, int64_t wn,
                                                            int aligned) {
  const int lane = threadIdx.x & 63;
  const int64_t total = rows_pad * wn;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t e0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * kVmU);
       e0 < total; e0 += waves * (64 * kVmU)) {
    int64_t vr[kVmU], gr[kVmU];
    int64_t v = (e0 + lane) / wn, g = (e0 + lane) % wn;
#pragma unroll
    for (int u = 0; u < kVmU; ++u) {
      vr[u] = v;
      gr[u] = g;
      g += 64;
      while (g >= wn) { g -= wn; ++v; }
    }
    uint32_t x[kVmU];
    row_words16(s, vr, gr, aligned != 0, x);
#pragma unroll
    for (int u = 0; u < kVmU; ++u) {
      const int64_t e = e0 + 64 * u + lane;
      if (e < total) D[e] = x[u];
    }
  }
}

bool rows_dword_aligned(const Sel& s) {
  return (s.bpv % 4) == 0 && (reinterpret_cast<uintptr_t>(s.bed) % 4) == 0;
}

static unsigned stride_grid(int64_t items) {
  const int64_t b = ceil_div(items, 256);
  return (unsigned)(b < 65536 ? b : 65536);
}

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
  if (!s.idx) {
    const int64_t blocks = sample_major_job_blocks(rows_pad, wp);
    hipLaunchKernelGGL(k_sample_major_tiled, dim3((unsigned)blocks), dim3(256), 0, st, s, T,
                       rows_pad, wp, (int)rows_dword_aligned(s));
    return check_launch("sample_major_tiled");
  }
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
  if (!s.idx) {
    hipLaunchKernelGGL(k_ibs_planes_fast, dim3(stride_grid(rows_pad / 16 * words_pad)), dim3(256),
                       0, st, s, P, rows_pad, words_pad, (int)rows_dword_aligned(s));
    return check_launch("ibs_planes_fast");
  }
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
  if (!s.idx) {
    hipLaunchKernelGGL(k_variant_major_fast, dim3(stride_grid(ceil_div(rows_pad * wn, kVmU))),
                       dim3(256), 0, st, s, D, rows_pad, wn, (int)rows_dword_aligned(s));
    return check_launch("variant_major_fast");
  }
  dim3 grid((unsigned)ceil_div(rows_pad * wn, 256));
  hipLaunchKernelGGL(k_variant_major_2bit, grid, dim3(256), 0, st, s, D, rows_pad, wn);
  return check_launch("variant_major_2bit");
}

// LD bit planes without a sample list, staged through LDS: a block owns 64
// variants x 32 plane words (1,024 samples).  Lanes read consecutive dwords of
// one variant row (coalesced), the three 16-bit half-planes of each dword go
// to LDS, and lanes then write consecutive variants of one plane word
// (coalesced).
__global__ __launch_bounds__(256) void k_ld_planes_tiled(Sel s, uint32_t* __restrict__ P,
                                                         int64_t rows_pad, int64_t words_pad,
                                                         int aligned) {
  __shared__ uint16_t half[3][64][65];
  const int t = threadIdx.x;
  const int64_t nrb = rows_pad / 64;
  const int64_t v0 = ((int64_t)blockIdx.x % nrb) * 64;
  const int64_t w0 = ((int64_t)blockIdx.x / nrb) * 32;      // first plane word
  const int d = t & 63;                                      // 16-sample group in the block
#pragma unroll 1
  for (int k0 = 0; k0 < 16; k0 += 8) {
    int64_t vr[8], gr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { vr[k] = v0 + (t >> 6) + 4 * (k0 + k); gr[k] = 2 * w0 + d; }
    uint32_t xs[8];
    row_words16(s, vr, gr, aligned != 0, xs);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int row = (t >> 6) + 4 * (k0 + k);
      const uint32_t lo = xs[k] & 0x55555555u, hi = (xs[k] >> 1) & 0x55555555u;
      half[0][row][d] = (uint16_t)compact_even_bits(lo & hi);
      half[1][row][d] = (uint16_t)compact_even_bits(~(lo | hi) & 0x55555555u);
      half[2][row][d] = (uint16_t)compact_even_bits(~(lo & ~hi) & 0x55555555u);
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int k = 0; k < 24; ++k) {
    const int e = t + 256 * k;
    const int row = e & 63;
    const int pw = e >> 6;                                   // 0..95
    const int p = pw % 3, w = pw / 3;
    if (w0 + w < words_pad)
      P[((w0 + w) * 3 + p) * rows_pad + v0 + row] =
          (uint32_t)half[p][row][2 * w] | ((uint32_t)half[p][row][2 * w + 1] << 16);
  }
}

int launch_ld_planes(const Sel& s, uint32_t* P, int64_t rows_pad, int64_t words_pad,
                     hipStream_t st) {
  if (!s.idx) {
    const int64_t blocks = (rows_pad / 64) * ceil_div(words_pad, 32);
    hipLaunchKernelGGL(k_ld_planes_tiled, dim3((unsigned)blocks), dim3(256), 0, st, s, P, rows_pad,
                       words_pad, (int)rows_dword_aligned(s));
  } else {
    hipLaunchKernelGGL(k_ld_planes, dim3(stride_grid(rows_pad * words_pad)), dim3(256), 0, st, s,
                       P, rows_pad, words_pad);
  }
  return check_launch("ld_planes");
}

int launch_sample_major_rep(const Sel& s, uint32_t* R, int64_t rows_pad, int64_t rp,
                            hipStream_t st) {
  if (!s.idx) {
    hipLaunchKernelGGL(k_sample_major_rep, dim3(stride_grid(rows_pad / 16 * (rp / 16))), dim3(256),
                       0, st, s, R, rows_pad, rp, (int)rows_dword_aligned(s));
  } else {
    hipLaunchKernelGGL(k_sample_major_rep_gather, dim3(stride_grid(rows_pad * (rp / 2))), dim3(256),
                       0, st, s, R, rows_pad, rp);
  }
  return check_launch("sample_major_rep");
}

}  // namespace pg
