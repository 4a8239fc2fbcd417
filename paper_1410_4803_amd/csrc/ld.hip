// Linkage-disequilibrium window kernels (section "Bit population count").
//
// For variants a < b <= a + window, with x = -1 / 0 / +1 for homozygous A1 /
// heterozygous / homozygous A2, the six sums over the samples where neither
// call is missing are six contractions over samples of per-call int8
// features (all zero for a missing call): m = 1, x, h = x^2:
//   n = <m_a, m_b>, Sx = <x_a, m_b>, Sy = <m_a, x_b>, Sxx = <h_a, m_b>,
//   Syy = <m_a, h_b>, Sxy = <x_a, x_b>.
// The main kernel runs these on the int8 matrix cores over a band of 64x64
// variant tiles and, per pair, evaluates r^2 and the emission test.  Emitted
// pairs are marked in a per-row bitmap and counted per row (atomic OR / add:
// the result does not depend on their order).  A scan turns row counts into
// offsets, and the emit kernel writes each marked pair at its offset in (a, b)
// order, recomputing its sums with popcounts over the same 2-bit words -- an
// independent integer route to the same exact values.
#include "pg_internal.h"

namespace pg {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Byte c = feature value of code c (0 homA1, 1 missing, 2 het, 3 homA2).
constexpr uint32_t kLdLutM = 0x01010001u;  //  1  0  1  1
constexpr uint32_t kLdLutX = 0x010000FFu;  // -1  0  0  1
constexpr uint32_t kLdLutH = 0x01000001u;  //  1  0  0  1

__device__ __forceinline__ void ld_spread(uint32_t w, uint32_t c[4]) {
  c[0] = w & 0x03030303u;
  c[1] = (w >> 2) & 0x03030303u;
  c[2] = (w >> 4) & 0x03030303u;
  c[3] = (w >> 6) & 0x03030303u;
}

__device__ __forceinline__ v4i ld_lookup(uint32_t lut, const uint32_t c[4]) {
  v4i r;
  r[0] = (int)__builtin_amdgcn_perm(0u, lut, c[0]);
  r[1] = (int)__builtin_amdgcn_perm(0u, lut, c[1]);
  r[2] = (int)__builtin_amdgcn_perm(0u, lut, c[2]);
  r[3] = (int)__builtin_amdgcn_perm(0u, lut, c[3]);
  return r;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static int fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return PG_OK;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
  return check_launch("fill");
}

// Emission test for one pair (a < b <= a + window, b < nv checked by the
// caller): marks bit (b - a - 1) of row a and counts it.
__device__ __forceinline__ void ld_mark(const LdScratch& sc, int64_t a, int64_t b, double r2_min,
                                        int64_t n, int64_t sx, int64_t sy, int64_t sxx,
                                        int64_t syy, int64_t sxy) {
  const double r2 = ld_r2(n, sx, sy, sxx, syy, sxy);
  if (r2 >= r2_min) {
    const int64_t d = b - a - 1;
    atomicOr(&sc.bitmap[a * sc.bm_words + (d >> 5)], 1u << (d & 31));
    atomicAdd(&sc.rowcnt[a], 1u);
  }
}

int ld_clear(const LdScratch& sc, int64_t rows_pad, hipStream_t st) {
  int rc = fill_u32(sc.bitmap, rows_pad * sc.bm_words, 0u, st);
  if (rc == PG_OK) rc = fill_u32(sc.rowcnt, rows_pad, 0u, st);
  return rc;
}

// ---- banded popcount kernel ---------------------------------------------------------
// Per 32-sample word of the planes P (homA2), Q (homA1), M (non-missing):
//   Sx  += popc(Pa & Mb) - popc(Qa & Mb),  Sxx += popc(Pa & Mb) + popc(Qa & Mb),
//   Sy  += popc(Pb & Ma) - popc(Qb & Ma),  Syy += popc(Pb & Ma) + popc(Qb & Ma),
//   n   += popc(Ma & Mb),
//   Sxy += popc((Pa & Pb) | (Qa & Qb)) - popc((Pa & Qb) | (Qa & Pb)).
// (x*y is +1 for equal homozygotes, -1 for opposite ones, 0 otherwise.)
// Block: 256 threads over a 64x64 tile, 4x4 pairs per thread.
constexpr int kLP = 64;
constexpr int kLPW = kLdPopcKWords;

__global__ __launch_bounds__(256) void k_ld_popc(const uint32_t* __restrict__ P, int64_t words_pad,
                                                 int64_t nv, int64_t rows_pad, int64_t n_band,
                                                 int32_t window, double r2_min, LdScratch sc) {
  const int64_t n_row_tiles = rows_pad / kLP;
  const int64_t I = (int64_t)blockIdx.x / n_band;
  const int64_t J = I + (int64_t)blockIdx.x % n_band;
  if (J >= n_row_tiles) return;
  __shared__ __attribute__((aligned(16))) uint32_t sA[kLPW * 3 * kLP];
  __shared__ __attribute__((aligned(16))) uint32_t sB[kLPW * 3 * kLP];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  uint32_t al[4][4], be[4][4], ga[4][4], de[4][4], cn[4][4], sp[4][4], sm[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) al[r][c] = be[r][c] = ga[r][c] = de[r][c] = cn[r][c] = sp[r][c] = sm[r][c] = 0;

  for (int64_t kc = 0; kc < words_pad; kc += kLPW) {
    for (int h = 0; h < 3; ++h) {
      const int e = t + 256 * h;
      const int row = e >> 4;
      const int col = (e & 15) * 4;
      const int64_t gw = (kc * 3 + row) * rows_pad;
      const uint4 a = *reinterpret_cast<const uint4*>(P + gw + I * kLP + col);
      const uint4 b = *reinterpret_cast<const uint4*>(P + gw + J * kLP + col);
      *reinterpret_cast<uint4*>(&sA[row * kLP + col]) = a;
      *reinterpret_cast<uint4*>(&sB[row * kLP + col]) = b;
    }
    __syncthreads();
#pragma unroll 2
    for (int w = 0; w < kLPW; ++w) {
      const uint4 ap = *reinterpret_cast<const uint4*>(&sA[(w * 3 + 0) * kLP + ty * 4]);
      const uint4 aq = *reinterpret_cast<const uint4*>(&sA[(w * 3 + 1) * kLP + ty * 4]);
      const uint4 am = *reinterpret_cast<const uint4*>(&sA[(w * 3 + 2) * kLP + ty * 4]);
      const uint4 bp = *reinterpret_cast<const uint4*>(&sB[(w * 3 + 0) * kLP + tx * 4]);
      const uint4 bq = *reinterpret_cast<const uint4*>(&sB[(w * 3 + 1) * kLP + tx * 4]);
      const uint4 bm = *reinterpret_cast<const uint4*>(&sB[(w * 3 + 2) * kLP + tx * 4]);
      const uint32_t AP[4] = {ap.x, ap.y, ap.z, ap.w}, AQ[4] = {aq.x, aq.y, aq.z, aq.w},
                     AM[4] = {am.x, am.y, am.z, am.w};
      const uint32_t BP[4] = {bp.x, bp.y, bp.z, bp.w}, BQ[4] = {bq.x, bq.y, bq.z, bq.w},
                     BM[4] = {bm.x, bm.y, bm.z, bm.w};
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          al[r][c] += __builtin_popcount(AP[r] & BM[c]);
          be[r][c] += __builtin_popcount(AQ[r] & BM[c]);
          ga[r][c] += __builtin_popcount(BP[c] & AM[r]);
          de[r][c] += __builtin_popcount(BQ[c] & AM[r]);
          cn[r][c] += __builtin_popcount(AM[r] & BM[c]);
          sp[r][c] += __builtin_popcount((AP[r] & BP[c]) | (AQ[r] & BQ[c]));
          sm[r][c] += __builtin_popcount((AP[r] & BQ[c]) | (AQ[r] & BP[c]));
        }
    }
    __syncthreads();
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      const int64_t a = I * kLP + ty * 4 + r;
      const int64_t b = J * kLP + tx * 4 + c;
      if (!(a < b && b - a <= window && b < nv)) continue;
      ld_mark(sc, a, b, r2_min, cn[r][c], (int64_t)al[r][c] - be[r][c],
              (int64_t)ga[r][c] - de[r][c], (int64_t)al[r][c] + be[r][c],
              (int64_t)ga[r][c] + de[r][c], (int64_t)sp[r][c] - sm[r][c]);
    }
}

int launch_ld_popc(const uint32_t* P, int64_t words_pad, int64_t nv, int64_t rows_pad,
                   int32_t window, double r2_min, const LdScratch& sc, hipStream_t st) {
  const int64_t n_band = ((int64_t)window + kLP - 1) / kLP + 1;
  const int64_t blocks = rows_pad / kLP * n_band;
  hipLaunchKernelGGL(k_ld_popc, dim3((unsigned)blocks), dim3(256), 0, st, P, words_pad, nv,
                     rows_pad, n_band, window, r2_min, sc);
  int rc = check_launch("ld_popc");
  mark_stage(2, st);
  return rc;
}

// ---- banded matrix-core kernel ----------------------------------------------------
// Block: 256 threads = 4 waves (2x2) over a 64x64 tile (rows a, columns b);
// each wave owns one 32x32 block and six v_mfma_i32_32x32x32_i8 accumulators.
// K runs over samples in chunks of 16 words (256 samples): the next chunk is
// fetched into registers while the current one is consumed from one of two
// LDS buffers, and the features of step s+1 are expanded while the MFMAs of
// step s run.  A wave whose 32x32 block has no pair inside the window skips
// its MFMAs (it still helps stage the tiles).
constexpr int kL = kLdTile;
constexpr int kLW = kLdKWords;
constexpr int kLStride = kLW + 4;

struct Feat3 {
  v4i m, x, h;
};

__device__ __forceinline__ Feat3 ld_expand(uint32_t word) {
  uint32_t c[4];
  ld_spread(word, c);
  return Feat3{ld_lookup(kLdLutM, c), ld_lookup(kLdLutX, c), ld_lookup(kLdLutH, c)};
}

__global__ __launch_bounds__(256, 2) void k_ld_mfma(const uint32_t* __restrict__ D, int64_t wn,
                                                 int64_t nv, int64_t n_row_tiles, int64_t n_band,
                                                 int32_t window, double r2_min, LdScratch sc) {
  const int64_t I = (int64_t)blockIdx.x / n_band;
  const int64_t J = I + (int64_t)blockIdx.x % n_band;
  if (J >= n_row_tiles) return;
  __shared__ __attribute__((aligned(16))) uint32_t sA[2][kL * kLStride];
  __shared__ __attribute__((aligned(16))) uint32_t sB[2][kL * kLStride];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int g = lane >> 5;
  const int rl = lane & 31;
  // does this wave's 32x32 block hold any pair a < b <= a + window?
  const int64_t a_lo = I * kL + wr * 32, b_lo = J * kL + wc * 32;
  const bool active = (b_lo + 31 > a_lo) && (b_lo - (a_lo + 31) <= window) && (b_lo < nv);

  const int lrow = t >> 2;
  const int lq = (t & 3) * 4;
  const uint32_t* pa = D + (I * kL + lrow) * wn + lq;
  const uint32_t* pb = D + (J * kL + lrow) * wn + lq;
  uint4 ga, gb;
  auto gload = [&](int64_t kc) {
    ga = *reinterpret_cast<const uint4*>(pa + kc);
    gb = *reinterpret_cast<const uint4*>(pb + kc);
  };
  auto lstore = [&](int buf) {
    *reinterpret_cast<uint4*>(&sA[buf][lrow * kLStride + lq]) = ga;
    *reinterpret_cast<uint4*>(&sB[buf][lrow * kLStride + lq]) = gb;
  };

  v16i s_n = (v16i){0}, s_x = (v16i){0}, s_y = (v16i){0};
  v16i s_xx = (v16i){0}, s_yy = (v16i){0}, s_xy = (v16i){0};
  const int64_t nchunks = wn / kLW;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int64_t k = 0; k < nchunks; ++k) {
    const int buf = (int)(k & 1);
    if (k + 1 < nchunks) gload((k + 1) * kLW);
    if (active) {
      const uint32_t* ra = &sA[buf][(wr * 32 + rl) * kLStride + g * 8];
      const uint32_t* rb = &sB[buf][(wc * 32 + rl) * kLStride + g * 8];
      const uint4 a0 = *reinterpret_cast<const uint4*>(ra);
      const uint4 a1 = *reinterpret_cast<const uint4*>(ra + 4);
      const uint4 b0 = *reinterpret_cast<const uint4*>(rb);
      const uint4 b1 = *reinterpret_cast<const uint4*>(rb + 4);
      const uint32_t wa[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
      const uint32_t wb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
      Feat3 fa = ld_expand(wa[0]), fb = ld_expand(wb[0]);
#pragma unroll
      for (int s = 0; s < kLW / 2; ++s) {
        Feat3 na, nb;
        if (s + 1 < kLW / 2) {
          na = ld_expand(wa[s + 1]);
          nb = ld_expand(wb[s + 1]);
        }
        s_n = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa.m, fb.m, s_n, 0, 0, 0);
        s_x = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa.x, fb.m, s_x, 0, 0, 0);
        s_y = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa.m, fb.x, s_y, 0, 0, 0);
        s_xx = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa.h, fb.m, s_xx, 0, 0, 0);
        s_yy = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa.m, fb.h, s_yy, 0, 0, 0);
        s_xy = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa.x, fb.x, s_xy, 0, 0, 0);
        if (s + 1 < kLW / 2) {
          fa = na;
          fb = nb;
        }
      }
    }
    if (k + 1 < nchunks) lstore(buf ^ 1);
    __syncthreads();
  }
  if (!active) return;

  // 32x32 accumulator layout: register v of lane l holds row
  // 8*(v/4) + 4*(l/32) + v%4 and column l%32.
  for (int v = 0; v < 16; ++v) {
    const int64_t a = a_lo + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int64_t b = b_lo + (lane & 31);
    if (!(a < b && b - a <= window && b < nv)) continue;
    ld_mark(sc, a, b, r2_min, s_n[v], s_x[v], s_y[v], s_xx[v], s_yy[v], s_xy[v]);
  }
}

int launch_ld_mfma(const uint32_t* D, int64_t wn, int64_t nv, int64_t rows_pad, int32_t window,
                   double r2_min, const LdScratch& sc, hipStream_t st) {
  int rc;
  const int64_t n_row_tiles = rows_pad / kL;
  const int64_t n_band = ((int64_t)window + kL - 1) / kL + 1;
  const int64_t blocks = n_row_tiles * n_band;
  hipLaunchKernelGGL(k_ld_mfma, dim3((unsigned)blocks), dim3(256), 0, st, D, wn, nv, n_row_tiles,
                     n_band, window, r2_min, sc);
  rc = check_launch("ld_mfma");
  mark_stage(2, st);
  return rc;
}

// ---- scan: row counts -> row offsets, total -> *n_out ----------------------------
// Three passes: per-block sums (4096 rows per block), one block scanning the
// block sums, then per-block exclusive scans plus the block's offset.
constexpr int kScanPer = 16;                  // rows per thread
constexpr int kScanBlock = 256 * kScanPer;    // rows per block

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < (int)blockDim.x; d <<= 1) {
    const int64_t add = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int64_t incl = sh[t];
  if (total) *total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_sums(const uint32_t* __restrict__ cnt, int64_t nv,
                                                   int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  int64_t s = 0;
  for (int i = 0; i < kScanPer; ++i)
    if (base + i < nv) s += cnt[base + i];
  int64_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int64_t* __restrict__ bsum, int64_t nb,
                                                   int64_t nv, int64_t* __restrict__ off,
                                                   int64_t* n_out) {
  __shared__ int64_t sh[1024];
  const int64_t per = ceil_div(nb, 1024);
  const int64_t lo = threadIdx.x * per;
  int64_t s = 0;
  for (int64_t i = lo; i < lo + per && i < nb; ++i) s += bsum[i];
  int64_t tot;
  int64_t run = block_exclusive_scan(s, sh, &tot);
  for (int64_t i = lo; i < lo + per && i < nb; ++i) {
    const int64_t v = bsum[i];
    bsum[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) {
    off[nv] = tot;
    *n_out = tot;
  }
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ cnt, int64_t nv,
                                                    const int64_t* __restrict__ bsum,
                                                    int64_t* __restrict__ off) {
  __shared__ int64_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  int64_t s = 0;
  for (int i = 0; i < kScanPer; ++i)
    if (base + i < nv) s += cnt[base + i];
  int64_t run = block_exclusive_scan(s, sh, nullptr) + bsum[blockIdx.x];
  for (int i = 0; i < kScanPer; ++i)
    if (base + i < nv) {
      off[base + i] = run;
      run += cnt[base + i];
    }
}

// ---- emit: one record per thread ---------------------------------------------------
// Record r (< min(total, capacity)) belongs to the row a with off[a] <= r <
// off[a+1] (binary search), and to the (r - off[a])-th marked bit of that
// row's bitmap.  Its sums are recomputed with popcounts over the operand the
// pair kernel used (2-bit words or bit planes) -- an independent integer route
// to the same exact values.
struct Sums6 {
  int n, sx, sy, sxx, syy, sxy;
};

__device__ __forceinline__ void add_plane_sums(Sums6& z, uint32_t pa, uint32_t qa, uint32_t ma,
                                               uint32_t pb, uint32_t qb, uint32_t mb) {
  z.n += __builtin_popcount(ma & mb);
  z.sx += __builtin_popcount(pa & mb) - __builtin_popcount(qa & mb);
  z.sy += __builtin_popcount(pb & ma) - __builtin_popcount(qb & ma);
  z.sxx += __builtin_popcount((pa | qa) & mb);
  z.syy += __builtin_popcount((pb | qb) & ma);
  z.sxy += __builtin_popcount((pa & pb) | (qa & qb)) - __builtin_popcount((pa & qb) | (qa & pb));
}

// 2-bit word (16 codes) -> the three indicator masks at the even bit positions.
__device__ __forceinline__ void masks_of_word(uint32_t x, uint32_t& p, uint32_t& q, uint32_t& m) {
  const uint32_t lo = x & 0x55555555u, hi = (x >> 1) & 0x55555555u;
  p = lo & hi;                       // homA2
  q = ~(lo | hi) & 0x55555555u;      // homA1
  m = ~(lo & ~hi) & 0x55555555u;     // not code 01
}

template <bool kPlanes>
__global__ __launch_bounds__(256) void k_ld_emit(const uint32_t* __restrict__ X, int64_t words,
                                                 int64_t rows_pad, int64_t nv, int64_t v0,
                                                 LdScratch sc, pg_ld_pair* __restrict__ out,
                                                 int64_t capacity) {
  const int64_t total = sc.rowoff[nv] < capacity ? sc.rowoff[nv] : capacity;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nv;                       // find last a with off[a] <= r
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (sc.rowoff[mid] <= r) lo = mid; else hi = mid;
    }
    const int64_t a = lo;
    int64_t k = r - sc.rowoff[a];
    int64_t b = -1;
    for (int64_t q = 0; q < sc.bm_words; ++q) {
      uint32_t bits = sc.bitmap[a * sc.bm_words + q];
      const int pc = __builtin_popcount(bits);
      if (k < pc) {
        for (; k > 0; --k) bits &= bits - 1;
        b = a + 1 + q * 32 + __builtin_ctz(bits);
        break;
      }
      k -= pc;
    }
    if (b < 0) continue;   // unreachable when counts and bitmap agree
    Sums6 z{0, 0, 0, 0, 0, 0};
    if constexpr (kPlanes) {
      for (int64_t w = 0; w < words; ++w) {
        const uint32_t* pw = X + w * 3 * rows_pad;
        add_plane_sums(z, pw[a], pw[rows_pad + a], pw[2 * rows_pad + a], pw[b],
                       pw[rows_pad + b], pw[2 * rows_pad + b]);
      }
    } else {
      const uint4* ra = reinterpret_cast<const uint4*>(X + a * words);
      const uint4* rb = reinterpret_cast<const uint4*>(X + b * words);
      for (int64_t w4 = 0; w4 < words / 4; ++w4) {
        const uint4 A = ra[w4], B = rb[w4];
        const uint32_t xs[4] = {A.x, A.y, A.z, A.w}, ys[4] = {B.x, B.y, B.z, B.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          uint32_t pa, qa, ma, pb, qb, mb;
          masks_of_word(xs[e], pa, qa, ma);
          masks_of_word(ys[e], pb, qb, mb);
          add_plane_sums(z, pa, qa, ma, pb, qb, mb);
        }
      }
    }
    pg_ld_pair rec;
    rec.a = (int32_t)(v0 + a);
    rec.b = (int32_t)(v0 + b);
    rec.n = z.n; rec.sx = z.sx; rec.sy = z.sy; rec.sxx = z.sxx; rec.syy = z.syy; rec.sxy = z.sxy;
    rec.r2 = ld_r2(z.n, z.sx, z.sy, z.sxx, z.syy, z.sxy);
    out[r] = rec;
  }
}

int ld_scan_blocks(int64_t nv) { return (int)ceil_div(nv, kScanBlock); }

int launch_ld_finish(const uint32_t* X, bool planes, int64_t words, int64_t rows_pad, int64_t nv,
                     int64_t v0, const LdScratch& sc, pg_ld_pair* out, int64_t capacity,
                     int64_t* n_out, hipStream_t st) {
  const int64_t nb = ceil_div(nv, kScanBlock);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, st, sc.rowcnt, nv, sc.bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, sc.bsum, nb, nv, sc.rowoff, n_out);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, sc.rowcnt, nv, sc.bsum,
                     sc.rowoff);
  int rc = check_launch("ld_scan");
  mark_stage(3, st);
  if (rc == PG_OK && capacity > 0) {
    if (planes)
      hipLaunchKernelGGL(k_ld_emit<true>, dim3(2048), dim3(256), 0, st, X, words, rows_pad, nv, v0,
                         sc, out, capacity);
    else
      hipLaunchKernelGGL(k_ld_emit<false>, dim3(2048), dim3(256), 0, st, X, words, rows_pad, nv, v0,
                         sc, out, capacity);
    rc = check_launch("ld_emit");
  }
  mark_stage(4, st);
  return rc;
}

}  // namespace pg
