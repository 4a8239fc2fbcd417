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

__global__ __launch_bounds__(256) void k_ld_mfma(const uint32_t* __restrict__ D, int64_t wn,
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
    const double r2 = ld_r2(s_n[v], s_x[v], s_y[v], s_xx[v], s_yy[v], s_xy[v]);
    if (r2 >= r2_min) {
      const int64_t d = b - a - 1;
      atomicOr(&sc.bitmap[a * sc.bm_words + (d >> 5)], 1u << (d & 31));
      atomicAdd(&sc.rowcnt[a], 1u);
    }
  }
}

int launch_ld_mfma(const uint32_t* D, int64_t wn, int64_t nv, int64_t rows_pad, int32_t window,
                   double r2_min, const LdScratch& sc, hipStream_t st) {
  int rc = fill_u32(sc.bitmap, rows_pad * sc.bm_words, 0u, st);
  if (rc == PG_OK) rc = fill_u32(sc.rowcnt, rows_pad, 0u, st);
  if (rc != PG_OK) return rc;
  mark_stage(1, st);
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
// row's bitmap.  Its sums are recomputed with popcounts over the two rows'
// 2-bit words.
__global__ __launch_bounds__(256) void k_ld_emit(const uint32_t* __restrict__ D, int64_t wn,
                                                 int64_t nv, int64_t v0, LdScratch sc,
                                                 pg_ld_pair* __restrict__ out, int64_t capacity) {
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
    const uint4* ra = reinterpret_cast<const uint4*>(D + a * wn);
    const uint4* rb = reinterpret_cast<const uint4*>(D + b * wn);
    int cn = 0, csx = 0, csy = 0, csxx = 0, csyy = 0, csxy = 0;
    for (int64_t w4 = 0; w4 < wn / 4; ++w4) {
      const uint4 A = ra[w4], B = rb[w4];
      const uint32_t xs[4] = {A.x, A.y, A.z, A.w}, ys[4] = {B.x, B.y, B.z, B.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t xa = xs[e], xb = ys[e];
        const uint32_t la = xa & 0x55555555u, ha = (xa >> 1) & 0x55555555u;
        const uint32_t lb = xb & 0x55555555u, hb = (xb >> 1) & 0x55555555u;
        const uint32_t ma = ~(la & ~ha) & 0x55555555u;   // code != 01
        const uint32_t mb = ~(lb & ~hb) & 0x55555555u;
        const uint32_t pa = la & ha, qa = ~(la | ha) & 0x55555555u;  // homA2, homA1
        const uint32_t pb = lb & hb, qb = ~(lb | hb) & 0x55555555u;
        cn += __builtin_popcount(ma & mb);
        csx += __builtin_popcount(pa & mb) - __builtin_popcount(qa & mb);
        csy += __builtin_popcount(pb & ma) - __builtin_popcount(qb & ma);
        csxx += __builtin_popcount((pa | qa) & mb);
        csyy += __builtin_popcount((pb | qb) & ma);
        csxy += __builtin_popcount((pa & pb) | (qa & qb)) - __builtin_popcount((pa & qb) | (qa & pb));
      }
    }
    pg_ld_pair rec;
    rec.a = (int32_t)(v0 + a);
    rec.b = (int32_t)(v0 + b);
    rec.n = cn; rec.sx = csx; rec.sy = csy; rec.sxx = csxx; rec.syy = csyy; rec.sxy = csxy;
    rec.r2 = ld_r2(cn, csx, csy, csxx, csyy, csxy);
    out[r] = rec;
  }
}

int ld_scan_blocks(int64_t nv) { return (int)ceil_div(nv, kScanBlock); }

int launch_ld_finish(const uint32_t* D, int64_t wn, int64_t nv, int64_t v0, int32_t window,
                     const LdScratch& sc, pg_ld_pair* out, int64_t capacity, int64_t* n_out,
                     hipStream_t st) {
  (void)window;
  const int64_t nb = ceil_div(nv, kScanBlock);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, st, sc.rowcnt, nv, sc.bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, sc.bsum, nb, nv, sc.rowoff, n_out);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, sc.rowcnt, nv, sc.bsum,
                     sc.rowoff);
  int rc = check_launch("ld_scan");
  mark_stage(3, st);
  if (rc == PG_OK && capacity > 0) {
    hipLaunchKernelGGL(k_ld_emit, dim3(2048), dim3(256), 0, st, D, wn, nv, v0, sc, out, capacity);
    rc = check_launch("ld_emit");
  }
  mark_stage(4, st);
  return rc;
}

}  // namespace pg
