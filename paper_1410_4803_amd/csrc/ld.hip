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
#include "tiles.h"

namespace pg {

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

int fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return PG_OK;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
  return check_launch("fill");
}

int ld_clear(const LdScratch& sc, int64_t rows_pad, hipStream_t st) {
  int rc = fill_u32(sc.bitmap, rows_pad * sc.bm_words, 0u, st);
  if (rc == PG_OK) rc = fill_u32(sc.rowcnt, rows_pad, 0u, st);
  return rc;
}

__global__ __launch_bounds__(256) void k_ld_popc(const uint32_t* __restrict__ P, int64_t words_pad,
                                                 int64_t nv, int64_t rows_pad, int64_t n_band,
                                                 int32_t window, double r2_min, LdScratch sc) {
  const int64_t b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int64_t I = b / n_band;
  const int64_t J = I + b % n_band;
  if (J >= rows_pad / kLP) return;
  __shared__ __attribute__((aligned(16))) uint32_t smem[kLdPopcSmem];
  ld_popc_tile(P, words_pad, nv, rows_pad, I, J, window, r2_min, sc, (lds_t*)smem);
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

template <bool kFp4>
__global__ __launch_bounds__(256, 2) void k_ld_mfma(const uint32_t* __restrict__ D, int64_t wn,
                                                    int64_t nv, int64_t n_row_tiles, int64_t n_band,
                                                    int32_t window, double r2_min, LdScratch sc,
                                                    const int64_t* __restrict__ gsum,
                                                    const int* __restrict__ gmax,
                                                    const uint32_t* __restrict__ groups_ok,
                                                    uint32_t min_groups, int cap, int64_t budget) {
  const int64_t b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int64_t I = b / n_band;
  const int64_t J = I + b % n_band;
  if (J >= n_row_tiles) return;
  if (gsum && ld_tile_sparse(gsum, gmax, groups_ok, min_groups, I, J, cap, budget))
    return;   // the correction path's
  __shared__ __attribute__((aligned(16))) uint32_t smem[kLdMfmaSmem];
  if constexpr (kFp4)
    ld_fp4_tile_pipe(D, wn, nv, I, J, window, r2_min, sc, (lds_t*)smem);
  else
    ld_mfma_tile(D, wn, nv, I, J, window, r2_min, sc, (lds_t*)smem);
}

int launch_ld_mfma(const uint32_t* D, int64_t wn, int64_t nv, int64_t rows_pad, int32_t window,
                   double r2_min, const LdScratch& sc, hipStream_t st, const LdSparse* sp,
                   bool fp4) {
  int rc;
  const int64_t n_row_tiles = rows_pad / kL;
  const int64_t n_band = ((int64_t)window + kL - 1) / kL + 1;
  const int64_t blocks = n_row_tiles * n_band;
  hipLaunchKernelGGL(fp4 ? k_ld_mfma<true> : k_ld_mfma<false>, dim3((unsigned)blocks), dim3(256),
                     0, st, D, wn, nv, n_row_tiles,
                     n_band, window, r2_min, sc, sp ? sp->gsum : nullptr,
                     sp ? sp->gmax : nullptr, sp ? sp->groups_ok : nullptr,
                     sp ? sp->min_groups : 0u, sp ? sp->cap : 0, sp ? sp->budget : 0);
  rc = check_launch("ld_mfma");
  if (!sp) mark_stage(2, st);
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

constexpr int kEmitU = 4;

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
    // the row loops load kEmitU steps ahead, so a thread has that many
    // loads in flight instead of waiting on each
    Sums6 z{0, 0, 0, 0, 0, 0};
    if constexpr (kPlanes) {
      int64_t w = 0;
      for (; w + kEmitU <= words; w += kEmitU) {
        uint32_t v[kEmitU][6];
#pragma unroll
        for (int u = 0; u < kEmitU; ++u) {
          const uint32_t* pw = X + (w + u) * 3 * rows_pad;
          v[u][0] = pw[a]; v[u][1] = pw[rows_pad + a]; v[u][2] = pw[2 * rows_pad + a];
          v[u][3] = pw[b]; v[u][4] = pw[rows_pad + b]; v[u][5] = pw[2 * rows_pad + b];
        }
#pragma unroll
        for (int u = 0; u < kEmitU; ++u)
          add_plane_sums(z, v[u][0], v[u][1], v[u][2], v[u][3], v[u][4], v[u][5]);
      }
      for (; w < words; ++w) {
        const uint32_t* pw = X + w * 3 * rows_pad;
        add_plane_sums(z, pw[a], pw[rows_pad + a], pw[2 * rows_pad + a], pw[b],
                       pw[rows_pad + b], pw[2 * rows_pad + b]);
      }
    } else {
      const uint4* ra = reinterpret_cast<const uint4*>(X + a * words);
      const uint4* rb = reinterpret_cast<const uint4*>(X + b * words);
      auto add4 = [&z](const uint4& A, const uint4& B) {
        const uint32_t xs[4] = {A.x, A.y, A.z, A.w}, ys[4] = {B.x, B.y, B.z, B.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          uint32_t pa, qa, ma, pb, qb, mb;
          masks_of_word(xs[e], pa, qa, ma);
          masks_of_word(ys[e], pb, qb, mb);
          add_plane_sums(z, pa, qa, ma, pb, qb, mb);
        }
      };
      const int64_t n4 = words / 4;
      int64_t w4 = 0;
      for (; w4 + kEmitU <= n4; w4 += kEmitU) {
        uint4 A[kEmitU], B[kEmitU];
#pragma unroll
        for (int u = 0; u < kEmitU; ++u) { A[u] = ra[w4 + u]; B[u] = rb[w4 + u]; }
#pragma unroll
        for (int u = 0; u < kEmitU; ++u) add4(A[u], B[u]);
      }
      for (; w4 < n4; ++w4) add4(ra[w4], rb[w4]);
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
                     int64_t* n_out, hipStream_t st, bool marks) {
  const int64_t nb = ceil_div(nv, kScanBlock);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, st, sc.rowcnt, nv, sc.bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, sc.bsum, nb, nv, sc.rowoff, n_out);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, sc.rowcnt, nv, sc.bsum,
                     sc.rowoff);
  int rc = check_launch("ld_scan");
  if (marks) mark_stage(3, st);
  if (rc == PG_OK && capacity > 0) {
    if (planes)
      hipLaunchKernelGGL(k_ld_emit<true>, dim3(2048), dim3(256), 0, st, X, words, rows_pad, nv, v0,
                         sc, out, capacity);
    else
      hipLaunchKernelGGL(k_ld_emit<false>, dim3(2048), dim3(256), 0, st, X, words, rows_pad, nv, v0,
                         sc, out, capacity);
    rc = check_launch("ld_emit");
  }
  if (marks) mark_stage(4, st);
  return rc;
}

}  // namespace pg
