// LD-based variant pruning, the --indep-pairwise operation (section "Linkage
// disequilibrium-based variant pruning", Table 4).  The paper times it but
// does not define its greedy order; the reading implemented here:
//   windows of W consecutive variants start at 0, S, 2S, ... (the last is the
//   first that reaches the end); inside each window, pairs a < b of variants
//   still kept are visited in increasing a, then b; when r^2 > t, the variant
//   with the lower minor allele frequency is dropped (b on a tie).
//
// GPU plan.  The LD pair kernel (window W - 1, emission test r^2 > t) marks
// every pair above the threshold in its per-row bitmap.  A pair (a, b) first
// shares a window in window w(b) -- the first window whose end passes b --
// and is then visited there if a >= w(b)*S; in later windows both variants
// are either dropped already or the pair is below the threshold, so each
// window only has to visit its new pairs (b in [s_{w-1} + W, s_w + W)), in
// (a, b) order.  One block walks the (window, row) cells in that order:
// all threads extract a slice of marked pairs from the bitmap into LDS
// (with the drop side decided from the allele counts), then one thread
// applies them in order to a ring of keep bits in LDS; variants no later
// window can touch are flushed to the output as the windows advance.
#include "pg_internal.h"

namespace pg {

// ---- per-variant allele counts ---------------------------------------------
// 2-bit operand: row v holds `words` words of 16 codes; one wave per variant.
// Bit planes: plane p of word w at P[(w*3 + p)*rows_pad + v] (p = 0 homA2,
// 1 homA1, 2 non-missing); one thread per variant.
__device__ __forceinline__ int2 stats_of(int64_t hom2, int64_t hom1, int64_t nm) {
  const int64_t het = nm - hom2 - hom1;
  const int64_t a2 = 2 * hom2 + het;
  const int64_t minor = a2 < 2 * nm - a2 ? a2 : 2 * nm - a2;
  return make_int2((int)minor, nm > 0 ? (int)nm : 1);
}

__global__ __launch_bounds__(256) void k_stats_words(const uint32_t* __restrict__ D, int64_t words,
                                                     int64_t nv, int2* __restrict__ stats) {
  const int lane = threadIdx.x & 63;
  for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < nv;
       v += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const uint32_t* row = D + v * words;
    int h2 = 0, h1 = 0, nm = 0;
    for (int64_t w = lane; w < words; w += 64) {
      uint32_t p, q, m;
      masks_of_word(row[w], p, q, m);
      h2 += __builtin_popcount(p);
      h1 += __builtin_popcount(q);
      nm += __builtin_popcount(m);
    }
    for (int d = 32; d > 0; d >>= 1) {
      h2 += __shfl_xor(h2, d, 64);
      h1 += __shfl_xor(h1, d, 64);
      nm += __shfl_xor(nm, d, 64);
    }
    if (lane == 0) stats[v] = stats_of(h2, h1, nm);
  }
}

__global__ __launch_bounds__(256) void k_stats_planes(const uint32_t* __restrict__ P, int64_t words,
                                                      int64_t rows_pad, int64_t nv,
                                                      int2* __restrict__ stats) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
       v += (int64_t)gridDim.x * blockDim.x) {
    int64_t h2 = 0, h1 = 0, nm = 0;
    for (int64_t w = 0; w < words; ++w) {
      const uint32_t* pw = P + w * 3 * rows_pad + v;
      h2 += __builtin_popcount(pw[0]);
      h1 += __builtin_popcount(pw[rows_pad]);
      nm += __builtin_popcount(pw[2 * rows_pad]);
    }
    stats[v] = stats_of(h2, h1, nm);
  }
}

int launch_variant_stats(const uint32_t* X, bool planes, int64_t words, int64_t rows_pad,
                         int64_t nv, int2* stats, hipStream_t st) {
  if (planes) {
    const int64_t blocks = ceil_div(nv, 256) < 65536 ? ceil_div(nv, 256) : 65536;
    hipLaunchKernelGGL(k_stats_planes, dim3((unsigned)blocks), dim3(256), 0, st, X, words,
                       rows_pad, nv, stats);
  } else {
    const int64_t blocks = ceil_div(nv, 4) < 65536 ? ceil_div(nv, 4) : 65536;
    hipLaunchKernelGGL(k_stats_words, dim3((unsigned)blocks), dim3(256), 0, st, X, words, nv,
                       stats);
  }
  return check_launch("variant_stats");
}

// ---- the greedy pass ----------------------------------------------------------
constexpr int kPT = 1024;                 // threads of the one block
constexpr int kPCells = 16;               // (window, row) cells per thread per pass
constexpr int kPPass = kPT * kPCells;     // cells per pass
constexpr int kRingBits = 1 << 18;        // keep bits held in LDS (32 KB)
constexpr int kPBuf = 8192;               // pairs staged in LDS per slice (64 KB)

struct PruneGeom {
  int64_t nv, W, S;
};

// Cell c = (window w, row r): variant a = w*S + r and the bitmap bits
// [j0, j1) of row a (bit j <-> b = a + 1 + j) holding window w's new pairs.
__device__ __forceinline__ bool cell_bits(const PruneGeom& g, int64_t c, int64_t& a, int64_t& j0,
                                          int64_t& j1) {
  const int64_t w = c / g.W;
  const int64_t s = w * g.S;
  a = s + (c - w * g.W);
  const int64_t hi = s + g.W < g.nv ? s + g.W : g.nv;
  if (a + 1 >= hi) return false;
  const int64_t lo = w == 0 ? 0 : (g.W > g.S ? s - g.S + g.W : s);
  const int64_t d0 = lo - a > 1 ? lo - a : 1;
  const int64_t d1 = hi - a;
  if (d0 >= d1) return false;
  j0 = d0 - 1;
  j1 = d1 - 1;
  return true;
}

// Word q of a row restricted to bits [j0, j1).
__device__ __forceinline__ uint32_t seg_word(const uint32_t* row, int64_t q, int64_t j0,
                                             int64_t j1) {
  uint32_t x = row[q];
  const int64_t b0 = q * 32;
  if (j0 > b0) x &= ~0u << (j0 - b0);
  if (j1 < b0 + 32) x &= (1u << (j1 - b0)) - 1u;
  return x;
}

// Exclusive scan over the block; *total gets the block sum.
__device__ __forceinline__ int block_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (threadIdx.x < 64) {
    int s = threadIdx.x < kPT / 64 ? wsum[threadIdx.x] : 0;
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(s, d, 64);
      if (lane >= d) s += y;
    }
    if (threadIdx.x < kPT / 64) wsum[threadIdx.x] = s;
  }
  __syncthreads();
  const int base = wid ? wsum[wid - 1] : 0;
  *total = wsum[kPT / 64 - 1];
  __syncthreads();
  return base + x - v;
}

__global__ __launch_bounds__(kPT) void k_prune_greedy(const uint32_t* __restrict__ bitmap,
                                                      int64_t bm_words,
                                                      const int2* __restrict__ stats,
                                                      PruneGeom g, int64_t n_cells,
                                                      uint8_t* __restrict__ keep,
                                                      int64_t* __restrict__ n_kept) {
  __shared__ uint32_t ring[kRingBits / 32];
  __shared__ uint2 buf[kPBuf];
  __shared__ int wsum[kPT / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < kRingBits / 32; i += kPT) ring[i] = ~0u;
  __syncthreads();
  int64_t flushed = 0;
  int64_t kept = 0;
  // Writes keep flags of [flushed, to) and frees their ring bits.
  auto flush = [&](int64_t to) {
    for (int64_t x = flushed + tid; x < to; x += kPT) {
      const uint32_t ix = (uint32_t)x & (kRingBits - 1);
      const uint32_t alive = (ring[ix >> 5] >> (ix & 31)) & 1u;
      keep[x] = (uint8_t)alive;
      kept += alive;
      atomicOr(&ring[ix >> 5], 1u << (ix & 31));
    }
    flushed = to;
    __syncthreads();
  };
  for (int64_t c0 = 0; c0 < n_cells; c0 += kPPass) {
    // variants before the first window of this pass are final
    const int64_t w_first = c0 / g.W;
    flush(w_first * g.S < g.nv ? w_first * g.S : g.nv);
    int cnt = 0;
    for (int k = 0; k < kPCells; ++k) {
      int64_t a, j0, j1;
      const int64_t c = c0 + (int64_t)tid * kPCells + k;
      if (c >= n_cells || !cell_bits(g, c, a, j0, j1)) continue;
      const uint32_t* row = bitmap + a * bm_words;
      for (int64_t q = j0 >> 5; q <= (j1 - 1) >> 5; ++q)
        cnt += __builtin_popcount(seg_word(row, q, j0, j1));
    }
    int total;
    const int base = block_scan(cnt, wsum, &total);
    for (int s0 = 0; s0 < total; s0 += kPBuf) {
      const int s1 = s0 + kPBuf < total ? s0 + kPBuf : total;
      if (base < s1 && base + cnt > s0) {
        int pos = base;
        for (int k = 0; k < kPCells && pos < s1; ++k) {
          int64_t a, j0, j1;
          const int64_t c = c0 + (int64_t)tid * kPCells + k;
          if (c >= n_cells || !cell_bits(g, c, a, j0, j1)) continue;
          const uint32_t* row = bitmap + a * bm_words;
          const int2 sa = stats[a];
          for (int64_t q = j0 >> 5; q <= (j1 - 1) >> 5 && pos < s1; ++q) {
            uint32_t bits = seg_word(row, q, j0, j1);
            while (bits && pos < s1) {
              const int t = __builtin_ctz(bits);
              bits &= bits - 1;
              if (pos >= s0) {
                const int64_t b = a + 1 + q * 32 + t;
                const int2 sb = stats[b];
                // drop a when its minor allele frequency is strictly lower
                const bool drop_a = (int64_t)sa.x * sb.y < (int64_t)sb.x * sa.y;
                buf[pos - s0] = make_uint2((uint32_t)a, (uint32_t)b | (drop_a ? 0x80000000u : 0u));
              }
              ++pos;
            }
          }
        }
      }
      __syncthreads();
      if (tid == 0) {
        for (int p = 0; p < s1 - s0; ++p) {
          const uint2 e = buf[p];
          const uint32_t ia = e.x & (kRingBits - 1);
          const uint32_t ib = (e.y & 0x7fffffffu) & (kRingBits - 1);
          const uint32_t alive = (ring[ia >> 5] >> (ia & 31)) & (ring[ib >> 5] >> (ib & 31)) & 1u;
          if (alive) {
            const uint32_t x = (e.y >> 31) ? ia : ib;
            ring[x >> 5] &= ~(1u << (x & 31));
          }
        }
      }
      __syncthreads();
    }
  }
  flush(g.nv);
  // block sum of the kept counts
  int k32 = (int)kept;
  int total;
  block_scan(k32, wsum, &total);
  if (tid == 0 && n_kept) *n_kept = total;
}

int launch_prune_greedy(const LdScratch& sc, const int2* stats, int64_t nv, int64_t window,
                        int64_t step, uint8_t* keep, int64_t* n_kept, hipStream_t st) {
  const int64_t n_windows = nv <= window ? 1 : ceil_div(nv - window, step) + 1;
  const PruneGeom g{nv, window, step};
  hipLaunchKernelGGL(k_prune_greedy, dim3(1), dim3(kPT), 0, st, sc.bitmap, sc.bm_words, stats, g,
                     n_windows * window, keep, n_kept);
  return check_launch("prune_greedy");
}

}  // namespace pg
