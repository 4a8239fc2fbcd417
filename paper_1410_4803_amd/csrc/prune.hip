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
// (with the drop side, decided beforehand from the allele counts by a
// grid-wide kernel into a second bitmap), then one wave applies them in
// order to a ring of keep bits in LDS; variants no later window can touch
// are flushed to the output as the windows advance.
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
constexpr int kPGroup = 8;                // cells whose loads are issued together
constexpr int kPWords = 4;                // bitmap words per cell loaded up front
constexpr int kPPass = kPT * kPCells;     // cells per pass
constexpr int kRingBits = 1 << 18;        // keep bits held in LDS (32 KB)
constexpr int kPBuf = 8192;               // pairs staged in LDS per slice (64 KB)

struct PruneGeom {
  int64_t nv, W, S;
};

// Bits [j0, j1) of row a of the bitmap (bit j <-> b = a + 1 + j) that hold
// window w's new pairs, for the cell (window w, row r), a = w*S + r; empty
// (j0 == j1) when the cell has none.
__device__ __forceinline__ void cell_bits(const PruneGeom& g, int64_t w, int r, int& a, int& j0,
                                          int& j1) {
  const int64_t s = w * g.S;
  const int64_t av = s + r;
  const int64_t hi = s + g.W < g.nv ? s + g.W : g.nv;
  a = (int)av;
  j0 = j1 = 0;
  if (av + 1 >= hi) return;
  const int64_t lo = w == 0 ? 0 : (g.W > g.S ? s - g.S + g.W : s);
  const int64_t d0 = lo - av > 1 ? lo - av : 1;
  const int64_t d1 = hi - av;
  if (d0 >= d1) return;
  j0 = (int)(d0 - 1);
  j1 = (int)(d1 - 1);
}

// Bitmap word x (word q of its row) restricted to bits [j0, j1).
__device__ __forceinline__ uint32_t seg_bits(uint32_t x, int q, int j0, int j1) {
  const int b0 = q * 32;
  if (j0 > b0) x &= ~0u << (j0 - b0);
  if (j1 < b0 + 32) x &= (1u << (j1 - b0)) - 1u;
  return x;
}
__device__ __forceinline__ uint32_t seg_word(const uint32_t* row, int q, int j0, int j1) {
  return seg_bits(row[q], q, j0, j1);
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

constexpr int kClaim = 1024;               // slots of the per-batch claim table (8 KB)

// Applies staged pairs buf[0, n) in order to the keep ring; wave 0 only.
// 64 pairs at a time.  One LDS round trip reads both keep bits of every
// pair (the snapshot).  A pair whose snapshot is live acts -- drops its
// variant x -- unless an earlier pair of the batch that acted dropped one of
// its two variants.  Each lane needs the mask K of earlier live pairs whose
// x is one of its variants: every live lane sets its bit in claim[x mod
// kClaim], a lane ORs the slots of its two variants and keeps only the
// earlier pairs whose x (broadcast through xs) really is one of them, then
// every live lane clears its slot again.  Live pairs with K = 0 act whatever
// else happens; the others act when K misses every earlier pair that acted,
// settled in rounds over the whole wave.  The batch's drops are written before
// the next batch reads the ring (LDS operations of one wave complete in
// order, which also orders the claim writes, reads and clears).
__device__ __forceinline__ void apply_pairs(const uint2* buf, int n, uint32_t* ring, uint32_t* xs,
                                            unsigned long long* claim, int lane) {
  for (int p0 = 0; p0 < n; p0 += 64) {
    const int np = n - p0 < 64 ? n - p0 : 64;
    // variants are below 2^31: 0xfffffffe / 0xffffffff never match
    uint32_t ea = 0xfffffffeu, eb = 0xfffffffeu, x = 0xffffffffu;
    bool live = false;
    if (lane < np) {
      const uint2 e = buf[p0 + lane];
      ea = e.x;
      eb = e.y & 0x7fffffffu;
      const uint32_t ia = ea & (kRingBits - 1), ib = eb & (kRingBits - 1);
      live = ((ring[ia >> 5] >> (ia & 31)) & (ring[ib >> 5] >> (ib & 31)) & 1u) != 0;
      x = live ? ((e.y >> 31) ? ea : eb) : 0xffffffffu;
    }
    xs[lane] = x;
    if (live) atomicOr(&claim[x & (kClaim - 1)], 1ull << lane);
    uint64_t k = 0;
    if (live) {
      // earlier pairs whose x falls in the slots of ea or eb, then exactly
      k = (claim[ea & (kClaim - 1)] | claim[eb & (kClaim - 1)]) & ((1ull << lane) - 1ull);
      for (uint64_t c = k; c; c &= c - 1) {
        const int p = __builtin_ctzll(c);
        const uint32_t xp = xs[p];
        if (xp != ea && xp != eb) k &= ~(1ull << p);
      }
    }
    if (live) claim[x & (kClaim - 1)] = 0ull;
    const bool free_pair = live && k == 0;
    uint64_t acted = __ballot(free_pair);
    const uint64_t conflicted = __ballot(live && !free_pair);
    // Conflicted pairs settle in rounds: a pair is decided once an earlier
    // pair of its K acted (it does not act) or every pair of its K is decided
    // and none acted (it acts) -- the same outcome as taking them one by one
    // in order.  The lowest undecided pair always settles, so this ends.
    uint64_t decided = ~conflicted;
    while (conflicted & ~decided) {
      bool now = false, act = false;
      if ((conflicted & ~decided) >> lane & 1ull) {
        if (k & acted) {
          now = true;
        } else if ((k & ~decided) == 0) {
          now = true;
          act = true;
        }
      }
      decided |= __ballot(now);
      acted |= __ballot(act);
    }
    if ((acted >> lane) & 1ull) {
      const uint32_t ix = x & (kRingBits - 1);
      atomicAnd(&ring[ix >> 5], ~(1u << (ix & 31)));
    }
  }
}

// Drop side of every marked pair, beside the bitmap: bit (b - a - 1) of row
// a is set when a has the strictly lower minor allele frequency.  One thread
// per bitmap word.
__global__ __launch_bounds__(256) void k_prune_dropbits(const uint32_t* __restrict__ bitmap,
                                                        int64_t bm_words, int64_t nv,
                                                        const int2* __restrict__ stats,
                                                        uint32_t* __restrict__ drop) {
  const int64_t total = nv * bm_words;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint32_t bits = bitmap[e], out = 0;
    if (bits) {
      const int64_t a = e / bm_words, q = e - a * bm_words;
      const int2 sa = stats[a];
      while (bits) {
        const int t = __builtin_ctz(bits);
        bits &= bits - 1;
        const int2 sb = stats[a + 1 + q * 32 + t];
        if ((int64_t)sa.x * sb.y < (int64_t)sb.x * sa.y) out |= 1u << t;
      }
    }
    drop[e] = out;
  }
}

// Marked bits of every (window, row) cell's segment, for the greedy pass's
// count phase; zero past the last cell (the array is padded to whole passes).
__global__ __launch_bounds__(256) void k_prune_cellcount(const uint32_t* __restrict__ bitmap,
                                                         int64_t bm_words, PruneGeom g,
                                                         int64_t n_windows, int64_t n_pad,
                                                         uint16_t* __restrict__ cc) {
  const int64_t n_cells = n_windows * g.W;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_pad;
       c += (int64_t)gridDim.x * blockDim.x) {
    int cnt = 0;
    if (c < n_cells) {
      int a, j0, j1;
      cell_bits(g, c / g.W, (int)(c % g.W), a, j0, j1);
      if (j0 < j1) {
        const uint32_t* row = bitmap + (int64_t)a * bm_words;
        for (int q = j0 >> 5; q <= (j1 - 1) >> 5; ++q)
          cnt += __builtin_popcount(seg_word(row, q, j0, j1));
      }
    }
    cc[c] = (uint16_t)cnt;
  }
}

__global__ __launch_bounds__(kPT) void k_prune_greedy(const uint32_t* __restrict__ bitmap,
                                                      int64_t bm_words,
                                                      const uint32_t* __restrict__ drop,
                                                      PruneGeom g, int64_t n_windows,
                                                      const uint16_t* __restrict__ cc,
                                                      uint8_t* __restrict__ keep,
                                                      int64_t* __restrict__ n_kept) {
  __shared__ uint32_t ring[kRingBits / 32];
  __shared__ uint2 buf[kPBuf];
  __shared__ int wsum[kPT / 64];
  __shared__ __attribute__((aligned(16))) uint32_t xs[64];
  __shared__ unsigned long long claim[kClaim];
  __shared__ uint16_t s_cc[kPCells * kPT];   // per-cell counts, [cell][thread]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (int i = tid; i < kRingBits / 32; i += kPT) ring[i] = ~0u;
  for (int i = tid; i < kClaim; i += kPT) claim[i] = 0ull;
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
  const int W = (int)g.W;
  const int64_t n_cells = n_windows * g.W;
  for (int64_t c0 = 0; c0 < n_cells; c0 += kPPass) {
    // variants before the first window of this pass are final
    const int64_t w_first = c0 / g.W;
    flush(w_first * g.S < g.nv ? w_first * g.S : g.nv);
    // this thread's kPCells consecutive cells, as (window, row), then bits
    const int rr = (int)(c0 - w_first * g.W) + tid * kPCells;
    const int64_t w_start = w_first + rr / W;
    const int r_start = rr % W;
    // count: per group of kPGroup cells, the first kPWords words of every
    // segment are loaded together (one memory latency per group); the
    // per-cell counts are kept in LDS for the write phase
    int cnt = 0;
    if (cc) {
      // counts from k_prune_cellcount: this thread's kPCells consecutive cells
      const uint4* src = reinterpret_cast<const uint4*>(cc + c0 + (int64_t)tid * kPCells);
      static_assert(kPCells == 16, "two 16-byte loads of eight counts");
      const uint4 v0 = src[0], v1 = src[1];
      const uint32_t ws[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
      for (int k = 0; k < kPCells; ++k) {
        const int c = (int)((ws[k >> 1] >> (16 * (k & 1))) & 0xFFFFu);
        cnt += c;
        s_cc[k * kPT + tid] = (uint16_t)c;
      }
    } else {
      int64_t w = w_start;
      int r = r_start;
#pragma unroll
      for (int kb = 0; kb < kPCells; kb += kPGroup) {
        int ga[kPGroup], gj0[kPGroup], gj1[kPGroup];
        uint32_t gw[kPGroup][kPWords];
#pragma unroll
        for (int k = 0; k < kPGroup; ++k) {
          ga[k] = gj0[k] = gj1[k] = 0;
          if (w < n_windows) cell_bits(g, w, r, ga[k], gj0[k], gj1[k]);
          if (++r == W) {
            r = 0;
            ++w;
          }
#pragma unroll
          for (int u = 0; u < kPWords; ++u) gw[k][u] = 0;
          if (gj0[k] < gj1[k]) {
            const uint32_t* row = bitmap + (int64_t)ga[k] * bm_words;
            const int q0 = gj0[k] >> 5, qn = (gj1[k] - 1) >> 5;
#pragma unroll
            for (int u = 0; u < kPWords; ++u)
              if (q0 + u <= qn) gw[k][u] = row[q0 + u];
          }
        }
#pragma unroll
        for (int k = 0; k < kPGroup; ++k) {
          int c = 0;
          if (gj0[k] < gj1[k]) {
            const int q0 = gj0[k] >> 5, qn = (gj1[k] - 1) >> 5;
#pragma unroll
            for (int u = 0; u < kPWords; ++u)
              if (q0 + u <= qn) c += __builtin_popcount(seg_bits(gw[k][u], q0 + u, gj0[k], gj1[k]));
            const uint32_t* row = bitmap + (int64_t)ga[k] * bm_words;
            for (int q = q0 + kPWords; q <= qn; ++q)
              c += __builtin_popcount(seg_word(row, q, gj0[k], gj1[k]));
          }
          cnt += c;
          s_cc[(kb + k) * kPT + tid] = (uint16_t)c;
        }
      }
    }
    int total;
    const int base = block_scan(cnt, wsum, &total);
    for (int s0 = 0; s0 < total; s0 += kPBuf) {
      const int s1 = s0 + kPBuf < total ? s0 + kPBuf : total;
      if (base < s1 && base + cnt > s0) {
        int pos = base;
        int64_t w = w_start;
        int r = r_start;
        for (int k = 0; k < kPCells; ++k) {
          const int c = s_cc[k * kPT + tid];
          const int64_t wk = w;
          const int rk = r;
          if (++r == W) {
            r = 0;
            ++w;
          }
          // cells wholly before this slice, or empty, are skipped unread
          if (c == 0 || pos >= s1) continue;
          if (pos + c <= s0) {
            pos += c;
            continue;
          }
          int a, j0, j1;
          cell_bits(g, wk, rk, a, j0, j1);
          const int64_t base_w = (int64_t)a * bm_words;
          int left = c;
          for (int q = j0 >> 5; left > 0 && pos < s1; ++q) {
            uint32_t bits = seg_bits(bitmap[base_w + q], q, j0, j1);
            const uint32_t dw = drop[base_w + q];
            while (bits && pos < s1) {
              const int t = __builtin_ctz(bits);
              bits &= bits - 1;
              --left;
              if (pos >= s0) {
                const int b = a + 1 + q * 32 + t;
                buf[pos - s0] = make_uint2((uint32_t)a, (uint32_t)b | (((dw >> t) & 1u) << 31));
              }
              ++pos;
            }
          }
        }
      }
      __syncthreads();
      if (tid < 64) apply_pairs(buf, s1 - s0, ring, xs, claim, lane);
      __syncthreads();
    }
  }
  flush(g.nv);
  // block sum of the kept counts
  int total;
  block_scan((int)kept, wsum, &total);
  if (tid == 0 && n_kept) *n_kept = total;
}

int64_t prune_cells_padded(int64_t nv, int64_t window, int64_t step) {
  const int64_t n_windows = nv <= window ? 1 : ceil_div(nv - window, step) + 1;
  return round_up(n_windows * window, kPPass);
}

int64_t prune_count_capacity(int64_t nv, int64_t window) {
  // step 1 has the most windows, at most nv of them
  const int64_t worst = round_up(nv * window, kPPass);
  return worst < kPruneCountCellsMax ? worst : kPruneCountCellsMax;
}

int launch_prune_greedy(const LdScratch& sc, const int2* stats, uint32_t* drop, uint16_t* cc,
                        int64_t cc_capacity, int64_t nv, int64_t window, int64_t step,
                        uint8_t* keep, int64_t* n_kept, hipStream_t st) {
  const int64_t words = nv * sc.bm_words;
  const int64_t blocks = ceil_div(words, 256) < 65536 ? ceil_div(words, 256) : 65536;
  hipLaunchKernelGGL(k_prune_dropbits, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, st,
                     sc.bitmap, sc.bm_words, nv, stats, drop);
  int rc = check_launch("prune_dropbits");
  if (rc != PG_OK) return rc;
  const int64_t n_windows = nv <= window ? 1 : ceil_div(nv - window, step) + 1;
  const PruneGeom g{nv, window, step};
  int64_t n_pad = prune_cells_padded(nv, window, step);
  if (!cc || n_pad > cc_capacity) n_pad = 0;
  if (n_pad > 0) {
    const int64_t cb = ceil_div(n_pad, 256) < 65536 ? ceil_div(n_pad, 256) : 65536;
    hipLaunchKernelGGL(k_prune_cellcount, dim3((unsigned)cb), dim3(256), 0, st, sc.bitmap,
                       sc.bm_words, g, n_windows, n_pad, cc);
    rc = check_launch("prune_cellcount");
    if (rc != PG_OK) return rc;
  }
  hipLaunchKernelGGL(k_prune_greedy, dim3(1), dim3(kPT), 0, st, sc.bitmap, sc.bm_words, drop, g,
                     n_windows, n_pad > 0 ? cc : nullptr, keep, n_kept);
  return check_launch("prune_greedy");
}

}  // namespace pg
