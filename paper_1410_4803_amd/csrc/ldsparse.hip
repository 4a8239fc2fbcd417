// LD window sums with missing-call corrections (section "Bit population
// count": without missing calls the per-variant sums are fixed, and only
// sum x_a x_b has to be computed per pair).
//
// Per variant v over the selected samples: c_v missing calls (the list of
// their samples, in increasing order) and the totals over its non-missing
// calls, t_v = sum x and u_v = sum x^2.  With x_a[k] = 0 for a missing call,
// the sums of a pair (a, b) over the samples where neither call is missing
// are the totals minus what the other variant's missing calls remove:
//   n   = m - c_a - c_b + |miss(a) and miss(b)|
//   Sx  = t_a - sum over k in miss(b) of x_a[k],  Sxx = u_a - (same for x_a^2)
//   Sy  = t_b - sum over k in miss(a) of x_b[k],  Syy = u_b - (same for x_b^2)
// and Sxy is one int8 Gram over all samples on the matrix cores.  Every sum
// stays an exact integer.
//
// A correction reads one word per missing call and 16 variants: a word of
// the sample-major operand T holds the codes of 16 consecutive variants at
// one sample, and their per-variant counts of homozygous A1, homozygous A2
// and missing codes grow as bytes, one byte-permute lookup per four variants.
// T is stored in strips of 64 variants (a tile's side), so one tile side at
// one sample is 16 contiguous bytes and the samples of a strip are adjacent:
// the missing calls of a tile read from two contiguous runs, and a line
// fetched for one sample holds the tile's codes at seven neighbouring ones.
//
// Tiles are the 64 x 64 variant tiles of the dense kernel.  A tile takes
// this path when all of its variants have at most `cap` missing calls (the
// length of a list slot) and its missing calls are few enough (at most
// `budget` over its two 64-variant groups) that the corrections cost less
// than the five dense Grams they replace; the dense kernel runs the other
// tiles and skips these.
//
// Launch order: k_ld_vstats (lists, counts, totals) and k_ld_groups (group
// statistics, and whether enough groups qualify for the path to be on),
// k_ld_transpose (T, only when it is on), then the dense kernel and
// k_ld_sparse, each taking its own tiles.
#include "tiles.h"

namespace pg {

// Missing calls of every stride-th variant row of D (the first m samples),
// added to *gate: one wave per sampled row.
__global__ __launch_bounds__(256) void k_ld_miss_sample(const uint32_t* __restrict__ D, int64_t wn,
                                                        int64_t m, int64_t nv, int64_t stride,
                                                        unsigned long long* __restrict__ gate) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * stride;
  if (v >= nv) return;
  const uint32_t* row = D + v * wn;
  unsigned int c = 0;
  for (int64_t w = lane; w < wn; w += 64) {
    const uint32_t x = row[w];
    uint32_t miss = x & ~(x >> 1) & 0x55555555u;   // code 01
    const int64_t valid = m - 16 * w;              // selected samples in this word
    if (valid < 16) miss &= valid <= 0 ? 0u : ((1u << (2 * valid)) - 1u);
    c += __popc(miss);
  }
  for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
  if (lane == 0 && c) atomicAdd(gate, (unsigned long long)c);
}

// Per-variant missing-call list, count and totals: one wave per variant row
// of the variant-major operand D (padding samples are missing calls and are
// not listed; padding variants get zero counts and empty lists).  A list
// entry is the sample index.  Does nothing when a gate is given and the
// sampled count exceeds gate_max (the path stays off).
__global__ __launch_bounds__(256) void k_ld_vstats(const uint32_t* __restrict__ D, int64_t wn,
                                                   int64_t m, int64_t nv, int64_t rows_pad, int cap,
                                                   uint32_t* __restrict__ lists,
                                                   int4* __restrict__ vst,
                                                   const unsigned long long* __restrict__ gate,
                                                   unsigned long long gate_max) {
  if (gate && *gate > gate_max) return;
  const int lane = threadIdx.x & 63;
  const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (v >= rows_pad) return;
  if (v >= nv) {
    if (lane == 0) vst[v] = make_int4(0, 0, 0, 0);
    return;
  }
  const uint32_t* row = D + v * wn;
  uint32_t* list = lists + v * (int64_t)cap;
  int64_t c = 0;
  int n3 = 0, n0 = 0;
  constexpr int kU = 8;   // 64-word slices loaded ahead of the scan
  for (int64_t w0 = 0; w0 < wn; w0 += 64 * kU) {
    uint32_t x[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t w = w0 + 64 * u + lane;
      x[u] = w < wn ? row[w] : 0xAAAAAAAAu;   // past the row: hets, counted nowhere
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t w = w0 + 64 * u + lane;
      const uint32_t lo = x[u] & 0x55555555u, hi = (x[u] >> 1) & 0x55555555u;
      n3 += __popc(lo & hi);
      n0 += __popc(~(lo | hi) & 0x55555555u);
      uint32_t miss = lo & ~hi;
      const int64_t valid = m - 16 * w;   // selected samples in this word
      if (valid < 16) miss &= valid <= 0 ? 0u : ((1u << (2 * valid)) - 1u);
      if (__ballot(miss != 0) == 0) continue;   // (the same for the whole wave)
      // exclusive prefix sum of the per-lane counts (at most 16) over the
      // wave, one bit of the count at a time, with no cross-lane data moves
      const int k = __popc(miss);
      int excl = 0, total = 0;
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        const uint64_t bb = __ballot((k >> b) & 1);
        excl += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u)) << b;
        total += __popcll(bb) << b;
      }
      int64_t pos = c + excl;
      while (miss) {
        const int bit = __ffs(miss) - 1;
        const int64_t smp = 16 * w + (bit >> 1);
        if (pos < cap) list[pos] = (uint32_t)smp;
        ++pos;
        miss &= miss - 1;
      }
      c += total;
    }
  }
  for (int d = 32; d > 0; d >>= 1) {
    n3 += __shfl_xor(n3, d, 64);
    n0 += __shfl_xor(n0, d, 64);
  }
  if (lane == 0) vst[v] = make_int4((int)c, n3 - n0, n3 + n0, 0);
}

// Per group of 64 variants: total and largest missing-call count, and the
// number of groups whose diagonal tile qualifies (groups_ok, cleared
// before).  A tile (I, J) can qualify only if one of its groups has total
// <= budget / 2, whose diagonal tile then qualifies too.
constexpr int kGrpPerBlock = 64;   // groups per block of k_ld_groups (16 per wave)

__global__ __launch_bounds__(256) void k_ld_groups(const int4* __restrict__ vst, int64_t n_groups,
                                                   int cap, int64_t budget,
                                                   int64_t* __restrict__ gsum,
                                                   int* __restrict__ gmax,
                                                   uint32_t* __restrict__ groups_ok,
                                                   const unsigned long long* __restrict__ gate,
                                                   unsigned long long gate_max) {
  __shared__ uint32_t s_ok;
  if (gate && *gate > gate_max) return;   // groups_ok stays 0: the path is off
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_ok = 0;
  __syncthreads();
  uint32_t ok = 0;
  for (int i = 0; i < kGrpPerBlock / 4; ++i) {
    const int64_t g = (int64_t)blockIdx.x * kGrpPerBlock + wave * (kGrpPerBlock / 4) + i;
    if (g >= n_groups) break;
    const int c = vst[g * 64 + lane].x;
    int64_t sum = c;
    int mx = c;
    for (int d = 32; d > 0; d >>= 1) {
      sum += __shfl_xor(sum, d, 64);
      const int o = __shfl_xor(mx, d, 64);
      mx = o > mx ? o : mx;
    }
    if (lane == 0) {
      gsum[g] = sum;
      gmax[g] = mx;
    }
    ok += mx <= cap && 2 * sum <= budget;
  }
  if (lane == 0 && ok) atomicAdd(&s_ok, ok);
  __syncthreads();
  if (threadIdx.x == 0 && s_ok) atomicAdd(groups_ok, s_ok);
}

constexpr int kSpS = 65;          // LDS row stride of the per-pair cells (words)
constexpr int kSpBatch = 8;       // missing calls per lane and batch
constexpr int kSpFlush = 248;     // missing calls between byte-counter flushes (< 256)

__device__ __forceinline__ uint32_t gather_word(const uint32_t* p) { return *p; }

// Walks one lane's missing-call list (cnt entries; the wave's longest list
// has cmax) in batches of kSpBatch and hands each batch of gathered words to
// consume(); the word of sample k is at base + 16 k + lane_bytes (one strip
// of T).  Lanes past their list get `idle`.  Two stages in flight: the
// entries of batch j + 2 and the words of batch j + 1 load while batch j is
// counted.  List slots hold a multiple of kSpBatch entries and cmax does not
// exceed the slot, so every list read stays inside the slot (entries past
// cnt are read but not used).
template <typename W, typename F>
__device__ __forceinline__ void gather_list(const uint32_t* __restrict__ list, int cnt, int cmax,
                                            const char* __restrict__ base, uint32_t lane_bytes,
                                            W idle, F&& consume) {
  const int nb = (cmax + kSpBatch - 1) / kSpBatch;
  if (nb == 0) return;
  uint32_t ks[kSpBatch];
  auto load_ks = [&](int j) {
    const uint4 a = *reinterpret_cast<const uint4*>(list + j * kSpBatch);
    const uint4 b = *reinterpret_cast<const uint4*>(list + j * kSpBatch + 4);
    ks[0] = a.x; ks[1] = a.y; ks[2] = a.z; ks[3] = a.w;
    ks[4] = b.x; ks[5] = b.y; ks[6] = b.z; ks[7] = b.w;
  };
  W w[kSpBatch];
  auto load_w = [&](int j) {
#pragma unroll
    for (int u = 0; u < kSpBatch; ++u) {
      const char* p = base + (((uint64_t)ks[u] << 4) + lane_bytes);
      w[u] = j * kSpBatch + u < cnt ? gather_word(reinterpret_cast<const W*>(p)) : idle;
    }
  };
  load_ks(0);
  load_w(0);
  if (nb > 1) load_ks(1);
  for (int j = 0; j < nb; ++j) {
    W cur[kSpBatch];
#pragma unroll
    for (int u = 0; u < kSpBatch; ++u) cur[u] = w[u];
    if (j + 1 < nb) load_w(j + 1);
    if (j + 2 < nb) load_ks(j + 2);
    consume(cur);
  }
}

// Byte c of each table is the count increment of code c: homA1 in the low
// nibble and homA2 in the high nibble of one byte, or missing.
constexpr uint32_t kNibHom = 0x10000001u;
constexpr uint32_t kCntMiss = 0x00000100u;

// Per-variant counters of one batch of 16-code words: counter dword d, byte
// e counts position 4e + d.  homA1 / homA2 grow as nibbles over the batch
// (at most kSpBatch < 16 per nibble) and are then added to the byte counters
// h1 / h2; missing codes (kMiss) go straight to the byte counters ms.
template <bool kMiss>
__device__ __forceinline__ void count_batch(const uint32_t (&words)[kSpBatch], uint32_t (&h1)[4],
                                            uint32_t (&h2)[4], uint32_t (&ms)[4]) {
  uint32_t nib[4] = {0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < kSpBatch; ++u) {
    uint32_t c[4];
    spread_codes(words[u], c);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      nib[d] += __builtin_amdgcn_perm(0u, kNibHom, c[d]);
      if constexpr (kMiss) ms[d] += __builtin_amdgcn_perm(0u, kCntMiss, c[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    h1[d] += nib[d] & 0x0F0F0F0Fu;
    h2[d] += (nib[d] >> 4) & 0x0F0F0F0Fu;
  }
}

__global__ __launch_bounds__(256, 3) void k_ld_sparse(
    const uint32_t* __restrict__ D, int64_t wn, const uint32_t* __restrict__ T, int64_t t_rows,
    const uint32_t* __restrict__ lists, const int4* __restrict__ vst,
    const int64_t* __restrict__ gsum, const int* __restrict__ gmax,
    const uint32_t* __restrict__ groups_ok, uint32_t min_groups, int cap, int64_t budget,
    int64_t m, int64_t nv, int64_t n_row_tiles, int64_t n_band, int32_t window,
    double r2_min, LdScratch sc, pg_ld_pair* __restrict__ dbg, int64_t v0) {
  const int64_t blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int64_t I = blk / n_band;
  const int64_t J = I + blk % n_band;
  if (J >= n_row_tiles || !ld_tile_sparse(gsum, gmax, groups_ok, min_groups, I, J, cap, budget))
    return;

  // per-pair cells: first the Sxy partial sums, then the b-side corrections
  // (row a, column b); the a-side corrections (row b, column a): homA1 |
  // homA2 << 16 and the shared missing calls
  __shared__ uint32_t s_cell[kLdTile * kSpS];
  __shared__ uint32_t s_acell[kLdTile * kSpS];
  __shared__ uint32_t s_mcell[kLdTile * kSpS];
  const int t = threadIdx.x, lane = t & 63;
  const int wid = __builtin_amdgcn_readfirstlane(t >> 6);
  const int g = lane >> 5, rl = lane & 31;
  const int qi = wid >> 1, qj = wid & 1;   // this wave's 32 x 32 quadrant
  for (int e = t; e < kLdTile * kSpS; e += 256) s_cell[e] = s_acell[e] = s_mcell[e] = 0;
  __syncthreads();

  // ---- Sxy: each wave takes a quarter of the samples for the whole tile
  // (2 x 2 blocks of 32 x 32); lane group g holds words 8q + 4g .. + 3 of its
  // rows, and A and B use the same word order, so K matches.
  {
    const uint32_t* pa = D + (I * kLdTile + rl) * wn + 4 * g;
    const uint32_t* pb = D + (J * kLdTile + rl) * wn + 4 * g;
    const int64_t off1 = 32 * wn;
    const int64_t ngroups = wn / 8;
    const int64_t q0 = ngroups * wid / 4, q1 = ngroups * (wid + 1) / 4;
    v16i acc00 = (v16i){0}, acc01 = (v16i){0}, acc10 = (v16i){0}, acc11 = (v16i){0};
    // three register sets, rotating, so the prefetch (two groups ahead)
    // needs no copies
    uint4 r0[4], r1[4], r2[4];
    auto load = [&](uint4 (&r)[4], int64_t q) {
      r[0] = *reinterpret_cast<const uint4*>(pa + 8 * q);
      r[1] = *reinterpret_cast<const uint4*>(pa + off1 + 8 * q);
      r[2] = *reinterpret_cast<const uint4*>(pb + 8 * q);
      r[3] = *reinterpret_cast<const uint4*>(pb + off1 + 8 * q);
    };
    auto step = [&](const uint4 (&r)[4]) {
      const uint32_t wa0[4] = {r[0].x, r[0].y, r[0].z, r[0].w};
      const uint32_t wa1[4] = {r[1].x, r[1].y, r[1].z, r[1].w};
      const uint32_t wb0[4] = {r[2].x, r[2].y, r[2].z, r[2].w};
      const uint32_t wb1[4] = {r[3].x, r[3].y, r[3].z, r[3].w};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        uint32_t c[4];
        spread_codes(wa0[s], c);
        const v4i xa0 = ld_lookup(kLdLutX, c);
        spread_codes(wa1[s], c);
        const v4i xa1 = ld_lookup(kLdLutX, c);
        spread_codes(wb0[s], c);
        const v4i xb0 = ld_lookup(kLdLutX, c);
        spread_codes(wb1[s], c);
        const v4i xb1 = ld_lookup(kLdLutX, c);
        acc00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa0, xb0, acc00, 0, 0, 0);
        acc01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa0, xb1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa1, xb0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa1, xb1, acc11, 0, 0, 0);
      }
    };
    if (q0 < q1) load(r0, q0);
    if (q0 + 1 < q1) load(r1, q0 + 1);
    for (int64_t q = q0; q < q1; q += 3) {
      if (q + 2 < q1) load(r2, q + 2);
      step(r0);
      if (q + 3 < q1) load(r0, q + 3);
      if (q + 1 < q1) step(r1);
      if (q + 4 < q1) load(r1, q + 4);
      if (q + 2 < q1) step(r2);
    }
    // 32x32 accumulator layout: register v of lane l holds row
    // 8*(v/4) + 4*(l/32) + v%4 and column l%32.
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v >> 2) + 4 * g + (v & 3);
      atomicAdd(&s_cell[r * kSpS + rl], (uint32_t)acc00[v]);
      atomicAdd(&s_cell[r * kSpS + 32 + rl], (uint32_t)acc01[v]);
      atomicAdd(&s_cell[(32 + r) * kSpS + rl], (uint32_t)acc10[v]);
      atomicAdd(&s_cell[(32 + r) * kSpS + 32 + rl], (uint32_t)acc11[v]);
    }
  }
  __syncthreads();
  // this lane's 16 pairs of the quadrant: rows al(v) of tile I, column bl of J
  const int bl = 32 * qj + rl;
  int xy[16];
#pragma unroll
  for (int v = 0; v < 16; ++v)
    xy[v] = (int)s_cell[(32 * qi + 8 * (v >> 2) + 4 * g + (v & 3)) * kSpS + bl];
  __syncthreads();

  // ---- corrections.  Lane (16 * wave + lane / 4, q = lane % 4) owns
  // variant `own` of each tile side and the 16 variants of word q of the
  // other side.  b-side: at the missing calls of variant own of tile I, the
  // codes of word q of tile J, into s_cell; the first flush stores, so every
  // cell is written even for an empty list.  a-side: at the missing calls of
  // variant own of tile J, the codes of word q of tile I, into s_acell and
  // s_mcell.  The four lanes of one variant read one 16-byte piece.
  const int own = 16 * wid + (lane >> 2), q = lane & 3;
  uint32_t bh1[4] = {0, 0, 0, 0}, bh2[4] = {0, 0, 0, 0}, bms[4];
  uint32_t ah1[4] = {0, 0, 0, 0}, ah2[4] = {0, 0, 0, 0}, ams[4] = {0, 0, 0, 0};
  bool first = true;
  int since_b = 0, since_a = 0;
  auto flush_b = [&]() {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = own * kSpS + 16 * q + 4 * e + d;
        const uint32_t val = ((bh1[d] >> (8 * e)) & 0xFFu) | (((bh2[d] >> (8 * e)) & 0xFFu) << 16);
        s_cell[idx] = first ? val : s_cell[idx] + val;
      }
      bh1[d] = bh2[d] = 0;
    }
    first = false;
  };
  auto flush_a = [&]() {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = own * kSpS + 16 * q + 4 * e + d;
        s_acell[idx] += ((ah1[d] >> (8 * e)) & 0xFFu) | (((ah2[d] >> (8 * e)) & 0xFFu) << 16);
        s_mcell[idx] += (ams[d] >> (8 * e)) & 0xFFu;
      }
      ah1[d] = ah2[d] = ams[d] = 0;
    }
  };
  auto count_b = [&](const uint32_t (&w)[kSpBatch]) {
    count_batch<false>(w, bh1, bh2, bms);
    since_b += kSpBatch;
    if (since_b == kSpFlush) {
      flush_b();
      since_b = 0;
    }
  };
  auto count_a = [&](const uint32_t (&w)[kSpBatch]) {
    count_batch<true>(w, ah1, ah2, ams);
    since_a += kSpBatch;
    if (since_a == kSpFlush) {
      flush_a();
      since_a = 0;
    }
  };
  const uint32_t* stripI = T + I * t_rows * 4;
  const uint32_t* stripJ = T + J * t_rows * 4;
  {
    const int cnt = vst[I * kLdTile + own].x;
    int cmax = cnt;
    for (int d = 32; d > 0; d >>= 1) {
      const int o = __shfl_xor(cmax, d, 64);
      cmax = o > cmax ? o : cmax;
    }
    cmax = __builtin_amdgcn_readfirstlane(cmax);
    gather_list(lists + (I * kLdTile + own) * (int64_t)cap, cnt, cmax,
                reinterpret_cast<const char*>(stripJ), 4u * q, 0xAAAAAAAAu, count_b);
  }
  {
    const int cnt = vst[J * kLdTile + own].x;
    int cmax = cnt;
    for (int d = 32; d > 0; d >>= 1) {
      const int o = __shfl_xor(cmax, d, 64);
      cmax = o > cmax ? o : cmax;
    }
    cmax = __builtin_amdgcn_readfirstlane(cmax);
    gather_list(lists + (J * kLdTile + own) * (int64_t)cap, cnt, cmax,
                reinterpret_cast<const char*>(stripI), 4u * q, 0xAAAAAAAAu, count_a);
  }
  if (since_b || first) flush_b();
  if (since_a) flush_a();
  __syncthreads();

  // ---- pairs
  const int64_t b = J * kLdTile + bl;
  if (b >= nv) return;
  const int4 sb = vst[b];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int al = 32 * qi + 8 * (v >> 2) + 4 * g + (v & 3);
    const int64_t a = I * kLdTile + al;
    if (!(a < b && b - a <= window)) continue;
    const int4 sa = vst[a];
    const uint32_t pb = s_cell[al * kSpS + bl], pa = s_acell[bl * kSpS + al];
    const int64_t a1 = pa & 0xFFFFu, a2 = pa >> 16;
    const int64_t b1 = pb & 0xFFFFu, b2 = pb >> 16;
    const int64_t both = s_mcell[bl * kSpS + al];
    const int64_t n = m - sa.x - sb.x + both;
    const int64_t sx = sa.y - (a2 - a1), sy = sb.y - (b2 - b1);
    const int64_t sxx = sa.z - (a2 + a1), syy = sb.z - (b2 + b1), sxy = xy[v];
    if (dbg) {
      pg_ld_pair rec;
      rec.a = (int32_t)(v0 + a);
      rec.b = (int32_t)(v0 + b);
      rec.n = n; rec.sx = sx; rec.sy = sy; rec.sxx = sxx; rec.syy = syy; rec.sxy = sxy;
      rec.r2 = ld_r2(n, sx, sy, sxx, syy, sxy);
      dbg[a * window + (b - a - 1)] = rec;
    } else {
      ld_mark(sc, a, b, r2_min, n, sx, sy, sxx, syy, sxy);
    }
  }
}

constexpr int kTrW = 32;            // words per block side: 512 variants x 512 samples
constexpr int kTrS = kTrW + 1;      // LDS row stride (words)

// Sample-major operand T in strips of 64 variants from the variant-major D
// (rows_pad x wn words): word a (the codes of variants 16a..16a+15) at sample
// k is T[((a / 4) * t_rows + k) * 4 + a % 4].  A block takes 32 words of each
// side; lanes read consecutive words of a D row (full lines), the 16x16
// transposes land in LDS, and each half-wave writes one sample's 32 words as
// eight 16-byte pieces of eight strips (consecutive samples of a strip are
// adjacent, so a block fills whole lines).  Variants past rows_pad read as
// missing.  Does nothing while *gate < gate_min.
__global__ __launch_bounds__(256) void k_ld_transpose(const uint32_t* __restrict__ D,
                                                      int64_t rows_pad, int64_t wn,
                                                      uint32_t* __restrict__ T, int64_t t_rows,
                                                      int64_t tw, const uint32_t* __restrict__ gate,
                                                      uint32_t gate_min) {
  if (*gate < gate_min) return;
  __shared__ uint32_t s_out[16 * kTrW * kTrS];
  const int64_t nb_a = ceil_div(tw, kTrW);
  const int64_t a0 = ((int64_t)blockIdx.x % nb_a) * kTrW;   // T word (16 variants)
  const int64_t g0 = ((int64_t)blockIdx.x / nb_a) * kTrW;   // D word (16 samples)
  const int t = threadIdx.x;
  const int gl = t % kTrW;
#pragma unroll 1
  for (int i = 0; i < 4; ++i) {
    const int al = t / kTrW + 8 * i;
    const int64_t a = a0 + al, g = g0 + gl;
    uint32_t x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t v = 16 * a + r;
      x[r] = (v < rows_pad && g < wn) ? D[v * wn + g] : kAllMissing16;
    }
    transpose16_2bit(x);
#pragma unroll
    for (int c = 0; c < 16; ++c) s_out[(c * kTrW + gl) * kTrS + al] = x[c];
  }
  __syncthreads();
  const int lane = t & 63, wave = t >> 6;
  for (int row = 2 * wave + (lane >> 5); row < 16 * kTrW; row += 8) {
    const int64_t k = 16 * g0 + row, a = a0 + (lane & 31);
    if (k < t_rows && a < tw)   // T row 16 gl + c is LDS row c * kTrW + gl
      T[((a >> 2) * t_rows + k) * 4 + (a & 3)] =
          s_out[((row & 15) * kTrW + (row >> 4)) * kTrS + (lane & 31)];
  }
}

int launch_ld_sparse_stats(const uint32_t* D, int64_t wn, int64_t m, int64_t nv,
                           int64_t rows_pad, const LdSparse& sp, hipStream_t st) {
  int rc = PG_OK;
  unsigned long long* gate = reinterpret_cast<unsigned long long*>(sp.gate);
  if (gate) {
    rc = fill_u32(reinterpret_cast<uint32_t*>(gate), 2, 0u, st);
    if (rc != PG_OK) return rc;
    const int64_t n_samp = ceil_div(nv, sp.gate_stride);
    hipLaunchKernelGGL(k_ld_miss_sample, dim3((unsigned)ceil_div(n_samp, 4)), dim3(256), 0, st, D,
                       wn, m, nv, sp.gate_stride, gate);
    rc = check_launch("ld_miss_sample");
    if (rc != PG_OK) return rc;
  }
  const dim3 grid((unsigned)ceil_div(rows_pad, 4));
  hipLaunchKernelGGL(k_ld_vstats, grid, dim3(256), 0, st, D, wn, m, nv, rows_pad, sp.cap, sp.lists,
                     sp.vst, gate, (unsigned long long)sp.gate_max);
  rc = check_launch("ld_vstats");
  if (rc == PG_OK) rc = fill_u32(sp.groups_ok, 1, 0u, st);
  if (rc != PG_OK) return rc;
  const int64_t n_groups = rows_pad / kLdTile;
  hipLaunchKernelGGL(k_ld_groups, dim3((unsigned)ceil_div(n_groups, kGrpPerBlock)), dim3(256), 0,
                     st, sp.vst,
                     n_groups, sp.cap, sp.budget, sp.gsum, sp.gmax, sp.groups_ok, gate,
                     (unsigned long long)sp.gate_max);
  return check_launch("ld_groups");
}

int launch_ld_transpose(const uint32_t* D, int64_t rows_pad, int64_t wn, uint32_t* T,
                        int64_t t_rows, int64_t tw, const LdSparse& sp, hipStream_t st) {
  const int64_t blocks = ceil_div(tw, kTrW) * ceil_div(t_rows, 16 * kTrW);
  hipLaunchKernelGGL(k_ld_transpose, dim3((unsigned)blocks), dim3(256), 0, st, D, rows_pad, wn, T,
                     t_rows, tw, sp.groups_ok, sp.min_groups);
  return check_launch("ld_transpose");
}

int launch_ld_sparse(const uint32_t* D, int64_t wn, const uint32_t* T, int64_t t_rows, int64_t m,
                     int64_t nv, int64_t rows_pad, int32_t window, double r2_min,
                     const LdScratch& sc, const LdSparse& sp, hipStream_t st, pg_ld_pair* dbg,
                     int64_t v0) {
  int rc;
  // the dense kernel takes the tiles this path leaves
  if (!dbg) {
    rc = launch_ld_mfma(D, wn, nv, rows_pad, window, r2_min, sc, st, &sp, m < kFp4MaxVariants);
    if (rc != PG_OK) return rc;
  }
  const int64_t n_row_tiles = rows_pad / kLdTile;
  const int64_t n_band = ((int64_t)window + kLdTile - 1) / kLdTile + 1;
  hipLaunchKernelGGL(k_ld_sparse, dim3((unsigned)(n_row_tiles * n_band)), dim3(256), 0, st, D, wn,
                     T, t_rows, sp.lists, sp.vst, sp.gsum, sp.gmax, sp.groups_ok, sp.min_groups,
                     sp.cap, sp.budget, m, nv, n_row_tiles, n_band, window, r2_min, sc,
                     dbg, v0);
  rc = check_launch("ld_sparse");
  mark_stage(2, st);
  return rc;
}

}  // namespace pg
