// Identity-by-state pair kernels.  Both paths produce, for every sample pair
// of an upper-triangle tile, the exact counts IBS0, IBS1, IBS2 and N over the
// variants where neither call is missing (section "Bitwise parallelism").
//
// Matrix-core path.  Each call becomes four int8 features, all zero when the
// call is missing:
//   m = 1;  w = +1 homozygote, -1 heterozygote;  h = [homozygote];
//   c = -1 homozygous A1, 0 heterozygote, +1 homozygous A2.
// For two non-missing calls, h_i h_j - c_i c_j is 2 for opposite homozygotes
// and 0 otherwise, and m_i m_j - w_i w_j is 2 for a homozygote against a
// heterozygote and 0 otherwise.  Contracting over the variants (int32
// accumulation, |sum| <= V) therefore gives
//   N = G_m,  IBS0 = (G_h - G_c) / 2,  IBS1 = (G_m - G_w) / 2,
//   IBS2 = N - IBS0 - IBS1,
// exactly.  G_h - G_c is accumulated in one register set by feeding -c on
// the B side.
//
// Popcount path.  Per 32-variant word of the bit planes H (high code bit),
// L (low code bit) and M (non-missing): m = Mi & Mj, xh = Hi ^ Hj,
// xl = Li ^ Lj; N += popc(m), IBS0 += popc(xh & xl & m) (homozygotes 00 vs
// 11 differ in both bits), IBS1 += popc((xh ^ xl) & m) (exactly one bit
// differs: 00/10 or 10/11).  This is the paper's XOR / mask / popcount step,
// with the one popcount it describes (IBS1 + 2 IBS0) split into two.
#include "tiles.h"

namespace pg {

template <bool kHints>
__global__ __launch_bounds__(256, 1) void k_ibs_mfma(const uint32_t* __restrict__ T, int64_t wp,
                                                     int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  int64_t I, J;
  if (!band_tile(xcd_swizzle(blockIdx.x, gridDim.x), nt, I, J)) return;
  ibs_mfma_tile<kHints>(T, wp, I, J, o, (lds_t*)smem);
}

template <bool kHints>
__global__ __launch_bounds__(256, 1) void k_ibs_mfma_pipe(const uint32_t* __restrict__ T,
                                                          int64_t wp, int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  int64_t I, J;
  if (!band_tile(xcd_swizzle(blockIdx.x, gridDim.x), nt, I, J)) return;
  ibs_mfma_tile_pipe<kHints>(T, wp, I, J, o, (lds_t*)smem);
}

// Cohorts of fewer than 512 tiles (ibs_split): block b runs K range
// b / tiles of tile b % tiles and parks its raw sums; k_ibs_split_reduce
// adds the ranges in order and stores.
template <bool kFp4>
__global__ __launch_bounds__(256, 1) void k_ibs_mfma_split(const uint32_t* __restrict__ T,
                                                           int64_t wp, int64_t nt, IbsOut o,
                                                           int64_t cps, int32_t* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  const int64_t tiles = nt * (nt + 1) / 2;
  const int64_t tile = blockIdx.x % tiles, split = blockIdx.x / tiles;
  const int64_t chunks = wp / kKW;
  const int64_t c0 = split * cps, c1 = c0 + cps < chunks ? c0 + cps : chunks;
  int64_t I, J;
  tri_tile(tile, nt, I, J);
  int32_t* const q = part + (split * tiles + tile) * (192 * 256);
  if constexpr (kFp4)
    ibs_fp4_tile_pipe(T, wp, I, J, o, (lds_t*)smem, c0, c1, q);
  else
    ibs_mfma_tile_pipe<true>(T, wp, I, J, o, (lds_t*)smem, c0, c1, q);
}

// The counts of one entry from raw sums parked by split tiles: register v of
// lane l (32x32 block layout) is row 8*(v/4) + 4*(l/32) + v%4 and column
// l%32 of block ab; wave w covers rows 64*(w/2) and columns 64*(w%2) of the
// tile.  q(sp) points at range sp's 192 x 256 int32 sums of the tile; the
// ranges are added in order.
template <typename Q>
__device__ __forceinline__ void split_entry(Q q, int64_t n_split, int t, int k, int64_t I,
                                            int64_t J, const IbsOut& o) {
  const int ab = k / 16, v = k % 16;
  int32_t m = 0, w = 0, hc = 0;
  for (int64_t sp = 0; sp < n_split; ++sp) {
    const int32_t* r = q(sp) + (ab * 48 + v) * 256 + t;
    m += r[0];
    w += r[16 * 256];
    hc += r[32 * 256];
  }
  const uint32_t n = (uint32_t)m, z = (uint32_t)hc >> 1, one = (n - (uint32_t)w) >> 1;
  const int wid = t >> 6, lane = t & 63;
  const int row = (wid >> 1) * 64 + (ab >> 1) * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
  const int col = (wid & 1) * 64 + (ab & 1) * 32 + (lane & 31);
  store_counts(o, I * kT + row, J * kT + col, I != J, n, z, one);
}

// One thread per (tile, accumulator register, tile thread).
__global__ __launch_bounds__(256) void k_ibs_split_reduce(int64_t nt, int64_t n_split,
                                                          const int32_t* __restrict__ part,
                                                          IbsOut o) {
  const int64_t tiles = nt * (nt + 1) / 2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tiles * 64 * 256) return;
  const int t = (int)(e % 256);
  const int k = (int)((e / 256) % 64);    // (a, b) block and register
  const int64_t tile = e / (256 * 64);
  int64_t I, J;
  tri_tile(tile, nt, I, J);
  split_entry([&](int64_t sp) { return part + (sp * tiles + tile) * (192 * 256); }, n_split, t,
              k, I, J, o);
}

// Head of the tail split: block b runs tile b / 8 of XCD b % 8's run (the
// run's first `head` tiles, whole).
template <bool kFp4>
__global__ __launch_bounds__(256, 1) void k_ibs_head(const uint32_t* __restrict__ T, int64_t wp,
                                                     int64_t nt, IbsOut o, IbsTail tl) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  const int x = (int)(blockIdx.x % 8);
  int64_t I, J;
  valid_band_tile(tl.start[x] + blockIdx.x / 8, nt, I, J);
  if constexpr (kFp4)
    ibs_fp4_tile_pipe(T, wp, I, J, o, (lds_t*)smem);
  else
    ibs_mfma_tile_pipe<true>(T, wp, I, J, o, (lds_t*)smem);
}

// Tail: block b runs K range i % n_split of tail tile i / n_split (i = b / 8)
// of XCD b % 8's run, and parks its raw sums.
template <bool kFp4>
__global__ __launch_bounds__(256, 1) void k_ibs_tail(const uint32_t* __restrict__ T, int64_t wp,
                                                     int64_t nt, IbsOut o, IbsTail tl,
                                                     int32_t* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  const int x = (int)(blockIdx.x % 8);
  const int64_t i = blockIdx.x / 8;
  const int64_t j = i / tl.n_split, sp = i % tl.n_split;
  const int64_t v = tl.start[x] + tl.head + j;
  if (v >= tl.start[x + 1]) return;
  int64_t I, J;
  valid_band_tile(v, nt, I, J);
  const int64_t chunks = wp / kKW;
  const int64_t c0 = sp * tl.cps, c1 = c0 + tl.cps < chunks ? c0 + tl.cps : chunks;
  int32_t* const q = part + ((x * tl.rmax + j) * tl.n_split + sp) * (192 * 256);
  if constexpr (kFp4)
    ibs_fp4_tile_pipe(T, wp, I, J, o, (lds_t*)smem, c0, c1, q);
  else
    ibs_mfma_tile_pipe<true>(T, wp, I, J, o, (lds_t*)smem, c0, c1, q);
}

__global__ __launch_bounds__(256) void k_ibs_tail_reduce(int64_t nt, IbsTail tl,
                                                         const int32_t* __restrict__ part,
                                                         IbsOut o) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 8 * tl.rmax * 64 * 256) return;
  const int t = (int)(e % 256);
  const int k = (int)((e / 256) % 64);
  const int64_t slot = e / (256 * 64);
  const int x = (int)(slot / tl.rmax);
  const int64_t v = tl.start[x] + tl.head + slot % tl.rmax;
  if (v >= tl.start[x + 1]) return;
  int64_t I, J;
  valid_band_tile(v, nt, I, J);
  split_entry([&](int64_t sp) { return part + (slot * tl.n_split + sp) * (192 * 256); },
              tl.n_split, t, k, I, J, o);
}

template <bool kHints>
__global__ __launch_bounds__(512, 1) void k_ibs_mfma_w8(const uint32_t* __restrict__ T, int64_t wp,
                                                        int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  int64_t I, J;
  if (!band_tile(xcd_swizzle(blockIdx.x, gridDim.x), nt, I, J)) return;
  ibs_mfma_tile_w8<kHints>(T, wp, I, J, o, (lds_t*)smem);
}

__global__ __launch_bounds__(256, 1) void k_ibs_mfma_simple(const uint32_t* __restrict__ T,
                                                            int64_t wp, int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSimpleSmem];
  int64_t I, J;
  tri_tile(blockIdx.x, nt, I, J);
  ibs_mfma_tile_simple(T, wp, I, J, o, (lds_t*)smem);
}

__global__ __launch_bounds__(256, 1) void k_ibs_fp4(const uint32_t* __restrict__ T, int64_t wp,
                                                    int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  int64_t I, J;
  if (!band_tile(xcd_swizzle(blockIdx.x, gridDim.x), nt, I, J)) return;
  ibs_fp4_tile(T, wp, I, J, o, (lds_t*)smem);
}

__global__ __launch_bounds__(256, 1) void k_ibs_fp4_pipe(const uint32_t* __restrict__ T,
                                                         int64_t wp, int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsMfmaSmem];
  int64_t I, J;
  if (!band_tile(xcd_swizzle(blockIdx.x, gridDim.x), nt, I, J)) return;
  ibs_fp4_tile_pipe(T, wp, I, J, o, (lds_t*)smem);
}

__global__ __launch_bounds__(256, 1) void k_ibs_fp4rep(const uint32_t* __restrict__ R, int64_t rp,
                                                       int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsRepSmem];
  int64_t I, J;
  if (!band_tile(xcd_swizzle(blockIdx.x, gridDim.x), nt, I, J)) return;
  ibs_fp4rep_tile(R, rp, I, J, o, (lds_t*)smem);
}

__global__ __launch_bounds__(256) void k_ibs_popc(const uint32_t* __restrict__ P, int64_t rows_pad,
                                                  int64_t words_pad, int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t smem[kIbsPopcSmem];
  int64_t I, J;
  tri_tile(blockIdx.x, nt, I, J);
  ibs_popc_tile(P, rows_pad, words_pad, I, J, o, (lds_t*)smem);
}

// Host side of the tail split.  With T tiles, run x is tiles
// [floor(x T / 8), floor((x + 1) T / 8)); every run fills F = floor(shortest
// run / 32) whole rounds of its XCD's 32 CUs, and the r_x <= rmax tiles after
// them are the tail.  A tail of r tiles split in S ranges takes
// ceil(r S / 32) / S rounds of one tile; the split is taken when its best S
// (with 1% of a round charged per range for the ranges' pipeline prologues
// and the reduce) saves at least a quarter of a round.
IbsTail ibs_tail_plan(int64_t rows_pad, int64_t wp) {
  IbsTail t;
  constexpr int64_t kCusPerXcd = 32;
  const int64_t nt = rows_pad / kT;
  const int64_t chunks = wp / kKW;
  const int64_t tiles = nt * (nt + 1) / 2;
  if (nt < 1 || chunks < 4 || tiles < 512) return t;
  for (int x = 0; x <= 8; ++x) t.start[x] = x * tiles / 8;
  int64_t lmin = tiles, lmax = 0;
  for (int x = 0; x < 8; ++x) {
    const int64_t len = t.start[x + 1] - t.start[x];
    lmin = len < lmin ? len : lmin;
    lmax = len > lmax ? len : lmax;
  }
  t.head = (lmin / kCusPerXcd) * kCusPerXcd;
  t.rmax = lmax - t.head;
  if (t.rmax == 0 || t.rmax > kCusPerXcd) return t;
  double best = 1.0;
  int64_t best_s = 1;
  for (int64_t S = 2; S <= 8 && S <= chunks / 2; ++S) {
    const double cost = (double)ceil_div(t.rmax * S, kCusPerXcd) / (double)S + 0.01 * (double)S;
    if (cost < best) {
      best = cost;
      best_s = S;
    }
  }
  if (best_s == 1 || 1.0 - best < 0.25) return t;
  t.cps = ceil_div(chunks, best_s);
  t.n_split = ceil_div(chunks, t.cps);
  t.tail = true;
  return t;
}

// `variant` is resolved (resolve_ibs_variant): 1 .. kIbsVariants - 1.
int launch_ibs_mfma(const uint32_t* T, int64_t wp, const IbsOut& o, int variant, hipStream_t st,
                    int32_t* part) {
  const int64_t nt = ceil_div(o.m, kT);
  const int64_t blocks = variant == 2 ? nt * (nt + 1) / 2 : band_start((nt + 3) / 4, nt);
  const bool fp4 = variant == kIbsVariantFp4Pipe;
  int64_t n_split = 1, cps = 0;
  if ((variant == kIbsVariantPipe || fp4) && part) ibs_split(nt * kT, wp, n_split, cps);
  if ((variant == kIbsVariantPipe || fp4) && part && n_split == 1) {
    const IbsTail tl = ibs_tail_plan(nt * kT, wp);
    if (tl.tail) {
      if (tl.head > 0) {
        hipLaunchKernelGGL(fp4 ? k_ibs_head<true> : k_ibs_head<false>,
                           dim3((unsigned)(8 * tl.head)), dim3(256), 0, st, T, wp, nt, o, tl);
        int rc = check_launch("ibs_head");
        if (rc != PG_OK) return rc;
      }
      hipLaunchKernelGGL(fp4 ? k_ibs_tail<true> : k_ibs_tail<false>,
                         dim3((unsigned)(8 * tl.rmax * tl.n_split)), dim3(256), 0, st, T, wp, nt,
                         o, tl, part);
      int rc = check_launch("ibs_tail");
      if (rc != PG_OK) return rc;
      hipLaunchKernelGGL(k_ibs_tail_reduce, dim3((unsigned)ceil_div(8 * tl.rmax * 64 * 256, 256)),
                         dim3(256), 0, st, nt, tl, part, o);
      return check_launch("ibs_tail_reduce");
    }
  }
  if (n_split > 1) {
    const int64_t tiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(fp4 ? k_ibs_mfma_split<true> : k_ibs_mfma_split<false>,
                       dim3((unsigned)(tiles * n_split)), dim3(256), 0, st, T, wp, nt, o, cps, part);
    int rc = check_launch("ibs_mfma_split");
    if (rc != PG_OK) return rc;
    hipLaunchKernelGGL(k_ibs_split_reduce, dim3((unsigned)ceil_div(tiles * 64 * 256, 256)),
                       dim3(256), 0, st, nt, n_split, part, o);
    return check_launch("ibs_split_reduce");
  }
  const dim3 grid((unsigned)blocks);
  switch (variant) {
    case 1: hipLaunchKernelGGL(k_ibs_mfma<false>, grid, dim3(256), 0, st, T, wp, nt, o); break;
    case 2: hipLaunchKernelGGL(k_ibs_mfma_simple, grid, dim3(256), 0, st, T, wp, nt, o); break;
    case kIbsVariantFp4:
      hipLaunchKernelGGL(k_ibs_fp4, grid, dim3(256), 0, st, T, wp, nt, o);
      break;
    case kIbsVariantW8:
      hipLaunchKernelGGL(k_ibs_mfma_w8<true>, grid, dim3(512), 0, st, T, wp, nt, o);
      break;
    case kIbsVariantW8 + 1:
      hipLaunchKernelGGL(k_ibs_mfma_w8<false>, grid, dim3(512), 0, st, T, wp, nt, o);
      break;
    case kIbsVariantPipe:
      hipLaunchKernelGGL(k_ibs_mfma_pipe<true>, grid, dim3(256), 0, st, T, wp, nt, o);
      break;
    case kIbsVariantR1:
      hipLaunchKernelGGL(k_ibs_mfma<true>, grid, dim3(256), 0, st, T, wp, nt, o);
      break;
    default:
      hipLaunchKernelGGL(k_ibs_fp4_pipe, grid, dim3(256), 0, st, T, wp, nt, o);
      break;
  }
  return check_launch("ibs_mfma");
}

int launch_ibs_fp4rep(const uint32_t* R, int64_t rp, const IbsOut& o, hipStream_t st) {
  const int64_t nt = ceil_div(o.m, kT);
  const int64_t blocks = band_start((nt + 3) / 4, nt);
  hipLaunchKernelGGL(k_ibs_fp4rep, dim3((unsigned)blocks), dim3(256), 0, st, R, rp, nt, o);
  return check_launch("ibs_fp4rep");
}

int launch_ibs_popc(const uint32_t* P, int64_t rows_pad, int64_t words_pad, const IbsOut& o,
                    hipStream_t st) {
  const int64_t nt = rows_pad / kP;
  const int64_t blocks = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(k_ibs_popc, dim3((unsigned)blocks), dim3(256), 0, st, P, rows_pad, words_pad,
                     nt, o);
  return check_launch("ibs_popc");
}

}  // namespace pg
