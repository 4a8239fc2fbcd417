// Genomic relationship matrix (section "Partial sum lookup": a weighted
// distance matrix as a sum of per-marker increments, with the GCTA
// relationship increments (x - 2p)(y - 2p) / (2p(1-p)) as its example).
//
// The paper's CPU design precomputes, per marker, the increments of the seven
// genotype-pair cases and adds table entries per pair.  Here the increment
// factors: with z = (x - 2p) / sqrt(2p(1-p)) for a non-missing call and 0 for
// a missing one, the numerator of every pair is a dot product over markers,
//   S[i,j] = sum_v z[i,v] z[j,v],
// i.e. one double-precision Gram matrix, run on the fp64 matrix cores
// (v_mfma_f64_16x16x4_f64).  The operand is never materialised: tiles load
// the packed 2-bit codes and look each call's z up in the marker's four-entry
// table (indexed by the 2-bit code; code 1 = missing -> 0).  The denominator
// N[i,j] (markers where both calls are present) is a popcount of AND-ed
// non-missing masks, accumulated beside the fp64 sums.
//
// Markers whose increments are undefined (no call, or p equal to 0 or 1) are
// treated as missing for every sample.
#include "tiles.h"

namespace pg {

// ---- per-marker tables ---------------------------------------------------------
// One wave per selected variant: counts over the selected samples, then
// z for codes 0 (homozygous A1, x = 0), 2 (heterozygous, x = 1), 3
// (homozygous A2, x = 2); missing and undefined -> 0.  used2 gets bit 2t of
// word v/16 set (t = v % 16) for a variant with defined increments.
__global__ __launch_bounds__(256) void k_grm_table(Sel s, int64_t nv_pad, double* __restrict__ ztab,
                                                   uint32_t* __restrict__ used2) {
  const int lane = threadIdx.x & 63;
  for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < nv_pad;
       v += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    int calls = 0, a2 = 0;
    if (v < s.nv) {
      for (int64_t k = lane; k < s.m; k += 64) {
        const uint32_t c = code_at(s, v, k);
        calls += c != 1u;
        a2 += (int)(c >> 1) + (int)(c == 3u);   // 0 -> 0, 2 -> 1, 3 -> 2
      }
    }
    for (int d = 32; d > 0; d >>= 1) {
      calls += __shfl_xor(calls, d, 64);
      a2 += __shfl_xor(a2, d, 64);
    }
    if (lane == 0) {
      const bool used = calls > 0 && a2 > 0 && a2 < 2 * calls;
      double z0 = 0.0, z1 = 0.0, z2 = 0.0;
      if (used) {
        const double p = __ddiv_rn((double)a2, (double)(2 * calls));
        const double q = 1.0 - p;
        const double inv = __ddiv_rn(1.0, __dsqrt_rn(__dmul_rn(2.0, __dmul_rn(p, q))));
        const double tp = __dmul_rn(2.0, p);
        z0 = __dmul_rn(-tp, inv);
        z1 = __dmul_rn(__dsub_rn(1.0, tp), inv);
        z2 = __dmul_rn(__dsub_rn(2.0, tp), inv);
        atomicOr(&used2[v >> 4], 1u << (2 * (v & 15)));
      }
      double* t = ztab + v * 4;
      t[0] = z0;
      t[1] = 0.0;
      t[2] = z1;
      t[3] = z2;
    }
  }
}

// ---- the pair kernel ---------------------------------------------------------------
// Block: 256 threads = 4 waves (2 x 2) over a 128 x 128 tile of sample pairs
// (upper-triangle tiles only) and one range of K chunks: when the tiles
// alone cannot fill the chip, each tile's variants are split into ranges
// whose partial sums a second kernel adds in a fixed order.  Each wave owns 64 x 64 = 4 x 4 blocks of
// 16 x 16 fp64 accumulators.  K runs over variants in chunks of 128 (eight
// 2-bit words per sample): the loader stages both blocks' words (with
// undefined markers overridden to missing), the chunk's z tables and each
// row's 64-bit non-missing mask in LDS; the next chunk is fetched into
// registers meanwhile.  v_mfma_f64_16x16x4_f64 operand layout: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register r of lane l is
// D[l / 16 + 4 r][l % 16].
constexpr int kGT = 128;          // samples per tile side
constexpr int kGK = 128;          // variants per K chunk
constexpr int kGKW = kGK / 16;    // 2-bit words per row per chunk

typedef double grm_d4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) uint64_t lds_u64;

struct GrmOut {
  double* grm;
  uint32_t* n;
  int64_t m;
  int full;
  int64_t n_tiles;      // upper-triangle tiles
  int64_t n_split;      // K splits per tile (1: write the result directly)
  int64_t cps;          // K chunks per split
  double* part_s;       // n_split > 1: per (split, tile) 128 x 128 partial sums
  uint32_t* part_n;     //   and partial counts
};

// Stores one entry (i, j) of tile (I, J): A = S / N (NaN when N = 0),
// mirrored below the diagonal for the full layout.
__device__ __forceinline__ void grm_store(const GrmOut& o, int64_t i, int64_t j, bool diag, double S,
                                          uint32_t nn) {
  if (i >= o.m || j >= o.m) return;
  const double val = nn ? __ddiv_rn(S, (double)nn) : __longlong_as_double(0x7ff8000000000000ll);
  if (o.full) {
    o.grm[i * o.m + j] = val;
    o.n[i * o.m + j] = nn;
    if (!diag) {
      o.grm[j * o.m + i] = val;
      o.n[j * o.m + i] = nn;
    }
  } else if (i < j) {
    const int64_t idx = i * o.m - i * (i + 1) / 2 + (j - i - 1);
    o.grm[idx] = val;
    o.n[idx] = nn;
  }
}

// 16 codes -> 16-bit mask of non-missing calls (bit t <-> code t).
__device__ __forceinline__ uint32_t present16(uint32_t w) {
  uint32_t x = ~(w & ~(w >> 1)) & 0x55555555u;   // code != 01 at even bits
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}

// Wave grid kWR x kWC over the tile: each wave owns (128 / kWR) x (128 / kWC)
// = kNA x kNB blocks of 16 x 16: 2 x 2 waves (one per SIMD), 4 x 2 (two per
// SIMD) or 4 x 4 (four per SIMD).  More waves per SIMD hide the latency of
// the fp64 MFMAs at the cost of more table lookups per MFMA.
template <int kWR, int kWC>
__global__ __launch_bounds__(64 * kWR * kWC, 1) void k_grm_mfma(const uint32_t* __restrict__ T,
                                                                int64_t wp,
                                                                const double* __restrict__ ztab,
                                                                const uint32_t* __restrict__ used2,
                                                                int64_t nt, GrmOut o) {
  constexpr int kNA = kGT / kWR / 16, kNB = kGT / kWC / 16;
  // LDS (per buffer): codes of the I and J blocks [2][128][4] words, masks
  // [2][128] uint64, z tables [64][4] doubles.
  __shared__ uint32_t s_codes[2][2][kGT][kGKW];
  __shared__ uint64_t s_mask[2][2][kGT][kGKW / 4];
  __shared__ double s_z[2][kGK * 4];

  const int64_t tile = blockIdx.x % o.n_tiles;
  const int64_t split = blockIdx.x / o.n_tiles;
  int64_t I, J;
  tri_tile(tile, nt, I, J);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave / kWC, wc = wave % kWC;
  const bool loader = tid < 256;
  // this block's K chunks: [c_begin, c_end)
  const int64_t all_chunks = wp / kGKW;
  const int c_begin = (int)(split * o.cps);
  const int c_end = (int)((split + 1) * o.cps < all_chunks ? (split + 1) * o.cps : all_chunks);

  // loader role (threads 0..255): thread t stages row (t & 127) of block
  // (t >> 7) and one double of the z table
  const int lrow = tid & (kGT - 1), lblk = (tid >> 7) & 1;
  const int64_t grow = (lblk ? J : I) * kGT + lrow;
  const uint4* src = reinterpret_cast<const uint4*>(T + grow * wp);
  constexpr int kQ = kGKW / 4;      // uint4 pieces per row per chunk
  struct Fetch {
    uint4 w[kQ], u[kQ];
    double z[kGK * 4 / 256];
  };
  auto fetch = [&](int c, Fetch& f) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      f.w[q] = src[c * kQ + q];
      f.u[q] = reinterpret_cast<const uint4*>(used2)[c * kQ + q];
    }
#pragma unroll
    for (int q = 0; q < kGK * 4 / 256; ++q) f.z[q] = ztab[(int64_t)c * kGK * 4 + q * 256 + tid];
  };
  auto stage = [&](int buf, const Fetch& f) {
    // undefined markers read as missing (code 01)
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const uint32_t ws[4] = {f.w[q].x, f.w[q].y, f.w[q].z, f.w[q].w};
      const uint32_t us[4] = {f.u[q].x, f.u[q].y, f.u[q].z, f.u[q].w};
      uint64_t mask = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t undef = ~us[e] & 0x55555555u;
        const uint32_t x = (ws[e] & ~(undef | (undef << 1))) | undef;
        s_codes[buf][lblk][lrow][q * 4 + e] = x;
        mask |= (uint64_t)present16(x) << (16 * e);
      }
      s_mask[buf][lblk][lrow][q] = mask;
    }
#pragma unroll
    for (int q = 0; q < kGK * 4 / 256; ++q) s_z[buf][q * 256 + tid] = f.z[q];
  };

  grm_d4 acc[kNA][kNB];
  uint32_t cnt[kNA][kNB][4];
#pragma unroll
  for (int a = 0; a < kNA; ++a)
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      acc[a][b] = grm_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 4; ++r) cnt[a][b][r] = 0;
    }

  Fetch pf;
  if (c_begin < c_end && loader) {
    fetch(c_begin, pf);
    stage(0, pf);
  }
  __syncthreads();
  const int kq = lane >> 4;          // this lane's K index inside a step
  const int r16 = lane & 15;
  for (int c = c_begin; c < c_end; ++c) {
    const int buf = (c - c_begin) & 1;
    if (c + 1 < c_end && loader) fetch(c + 1, pf);
    const lds_t* ci = (const lds_t*)&s_codes[buf][0][0][0];
    const lds_t* cj = (const lds_t*)&s_codes[buf][1][0][0];
    const lds_f64* zt = (const lds_f64*)&s_z[buf][0];
#pragma unroll
    for (int wd = 0; wd < kGKW; ++wd) {
      uint32_t wa[kNA], wb[kNB];
#pragma unroll
      for (int q = 0; q < kNA; ++q) wa[q] = ci[(wr * kNA * 16 + q * 16 + r16) * kGKW + wd];
#pragma unroll
      for (int q = 0; q < kNB; ++q) wb[q] = cj[(wc * kNB * 16 + q * 16 + r16) * kGKW + wd];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int t = st * 4 + kq;                 // variant inside the word
        const int k = wd * 16 + t;                 // variant inside the chunk
        double av[kNA], bv[kNB];
#pragma unroll
        for (int q = 0; q < kNA; ++q) av[q] = zt[k * 4 + ((wa[q] >> (2 * t)) & 3u)];
#pragma unroll
        for (int q = 0; q < kNB; ++q) bv[q] = zt[k * 4 + ((wb[q] >> (2 * t)) & 3u)];
#pragma unroll
        for (int a = 0; a < kNA; ++a)
#pragma unroll
          for (int b = 0; b < kNB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    // pair counts: rows l / 16 + 4 r of each 16-row block, column l % 16
    {
      const lds_u64* mi = (const lds_u64*)&s_mask[buf][0][0][0];
      const lds_u64* mj = (const lds_u64*)&s_mask[buf][1][0][0];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        uint64_t colm[kNB];
#pragma unroll
        for (int b = 0; b < kNB; ++b) colm[b] = mj[(wc * kNB * 16 + b * 16 + r16) * kQ + q];
#pragma unroll
        for (int a = 0; a < kNA; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint64_t rm = mi[(wr * kNA * 16 + a * 16 + kq + 4 * r) * kQ + q];
#pragma unroll
            for (int b = 0; b < kNB; ++b) cnt[a][b][r] += (uint32_t)__popcll(rm & colm[b]);
          }
      }
    }
    if (c + 1 < c_end && loader) stage(buf ^ 1, pf);
    __syncthreads();
  }

  // epilogue: the result, or this split's partial sums and counts
  const bool diag = I == J;
#pragma unroll
  for (int a = 0; a < kNA; ++a)
#pragma unroll
    for (int b = 0; b < kNB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int il = wr * kNA * 16 + a * 16 + kq + 4 * r;
        const int jl = wc * kNB * 16 + b * 16 + r16;
        if (o.n_split == 1) {
          grm_store(o, I * kGT + il, J * kGT + jl, diag, acc[a][b][r], cnt[a][b][r]);
        } else {
          const int64_t e = ((split * o.n_tiles + tile) * kGT + il) * kGT + jl;
          o.part_s[e] = acc[a][b][r];
          o.part_n[e] = cnt[a][b][r];
        }
      }
}

// Sums the K splits of every tile entry in split order, then stores it.
__global__ __launch_bounds__(256) void k_grm_reduce(int64_t nt, GrmOut o) {
  const int64_t per_tile = (int64_t)kGT * kGT;
  const int64_t total = o.n_tiles * per_tile;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tile = e / per_tile;
    const int il = (int)((e % per_tile) / kGT), jl = (int)(e % kGT);
    double S = 0.0;
    uint32_t nn = 0;
    for (int64_t sp = 0; sp < o.n_split; ++sp) {
      S = __dadd_rn(S, o.part_s[sp * total + e]);
      nn += o.part_n[sp * total + e];
    }
    int64_t I, J;
    tri_tile(tile, nt, I, J);
    grm_store(o, I * kGT + il, J * kGT + jl, I == J, S, nn);
  }
}

int launch_grm(const Sel& s, const uint32_t* T, int64_t rows_pad, int64_t wp, double* ztab,
               uint32_t* used2, double* part, double* grm, uint32_t* n_used, int full,
               int waves, hipStream_t st) {
  int rc = fill_u32(used2, wp, 0u, st);
  if (rc != PG_OK) return rc;
  const int64_t nv_pad = wp * 16;
  const int64_t blocks = ceil_div(nv_pad, 4) < 65536 ? ceil_div(nv_pad, 4) : 65536;
  hipLaunchKernelGGL(k_grm_table, dim3((unsigned)blocks), dim3(256), 0, st, s, nv_pad, ztab, used2);
  rc = check_launch("grm_table");
  mark_stage(1, st);
  if (rc != PG_OK) return rc;
  const int64_t nt = rows_pad / kGT;
  const int64_t n_tiles = nt * (nt + 1) / 2;
  int64_t n_split, cps;
  grm_split(rows_pad, wp, n_split, cps);
  const int64_t part_entries = n_split > 1 ? n_split * n_tiles * kGT * kGT : 0;
  const GrmOut o{grm, n_used, s.m, full, n_tiles, n_split, cps, part,
                 (uint32_t*)(part + part_entries)};
  if (waves == 16)
    hipLaunchKernelGGL((k_grm_mfma<4, 4>), dim3((unsigned)(n_tiles * n_split)), dim3(1024), 0, st,
                       T, wp, ztab, used2, nt, o);
  else if (waves == 8)
    hipLaunchKernelGGL((k_grm_mfma<4, 2>), dim3((unsigned)(n_tiles * n_split)), dim3(512), 0, st, T,
                       wp, ztab, used2, nt, o);
  else
    hipLaunchKernelGGL((k_grm_mfma<2, 2>), dim3((unsigned)(n_tiles * n_split)), dim3(256), 0, st, T,
                       wp, ztab, used2, nt, o);
  rc = check_launch("grm_mfma");
  if (rc == PG_OK && n_split > 1) {
    const int64_t blocks = ceil_div(n_tiles * kGT * kGT, 256);
    hipLaunchKernelGGL(k_grm_reduce, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256),
                       0, st, nt, o);
    rc = check_launch("grm_reduce");
  }
  mark_stage(2, st);
  return rc;
}

}  // namespace pg
