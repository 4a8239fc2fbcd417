// Tile bodies of the pair kernels, shared by the one-problem kernels and the
// persistent batch kernel so both run exactly the same arithmetic.
// Every body is called by all 256 threads of a block, for one tile, with
// `smem` pointing at the block's LDS scratch (at least the size given by the
// matching k*Smem constant); bodies synchronise internally.
#pragma once

#include <type_traits>

#include "pg_internal.h"

namespace pg {

// LDS scratch, typed in the LDS address space so every access is a ds_read /
// ds_write (a generic pointer would compile to flat instructions).
typedef __attribute__((address_space(3))) uint32_t lds_t;
typedef unsigned int lds_v4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) lds_v4 lds_v4_t;

__device__ __forceinline__ uint4 lds_ld4(const lds_t* p) {
  const lds_v4 v = *reinterpret_cast<const lds_v4_t*>(p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void lds_st4(lds_t* p, const uint4& v) {
  lds_v4 x;
  x.x = v.x; x.y = v.y; x.z = v.z; x.w = v.w;
  *reinterpret_cast<lds_v4_t*>(p) = x;
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Byte c of each table is the int8 feature value of code c
// (0 homA1, 1 missing, 2 het, 3 homA2).
constexpr uint32_t kLutM = 0x01010001u;   //  1  0  1  1
constexpr uint32_t kLutW = 0x01FF0001u;   //  1  0 -1  1
constexpr uint32_t kLutH = 0x01000001u;   //  1  0  0  1
constexpr uint32_t kLutC = 0x010000FFu;   // -1  0  0  1
constexpr uint32_t kLutCn = 0xFF000001u;  //  1  0  0 -1

// Sixteen 2-bit codes -> four dwords whose bytes are the codes.  Byte e of
// dword d is the code at position 4e + d; A and B operands use the same
// order, so the permutation of K inside a word is harmless.
__device__ __forceinline__ void spread_codes(uint32_t w, uint32_t c[4]) {
  c[0] = w & 0x03030303u;
  c[1] = (w >> 2) & 0x03030303u;
  c[2] = (w >> 4) & 0x03030303u;
  c[3] = (w >> 6) & 0x03030303u;
}

__device__ __forceinline__ v4i lookup(uint32_t lut, const uint32_t c[4]) {
  v4i r;
  r[0] = (int)__builtin_amdgcn_perm(0u, lut, c[0]);
  r[1] = (int)__builtin_amdgcn_perm(0u, lut, c[1]);
  r[2] = (int)__builtin_amdgcn_perm(0u, lut, c[2]);
  r[3] = (int)__builtin_amdgcn_perm(0u, lut, c[3]);
  return r;
}

// Linear upper-triangle tile index -> (I, J), I <= J, row-major.
__device__ __forceinline__ void tri_tile(int64_t b, int64_t nt, int64_t& I, int64_t& J) {
  // rows start at s(I) = I*nt - I*(I-1)/2; estimate I, then correct.
  const double fn = (double)nt + 0.5;
  int64_t i = (int64_t)(fn - sqrt(fn * fn - 2.0 * (double)b));
  if (i < 0) i = 0;
  if (i > nt - 1) i = nt - 1;
  while (i > 0 && i * nt - i * (i - 1) / 2 > b) --i;
  while (i + 1 < nt && (i + 1) * nt - (i + 1) * i / 2 <= b) ++i;
  I = i;
  J = i + (b - (i * nt - i * (i - 1) / 2));
}

// Banded tile order for the stand-alone matrix-core kernels: tile rows are
// taken four at a time (band P = rows 4P..4P+3) and, inside a band, columns
// ascend with the four rows of a column adjacent.  Band P holds 4*(nt - 4P)
// virtual tiles starting at 4*nt*P - 8*P*(P-1); virtual tiles below the
// diagonal or past the matrix are empty (returns false).  Thirty-two
// consecutive indices cover a 4 x 8 block of tiles, which shares 4 row panels
// and 8 column panels.
__host__ __device__ __forceinline__ int64_t band_start(int64_t P, int64_t nt) {
  return 4 * nt * P - 8 * P * (P - 1);
}

__device__ __forceinline__ bool band_tile(int64_t b, int64_t nt, int64_t& I, int64_t& J) {
  const double f = 4.0 * (double)nt + 8.0;
  const double disc = f * f - 32.0 * (double)b;
  int64_t P = (int64_t)((f - sqrt(disc > 0.0 ? disc : 0.0)) / 16.0);
  const int64_t nb = (nt + 3) / 4;
  if (P < 0) P = 0;
  if (P > nb - 1) P = nb - 1;
  while (P > 0 && band_start(P, nt) > b) --P;
  while (P + 1 < nb && band_start(P + 1, nt) <= b) ++P;
  const int64_t local = b - band_start(P, nt);
  I = 4 * P + (local & 3);
  J = 4 * P + (local >> 2);
  return I < nt && J < nt && J >= I;
}

// The same banded order without the empty positions: valid tile v (0 <=
// v < nt(nt+1)/2) -> (I, J).  Band P has r = min(4, nt - 4P) rows; its
// first r columns hold 1, 2, .., r tiles (the diagonal block's upper
// triangle) and every later column r, so the band holds
// r(r+1)/2 + r(nt - 4P - r) tiles; within a column the rows ascend.
__host__ __device__ __forceinline__ void valid_band_tile(int64_t v, int64_t nt, int64_t& I,
                                                         int64_t& J) {
  int64_t P = 0, base = 0;
  for (;;) {
    const int64_t r = nt - 4 * P < 4 ? nt - 4 * P : 4;
    const int64_t tri = r * (r + 1) / 2;
    const int64_t cnt = tri + r * (nt - 4 * P - r);
    if (v < base + cnt || 4 * (P + 1) >= nt) {
      int64_t u = v - base, d, row;
      if (u < tri) {
        d = 0;
        while ((d + 1) * (d + 2) / 2 <= u) ++d;
        row = u - d * (d + 1) / 2;
      } else {
        u -= tri;
        d = r + u / r;
        row = u % r;
      }
      I = 4 * P + row;
      J = 4 * P + d;
      return;
    }
    base += cnt;
    ++P;
  }
}

// Blocks are handed to the 8 XCDs round-robin (block b runs on XCD b % 8);
// remap so each XCD takes a contiguous run of the tile order (for the first
// 8*(B/8) blocks) and its L2 sees neighbouring tiles.
__device__ __forceinline__ int64_t xcd_swizzle(int64_t b, int64_t nblocks) {
  const int64_t full = (nblocks / 8) * 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

// kU16: the arrays hold 16-bit counts (o.u16).  The tile epilogues choose
// the width once, outside their unrolled loops.
template <bool kU16>
__device__ __forceinline__ void store_counts_w(const IbsOut& o, int64_t i, int64_t j, bool mirror,
                                               uint32_t n, uint32_t z, uint32_t one) {
  if (i >= o.m || j >= o.m) return;
  const uint32_t two = n - z - one;
  auto put = [&](int64_t a) {
    if constexpr (kU16) {
      reinterpret_cast<uint16_t*>(o.ibs0)[a] = (uint16_t)z;
      reinterpret_cast<uint16_t*>(o.ibs1)[a] = (uint16_t)one;
      reinterpret_cast<uint16_t*>(o.ibs2)[a] = (uint16_t)two;
      reinterpret_cast<uint16_t*>(o.nonmiss)[a] = (uint16_t)n;
    } else {
      o.ibs0[a] = z; o.ibs1[a] = one; o.ibs2[a] = two; o.nonmiss[a] = n;
    }
  };
  if (o.full) {
    put(i * o.m + j);
    if (mirror) put(j * o.m + i);
  } else if (i < j) {
    put(i * o.m - i * (i + 1) / 2 + (j - i - 1));
  }
}

__device__ __forceinline__ void store_counts(const IbsOut& o, int64_t i, int64_t j, bool mirror,
                                             uint32_t n, uint32_t z, uint32_t one) {
  if (o.u16) store_counts_w<true>(o, i, j, mirror, n, z, one);
  else store_counts_w<false>(o, i, j, mirror, n, z, one);
}

// Stores the counts of one 32x32 accumulator block (register v of lane l is
// row 8*(v/4) + 4*(l/32) + v%4, column l%32).  The direct entries (i, j) go
// out as 4-byte stores that are contiguous across lanes; the mirrored entries
// (j, i) of an off-diagonal tile go out as one 16-byte store per four
// consecutive i, so each row receives whole 32-byte pieces (scalar stores at
// the matrix edge or when rows are not 16-byte aligned).
template <bool kU16>
__device__ __forceinline__ void store_block(const IbsOut& o, int64_t i_base, int64_t j,
                                            bool mirror, int lane, const uint32_t (&n)[16],
                                            const uint32_t (&z)[16], const uint32_t (&one)[16]) {
  const int64_t ib = i_base + 4 * (lane >> 5);
  if (!o.full) {
#pragma unroll
    for (int v = 0; v < 16; ++v)
      store_counts_w<kU16>(o, ib + 8 * (v >> 2) + (v & 3), j, false, n[v], z[v], one[v]);
    return;
  }
#pragma unroll
  for (int v = 0; v < 16; ++v)
    store_counts_w<kU16>(o, ib + 8 * (v >> 2) + (v & 3), j, false, n[v], z[v], one[v]);
  if (!mirror || j >= o.m) return;
  const bool vec_ok = (o.m & 3) == 0 &&
                      ((reinterpret_cast<uintptr_t>(o.ibs0) | reinterpret_cast<uintptr_t>(o.ibs1) |
                        reinterpret_cast<uintptr_t>(o.ibs2) | reinterpret_cast<uintptr_t>(o.nonmiss)) &
                       (kU16 ? 7 : 15)) == 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t i0 = ib + 8 * g;
    if (vec_ok && i0 + 3 < o.m) {
      const int64_t a = j * o.m + i0;
      uint4 t0, t1, t2, t3;
      t0 = make_uint4(z[4 * g], z[4 * g + 1], z[4 * g + 2], z[4 * g + 3]);
      t1 = make_uint4(one[4 * g], one[4 * g + 1], one[4 * g + 2], one[4 * g + 3]);
      t2 = make_uint4(n[4 * g] - z[4 * g] - one[4 * g], n[4 * g + 1] - z[4 * g + 1] - one[4 * g + 1],
                      n[4 * g + 2] - z[4 * g + 2] - one[4 * g + 2],
                      n[4 * g + 3] - z[4 * g + 3] - one[4 * g + 3]);
      t3 = make_uint4(n[4 * g], n[4 * g + 1], n[4 * g + 2], n[4 * g + 3]);
      if constexpr (kU16) {   // four 16-bit counts per 8-byte store
        auto pack = [](uint4 t) {
          return make_uint2((t.x & 0xFFFFu) | (t.y << 16), (t.z & 0xFFFFu) | (t.w << 16));
        };
        *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(o.ibs0) + a) = pack(t0);
        *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(o.ibs1) + a) = pack(t1);
        *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(o.ibs2) + a) = pack(t2);
        *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(o.nonmiss) + a) = pack(t3);
      } else {
        *reinterpret_cast<uint4*>(o.ibs0 + a) = t0;
        *reinterpret_cast<uint4*>(o.ibs1 + a) = t1;
        *reinterpret_cast<uint4*>(o.ibs2 + a) = t2;
        *reinterpret_cast<uint4*>(o.nonmiss + a) = t3;
      }
    } else {
      for (int e = 0; e < 4; ++e) {
        const int v = 4 * g + e;
        store_counts_w<kU16>(o, j, i0 + e, false, n[v], z[v], one[v]);
      }
    }
  }
}

// ---- matrix-core path ---------------------------------------------------------
// Block: 256 threads = 4 waves in a 2x2 grid over a 128x128 tile; each wave
// owns 64x64 = 2x2 blocks of v_mfma_i32_32x32x32_i8 and three accumulator sets
// (G_m, G_w, G_h - G_c).  K runs over variants in chunks of 16 words (256
// variants).  Lane group g = lane/32 of MFMA step s (0..7) holds the 16 codes
// of word 8g + s of its row, i.e. one MFMA lane's 16 K values are one 2-bit
// word.
//
// The pipelined kernel overlaps three things: the next chunk is fetched from
// global memory into registers while the current one is consumed from one of
// two LDS buffers; each lane reads its 8 words per row with two 128-bit LDS
// reads; and the features of step s+1 are expanded while the MFMAs of step s
// run.  Variant 0 (default) adds scheduling hints that interleave one MFMA
// with a few VALU instructions; variant 1 leaves the order to the compiler;
// variant 2 is the unpipelined form (single LDS buffer, no prefetch), kept as
// a reference point for the tuner.
constexpr int kT = kIbsMfmaTile;
constexpr int kKW = kIbsMfmaKWords;
constexpr int kLdsStride = kKW + 4;   // words per LDS row (padding vs. bank conflicts)

struct Feat4 {
  v4i m, w, h, c;
};

__device__ __forceinline__ Feat4 expand_a(uint32_t word) {
  uint32_t c[4];
  spread_codes(word, c);
  return Feat4{lookup(kLutM, c), lookup(kLutW, c), lookup(kLutH, c), lookup(kLutC, c)};
}

__device__ __forceinline__ Feat4 expand_b(uint32_t word) {
  uint32_t c[4];
  spread_codes(word, c);
  return Feat4{lookup(kLutM, c), lookup(kLutW, c), lookup(kLutH, c), lookup(kLutCn, c)};
}

struct IbsAcc {
  v16i m[2][2], w[2][2], hc[2][2];
};

__device__ __forceinline__ void mfma_step(IbsAcc& acc, const Feat4 (&fa)[2], const Feat4 (&fb)[2]) {
  // grouped by feature, so the two updates of each G_h - G_c accumulator are
  // never back to back
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (q == 0)
          acc.m[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].m, fb[b].m, acc.m[a][b], 0, 0, 0);
        else if (q == 1)
          acc.w[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].w, fb[b].w, acc.w[a][b], 0, 0, 0);
        else if (q == 2)
          acc.hc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].h, fb[b].h, acc.hc[a][b], 0, 0, 0);
        else
          acc.hc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].c, fb[b].c, acc.hc[a][b], 0, 0, 0);
      }
}

// 32x32 accumulator layout: register v of lane l holds row
// 8*(v/4) + 4*(l/32) + v%4 and column l%32 of the block.
__device__ __forceinline__ void ibs_epilogue(const IbsAcc& acc, const IbsOut& o, int64_t I,
                                             int64_t J, int wr, int wc, int lane) {
  const bool mirror = (I != J);
  auto stores = [&](auto width) {
    constexpr bool kU16 = decltype(width)::value;
  #pragma unroll
    for (int a = 0; a < 2; ++a)
  #pragma unroll
      for (int b = 0; b < 2; ++b) {
        uint32_t n[16], z[16], one[16];
  #pragma unroll
        for (int v = 0; v < 16; ++v) {
          n[v] = (uint32_t)acc.m[a][b][v];
          z[v] = (uint32_t)acc.hc[a][b][v] >> 1;
          one[v] = (n[v] - (uint32_t)acc.w[a][b][v]) >> 1;
        }
        store_block<kU16>(o, I * kT + wr * 64 + a * 32, J * kT + wc * 64 + b * 32 + (lane & 31), mirror,
                    lane, n, z, one);
      }
  };
  if (o.u16) stores(std::true_type{});
  else stores(std::false_type{});
}

__device__ __forceinline__ void zero_acc(IbsAcc& acc) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc.m[a][b] = (v16i){0};
      acc.w[a][b] = (v16i){0};
      acc.hc[a][b] = (v16i){0};
    }
}


// Chunks [c0, c1) of the tile's variants (c1 < 0: all of them).  With
// `part`, the raw sums go there instead of the counts: 12 accumulator sets x
// 16 registers per thread, stored [set * 16 + register][thread] with the sets
// in the order (a, b) = (0,0), (0,1), (1,0), (1,1), each as m, w, hc.
template <bool kHints>
__device__ __forceinline__ void ibs_mfma_tile(const uint32_t* __restrict__ T, int64_t wp,
                                              int64_t I, int64_t J, const IbsOut& o,
                                              lds_t* smem, int64_t c0 = 0, int64_t c1 = -1,
                                              int32_t* __restrict__ part = nullptr) {
  constexpr int kBuf = kT * kLdsStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int g = lane >> 5;
  const int rl = lane & 31;

  // this thread's share of a chunk: rows t/4 and t/4 + 64, words 4*(t%4)..+3
  const int lrow = t >> 2;
  const int lq = (t & 3) * 4;
  const uint32_t* pa = T + (I * kT + lrow) * wp + lq;
  const uint32_t* pb = T + (J * kT + lrow) * wp + lq;
  const int64_t half = 64 * wp;
  uint4 ga0, ga1, gb0, gb1;
  auto gload = [&](int64_t kc) {
    ga0 = *reinterpret_cast<const uint4*>(pa + kc);
    ga1 = *reinterpret_cast<const uint4*>(pa + half + kc);
    gb0 = *reinterpret_cast<const uint4*>(pb + kc);
    gb1 = *reinterpret_cast<const uint4*>(pb + half + kc);
  };
  auto lstore = [&](int buf) {
    lds_st4(&(sA + buf * kBuf)[lrow * kLdsStride + lq], ga0);
    lds_st4(&(sA + buf * kBuf)[(lrow + 64) * kLdsStride + lq], ga1);
    lds_st4(&(sB + buf * kBuf)[lrow * kLdsStride + lq], gb0);
    lds_st4(&(sB + buf * kBuf)[(lrow + 64) * kLdsStride + lq], gb1);
  };

  IbsAcc acc;
  zero_acc(acc);
  const int64_t nchunks = c1 < 0 ? wp / kKW : c1;
  gload(c0 * kKW);
  lstore(0);
  __syncthreads();
  for (int64_t k = c0; k < nchunks; ++k) {
    const int buf = (int)((k - c0) & 1);
    if (k + 1 < nchunks) gload((k + 1) * kKW);
    // this lane's 8 words of each of its two A rows and two B rows
    uint32_t wa[2][8], wb[2][8];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const lds_t* ra = &(sA + buf * kBuf)[(wr * 64 + x * 32 + rl) * kLdsStride + g * 8];
      const lds_t* rb = &(sB + buf * kBuf)[(wc * 64 + x * 32 + rl) * kLdsStride + g * 8];
      const uint4 a0 = lds_ld4(ra);
      const uint4 a1 = lds_ld4(ra + 4);
      const uint4 b0 = lds_ld4(rb);
      const uint4 b1 = lds_ld4(rb + 4);
      wa[x][0] = a0.x; wa[x][1] = a0.y; wa[x][2] = a0.z; wa[x][3] = a0.w;
      wa[x][4] = a1.x; wa[x][5] = a1.y; wa[x][6] = a1.z; wa[x][7] = a1.w;
      wb[x][0] = b0.x; wb[x][1] = b0.y; wb[x][2] = b0.z; wb[x][3] = b0.w;
      wb[x][4] = b1.x; wb[x][5] = b1.y; wb[x][6] = b1.z; wb[x][7] = b1.w;
    }
    Feat4 fa[2], fb[2];
    fa[0] = expand_a(wa[0][0]); fa[1] = expand_a(wa[1][0]);
    fb[0] = expand_b(wb[0][0]); fb[1] = expand_b(wb[1][0]);
#pragma unroll
    for (int s = 0; s < kKW / 2; ++s) {
      Feat4 na[2], nb[2];
      if (s + 1 < kKW / 2) {
        na[0] = expand_a(wa[0][s + 1]); na[1] = expand_a(wa[1][s + 1]);
        nb[0] = expand_b(wb[0][s + 1]); nb[1] = expand_b(wb[1][s + 1]);
      }
      mfma_step(acc, fa, fb);
      if constexpr (kHints) {
        // interleave: 1 MFMA, then up to 6 VALU instructions, 16 times
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);
        }
      }
      if (s + 1 < kKW / 2) {
        fa[0] = na[0]; fa[1] = na[1];
        fb[0] = nb[0]; fb[1] = nb[1];
      }
    }
    if (k + 1 < nchunks) lstore(buf ^ 1);
    __syncthreads();
  }
  if (part) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          int32_t* q = part + ((a * 2 + b) * 48 + v) * 256 + t;
          q[0] = acc.m[a][b][v];
          q[16 * 256] = acc.w[a][b][v];
          q[32 * 256] = acc.hc[a][b][v];
        }
    return;
  }
  ibs_epilogue(acc, o, I, J, wr, wc, lane);
}


// Pipelined form: the same tile, Grams, K order and arithmetic as
// ibs_mfma_tile, with the chunk boundary taken out of the critical path.
// ibs_mfma_tile reads a chunk's words from LDS and expands its first step
// after the chunk barrier, with no MFMA in flight; here every stage of chunk
// k + 1 happens while the MFMAs of chunk k run:
//   - chunk c is fetched from global memory two chunks ahead (in the middle
//     of chunk c - 2, right after the previous fetch was stored) and stored
//     to LDS buffer c % 2 in the middle of chunk c - 2;
//   - one barrier at the start of each chunk orders those stores before the
//     reads of the next chunk, and the reads of a buffer before it is
//     overwritten two chunks later;
//   - a lane reads the next chunk's words in two halves, words 0-3 during
//     step 4 (words 0-3 of the current chunk are expanded by then) and words
//     4-7 during step 7, into the same registers, and the first step of the
//     next chunk is expanded during the last step of the current one.
// Variant 7 of the matrix-core path.
template <bool kHints>
__device__ __forceinline__ void ibs_mfma_tile_pipe(const uint32_t* __restrict__ T, int64_t wp,
                                                   int64_t I, int64_t J, const IbsOut& o,
                                                   lds_t* smem, int64_t c0 = 0, int64_t c1 = -1,
                                                   int32_t* __restrict__ part = nullptr) {
  constexpr int kBuf = kT * kLdsStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int g = lane >> 5;
  const int rl = lane & 31;

  const int lrow = t >> 2;
  const int lq = (t & 3) * 4;
  const uint32_t* pa = T + (I * kT + lrow) * wp + lq;
  const uint32_t* pb = T + (J * kT + lrow) * wp + lq;
  const int64_t half = 64 * wp;
  uint4 ga0, ga1, gb0, gb1;
  auto gload = [&](int64_t kc) {
    ga0 = *reinterpret_cast<const uint4*>(pa + kc);
    ga1 = *reinterpret_cast<const uint4*>(pa + half + kc);
    gb0 = *reinterpret_cast<const uint4*>(pb + kc);
    gb1 = *reinterpret_cast<const uint4*>(pb + half + kc);
  };
  auto lstore = [&](int buf) {
    lds_st4(&(sA + buf * kBuf)[lrow * kLdsStride + lq], ga0);
    lds_st4(&(sA + buf * kBuf)[(lrow + 64) * kLdsStride + lq], ga1);
    lds_st4(&(sB + buf * kBuf)[lrow * kLdsStride + lq], gb0);
    lds_st4(&(sB + buf * kBuf)[(lrow + 64) * kLdsStride + lq], gb1);
  };
  uint32_t wa[2][8], wb[2][8];
  // words 4*h .. 4*h + 3 of this lane's two A rows and two B rows
  auto lread = [&](int buf, int h) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const lds_t* ra = &(sA + buf * kBuf)[(wr * 64 + x * 32 + rl) * kLdsStride + g * 8 + 4 * h];
      const lds_t* rb = &(sB + buf * kBuf)[(wc * 64 + x * 32 + rl) * kLdsStride + g * 8 + 4 * h];
      const uint4 a = lds_ld4(ra);
      const uint4 b = lds_ld4(rb);
      wa[x][4 * h] = a.x; wa[x][4 * h + 1] = a.y; wa[x][4 * h + 2] = a.z; wa[x][4 * h + 3] = a.w;
      wb[x][4 * h] = b.x; wb[x][4 * h + 1] = b.y; wb[x][4 * h + 2] = b.z; wb[x][4 * h + 3] = b.w;
    }
  };

  IbsAcc acc;
  zero_acc(acc);
  // The loop body has no branches, so the scheduler can interleave every
  // stage with the MFMAs: fetches past the last chunk re-read the last chunk
  // (in bounds), and the stores, reads and expansions past it fill buffers
  // and registers nothing reads afterwards.
  const int64_t nch = (c1 < 0 ? wp / kKW : c1) - c0;
  auto fetch = [&](int64_t c) { gload((c0 + (c < nch ? c : nch - 1)) * kKW); };
  fetch(0);
  lstore(0);
  fetch(1);
  lstore(1);
  fetch(2);
  __syncthreads();
  lread(0, 0);
  lread(0, 1);
  Feat4 fa[2], fb[2];
  fa[0] = expand_a(wa[0][0]); fa[1] = expand_a(wa[1][0]);
  fb[0] = expand_b(wb[0][0]); fb[1] = expand_b(wb[1][0]);
  for (int64_t k = 0; k < nch; ++k) {
    const int buf = (int)(k & 1);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kKW / 2; ++s) {
      if (s == 3) {
        lstore(buf);                                  // chunk k + 2
        fetch(k + 3);
      }
      if (s == 4) lread(buf ^ 1, 0);                  // words 0-3 of chunk k + 1
      if (s == 7) lread(buf ^ 1, 1);                  // words 4-7
      Feat4 na[2], nb[2];
      const int sn = (s + 1) & 7;                     // next step's word (chunk k + 1 at s = 7)
      na[0] = expand_a(wa[0][sn]); na[1] = expand_a(wa[1][sn]);
      nb[0] = expand_b(wb[0][sn]); nb[1] = expand_b(wb[1][sn]);
      mfma_step(acc, fa, fb);
      if constexpr (kHints) {
        // the step's memory operations first (LDS stores and global fetches
        // at step 3, LDS reads at steps 4 and 7), then one MFMA and up to six
        // VALU instructions, sixteen times
        if (s == 3) {
          __builtin_amdgcn_sched_group_barrier(0x200, 4, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 4, 0);
        }
        if (s == 4 || s == 7) __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);
        }
      }
      fa[0] = na[0]; fa[1] = na[1];
      fb[0] = nb[0]; fb[1] = nb[1];
    }
  }
  if (part) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          int32_t* q = part + ((a * 2 + b) * 48 + v) * 256 + t;
          q[0] = acc.m[a][b][v];
          q[16 * 256] = acc.w[a][b][v];
          q[32 * 256] = acc.hc[a][b][v];
        }
    return;
  }
  ibs_epilogue(acc, o, I, J, wr, wc, lane);
}

// Eight-wave form (variant 5): 512 threads = 8 waves in a 2x4 grid over the
// same 128x128 tile, each wave 64x32 = 2x1 blocks and three accumulator sets
// (96 accumulator registers), so two waves share each SIMD and one wave's
// feature expansion can run while the other's MFMAs do.  Each wave expands
// three words per step for eight MFMAs (the four-wave form: four words for
// sixteen).
struct IbsAcc21 {
  v16i m[2], w[2], hc[2];
};

__device__ __forceinline__ void mfma_step21(IbsAcc21& acc, const Feat4 (&fa)[2], const Feat4& fb) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (q == 0)
        acc.m[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].m, fb.m, acc.m[a], 0, 0, 0);
      else if (q == 1)
        acc.w[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].w, fb.w, acc.w[a], 0, 0, 0);
      else if (q == 2)
        acc.hc[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].h, fb.h, acc.hc[a], 0, 0, 0);
      else
        acc.hc[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a].c, fb.c, acc.hc[a], 0, 0, 0);
    }
}

template <bool kHints>
__device__ __forceinline__ void ibs_mfma_tile_w8(const uint32_t* __restrict__ T, int64_t wp,
                                                 int64_t I, int64_t J, const IbsOut& o,
                                                 lds_t* smem) {
  constexpr int kBuf = kT * kLdsStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 2, wc = wid & 3;
  const int g = lane >> 5;
  const int rl = lane & 31;

  // this thread's share of a chunk: row t/4 of both tiles, words 4*(t%4)..+3
  const int lrow = t >> 2;
  const int lq = (t & 3) * 4;
  const uint32_t* pa = T + (I * kT + lrow) * wp + lq;
  const uint32_t* pb = T + (J * kT + lrow) * wp + lq;
  uint4 ga, gb;
  auto gload = [&](int64_t kc) {
    ga = *reinterpret_cast<const uint4*>(pa + kc);
    gb = *reinterpret_cast<const uint4*>(pb + kc);
  };
  auto lstore = [&](int buf) {
    lds_st4(&(sA + buf * kBuf)[lrow * kLdsStride + lq], ga);
    lds_st4(&(sB + buf * kBuf)[lrow * kLdsStride + lq], gb);
  };

  IbsAcc21 acc;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    acc.m[a] = (v16i){0};
    acc.w[a] = (v16i){0};
    acc.hc[a] = (v16i){0};
  }
  const int64_t nchunks = wp / kKW;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int64_t k = 0; k < nchunks; ++k) {
    const int buf = (int)(k & 1);
    if (k + 1 < nchunks) gload((k + 1) * kKW);
    uint32_t wa[2][8], wb[8];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const lds_t* ra = &(sA + buf * kBuf)[(wr * 64 + x * 32 + rl) * kLdsStride + g * 8];
      const uint4 a0 = lds_ld4(ra);
      const uint4 a1 = lds_ld4(ra + 4);
      wa[x][0] = a0.x; wa[x][1] = a0.y; wa[x][2] = a0.z; wa[x][3] = a0.w;
      wa[x][4] = a1.x; wa[x][5] = a1.y; wa[x][6] = a1.z; wa[x][7] = a1.w;
    }
    {
      const lds_t* rb = &(sB + buf * kBuf)[(wc * 32 + rl) * kLdsStride + g * 8];
      const uint4 b0 = lds_ld4(rb);
      const uint4 b1 = lds_ld4(rb + 4);
      wb[0] = b0.x; wb[1] = b0.y; wb[2] = b0.z; wb[3] = b0.w;
      wb[4] = b1.x; wb[5] = b1.y; wb[6] = b1.z; wb[7] = b1.w;
    }
    Feat4 fa[2], fb;
    fa[0] = expand_a(wa[0][0]); fa[1] = expand_a(wa[1][0]);
    fb = expand_b(wb[0]);
#pragma unroll
    for (int s = 0; s < kKW / 2; ++s) {
      Feat4 na[2], nb;
      if (s + 1 < kKW / 2) {
        na[0] = expand_a(wa[0][s + 1]); na[1] = expand_a(wa[1][s + 1]);
        nb = expand_b(wb[s + 1]);
      }
      mfma_step21(acc, fa, fb);
      if constexpr (kHints) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 9, 0);
        }
      }
      if (s + 1 < kKW / 2) {
        fa[0] = na[0]; fa[1] = na[1];
        fb = nb;
      }
    }
    if (k + 1 < nchunks) lstore(buf ^ 1);
    __syncthreads();
  }
  const bool mirror = (I != J);
  auto stores = [&](auto width) {
    constexpr bool kU16 = decltype(width)::value;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      uint32_t n[16], z[16], one[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        n[v] = (uint32_t)acc.m[a][v];
        z[v] = (uint32_t)acc.hc[a][v] >> 1;
        one[v] = (n[v] - (uint32_t)acc.w[a][v]) >> 1;
      }
      store_block<kU16>(o, I * kT + wr * 64 + a * 32, J * kT + wc * 32 + (lane & 31), mirror,
                        lane, n, z, one);
    }
  };
  if (o.u16) stores(std::true_type{});
  else stores(std::false_type{});
}

// Unpipelined reference form (variant 2).
__device__ __forceinline__ void ibs_mfma_tile_simple(const uint32_t* __restrict__ T, int64_t wp,
                                                     int64_t I, int64_t J, const IbsOut& o,
                                                     lds_t* smem) {
  lds_t* const sA = smem;
  lds_t* const sB = smem + kT * kLdsStride;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const uint32_t* gA = T + I * kT * wp;
  const uint32_t* gB = T + J * kT * wp;
  IbsAcc acc;
  zero_acc(acc);
  for (int64_t kc = 0; kc < wp; kc += kKW) {
    for (int h = 0; h < 2; ++h) {
      const int r = (t >> 2) + 64 * h;
      const int q = t & 3;
      const uint4 a = *reinterpret_cast<const uint4*>(gA + r * wp + kc + q * 4);
      const uint4 b = *reinterpret_cast<const uint4*>(gB + r * wp + kc + q * 4);
      lds_st4(&sA[r * kLdsStride + q * 4], a);
      lds_st4(&sB[r * kLdsStride + q * 4], b);
    }
    __syncthreads();
    const int g = lane >> 5;
    const int rl = lane & 31;
#pragma unroll 2
    for (int s = 0; s < kKW / 2; ++s) {
      const int kw = g * (kKW / 2) + s;
      Feat4 fa[2], fb[2];
      for (int x = 0; x < 2; ++x) {
        fa[x] = expand_a(sA[(wr * 64 + x * 32 + rl) * kLdsStride + kw]);
        fb[x] = expand_b(sB[(wc * 64 + x * 32 + rl) * kLdsStride + kw]);
      }
      mfma_step(acc, fa, fb);
    }
    __syncthreads();
  }
  ibs_epilogue(acc, o, I, J, wr, wc, lane);
}


// ---- popcount path --------------------------------------------------------------
// Block: 256 threads over a 64x64 tile, 4x4 pairs per thread; K runs over
// 32-variant plane words in chunks of 16 staged through LDS.
constexpr int kP = kIbsPopcTile;
constexpr int kPW = kIbsPopcKWords;

__device__ __forceinline__ void ibs_popc_tile(const uint32_t* __restrict__ P, int64_t rows_pad,
                                              int64_t words_pad, int64_t I, int64_t J,
                                              const IbsOut& o, lds_t* smem) {
  lds_t* const sA = smem;
  lds_t* const sB = smem + kPW * 3 * kP;
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  uint32_t cn[4][4], cz[4][4], co[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) cn[r][c] = cz[r][c] = co[r][c] = 0;

  for (int64_t kc = 0; kc < words_pad; kc += kPW) {
    // kPW*3 rows of 64 words for each operand: 768 uint4, 3 per thread
    for (int h = 0; h < 3; ++h) {
      const int e = t + 256 * h;          // uint4 index
      const int row = e >> 4;             // (word, plane) row, 0..47
      const int col = (e & 15) * 4;       // sample offset
      const int64_t gw = (kc * 3 + row) * rows_pad;
      const uint4 a = *reinterpret_cast<const uint4*>(P + gw + I * kP + col);
      const uint4 b = *reinterpret_cast<const uint4*>(P + gw + J * kP + col);
      lds_st4(&sA[row * kP + col], a);
      lds_st4(&sB[row * kP + col], b);
    }
    __syncthreads();
#pragma unroll 4
    for (int w = 0; w < kPW; ++w) {
      const uint4 ah = lds_ld4(&sA[(w * 3 + 0) * kP + ty * 4]);
      const uint4 al = lds_ld4(&sA[(w * 3 + 1) * kP + ty * 4]);
      const uint4 am = lds_ld4(&sA[(w * 3 + 2) * kP + ty * 4]);
      const uint4 bh = lds_ld4(&sB[(w * 3 + 0) * kP + tx * 4]);
      const uint4 bl = lds_ld4(&sB[(w * 3 + 1) * kP + tx * 4]);
      const uint4 bm = lds_ld4(&sB[(w * 3 + 2) * kP + tx * 4]);
      const uint32_t AH[4] = {ah.x, ah.y, ah.z, ah.w}, AL[4] = {al.x, al.y, al.z, al.w},
                     AM[4] = {am.x, am.y, am.z, am.w};
      const uint32_t BH[4] = {bh.x, bh.y, bh.z, bh.w}, BL[4] = {bl.x, bl.y, bl.z, bl.w},
                     BM[4] = {bm.x, bm.y, bm.z, bm.w};
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          const uint32_t m = AM[r] & BM[c];
          const uint32_t xh = AH[r] ^ BH[c];
          const uint32_t xl = AL[r] ^ BL[c];
          cn[r][c] += __builtin_popcount(m);
          cz[r][c] += __builtin_popcount(xh & xl & m);
          co[r][c] += __builtin_popcount((xh ^ xl) & m);
        }
    }
    __syncthreads();
  }
  const bool mirror = (I != J);
  auto stores = [&](auto width) {
    constexpr bool kU16 = decltype(width)::value;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        store_counts_w<kU16>(o, I * kP + ty * 4 + r, J * kP + tx * 4 + c, mirror, cn[r][c],
                             cz[r][c], co[r][c]);
  };
  if (o.u16) stores(std::true_type{});
  else stores(std::false_type{});
}


// ---- matrix-core path, fp4 operands -----------------------------------------------
// The same four Grams on the fp4 (e2m1) matrix cores: v_mfma_f32_32x32x64_f8f6f4
// with both operands in fp4, unscaled (mfma_fp4).  Every feature value is -1, 0 or
// +1, exact in e2m1 (0b0010 = 1.0, 0b1010 = -1.0); every partial sum is an
// integer of magnitude <= V, exact in the fp32 accumulator while V < 2^24
// (the caller falls back to the int8 kernel above that).  One MFMA lane holds
// 32 K values = two 2-bit words; a word's codes are spread to nibbles (even
// codes, then odd codes -- the same K order on both sides) and each nibble is
// mapped to the four features with three-input bit operations.
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));

struct Fp4Feat {
  v8i m, w, h, c;
};

// Eight codes, one per nibble (bits 2-3 of each nibble clear) -> the fp4
// nibbles of m, w, h and c (negc: -c, for the B side).
__device__ __forceinline__ void fp4_nibbles(uint32_t x, bool negc, uint32_t& m, uint32_t& w,
                                            uint32_t& h, uint32_t& c) {
  constexpr uint32_t kMag = 0x22222222u;  // nibble bit 1: exponent LSB, |value| = 1.0
  const uint32_t y = x << 1;              // code low bit now at nibble bit 1
  m = (x | ~y) & kMag;                    // code != 01
  const uint32_t het = x & ~y & kMag;     // code 10
  w = m | (het << 2);                     // sign (nibble bit 3) for heterozygotes
  h = ~(x ^ y) & kMag;                    // code 00 or 11
  const uint32_t neg = negc ? (x & y & kMag) : (~x & ~y & kMag);  // 11 on B, 00 on A
  c = h | (neg << 2);
}

__device__ __forceinline__ Fp4Feat fp4_expand(uint32_t w0, uint32_t w1, bool negc) {
  Fp4Feat f;
  const uint32_t xs[4] = {w0 & 0x33333333u, (w0 >> 2) & 0x33333333u, w1 & 0x33333333u,
                          (w1 >> 2) & 0x33333333u};
  f.m = (v8i){0}; f.w = (v8i){0}; f.h = (v8i){0}; f.c = (v8i){0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t m, w, h, c;
    fp4_nibbles(xs[q], negc, m, w, h, c);
    f.m[q] = (int)m; f.w[q] = (int)w; f.h[q] = (int)h; f.c[q] = (int)c;
  }
  return f;
}

struct Fp4Acc {
  v16f m[2][2], w[2][2], hc[2][2];
};

// Formats 4/4 = e2m1 for A and B, scale operands 0: the compiler then emits
// the unscaled v_mfma_f32_32x32x64_f8f6f4 (one 64-bit instruction, no scale
// register), which computes the plain product.  With unit scales written out
// (127 in e8m0) it emits the scaled form, a 128-bit instruction pair that
// issues more slowly: 4% on the IBS tile, the same results.
__device__ __forceinline__ v16f mfma_fp4(const v8i& a, const v8i& b, const v16f& c) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 0, 0, 0);
}

__device__ __forceinline__ void fp4_step(Fp4Acc& acc, const Fp4Feat (&fa)[2],
                                         const Fp4Feat (&fb)[2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.m[a][b] = mfma_fp4(fa[a].m, fb[b].m, acc.m[a][b]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.w[a][b] = mfma_fp4(fa[a].w, fb[b].w, acc.w[a][b]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.hc[a][b] = mfma_fp4(fa[a].h, fb[b].h, acc.hc[a][b]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.hc[a][b] = mfma_fp4(fa[a].c, fb[b].c, acc.hc[a][b]);
}

// zshift: 1 when the hc accumulator holds 2 IBS0 (G_h - G_c), 0 when it
// holds IBS0 (the opposite-homozygote Gram set).
__device__ __forceinline__ void fp4_epilogue(const Fp4Acc& acc, const IbsOut& o, int64_t I,
                                             int64_t J, int wr, int wc, int lane,
                                             int zshift = 1) {
  const bool mirror = (I != J);
  auto stores = [&](auto width) {
    constexpr bool kU16 = decltype(width)::value;
  #pragma unroll
    for (int a = 0; a < 2; ++a)
  #pragma unroll
      for (int b = 0; b < 2; ++b) {
        uint32_t n[16], z[16], one[16];
  #pragma unroll
        for (int v = 0; v < 16; ++v) {
          n[v] = (uint32_t)(int)acc.m[a][b][v];
          z[v] = (uint32_t)(int)acc.hc[a][b][v] >> zshift;
          one[v] = (n[v] - (uint32_t)(int)acc.w[a][b][v]) >> 1;
        }
        store_block<kU16>(o, I * kT + wr * 64 + a * 32, J * kT + wc * 64 + b * 32 + (lane & 31), mirror,
                    lane, n, z, one);
      }
  };
  if (o.u16) stores(std::true_type{});
  else stores(std::false_type{});
}

__device__ __forceinline__ void ibs_fp4_tile(const uint32_t* __restrict__ T, int64_t wp,
                                             int64_t I, int64_t J, const IbsOut& o,
                                             lds_t* smem) {
  constexpr int kBuf = kT * kLdsStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int g = lane >> 5;
  const int rl = lane & 31;
  const int lrow = t >> 2;
  const int lq = (t & 3) * 4;
  const uint32_t* pa = T + (I * kT + lrow) * wp + lq;
  const uint32_t* pb = T + (J * kT + lrow) * wp + lq;
  const int64_t half = 64 * wp;
  uint4 ga0, ga1, gb0, gb1;
  auto gload = [&](int64_t kc) {
    ga0 = *reinterpret_cast<const uint4*>(pa + kc);
    ga1 = *reinterpret_cast<const uint4*>(pa + half + kc);
    gb0 = *reinterpret_cast<const uint4*>(pb + kc);
    gb1 = *reinterpret_cast<const uint4*>(pb + half + kc);
  };
  auto lstore = [&](int buf) {
    lds_st4(&(sA + buf * kBuf)[lrow * kLdsStride + lq], ga0);
    lds_st4(&(sA + buf * kBuf)[(lrow + 64) * kLdsStride + lq], ga1);
    lds_st4(&(sB + buf * kBuf)[lrow * kLdsStride + lq], gb0);
    lds_st4(&(sB + buf * kBuf)[(lrow + 64) * kLdsStride + lq], gb1);
  };
  Fp4Acc acc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc.m[a][b] = (v16f){0};
      acc.w[a][b] = (v16f){0};
      acc.hc[a][b] = (v16f){0};
    }
  const int64_t nchunks = wp / kKW;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int64_t k = 0; k < nchunks; ++k) {
    const int buf = (int)(k & 1);
    if (k + 1 < nchunks) gload((k + 1) * kKW);
    uint32_t wa[2][8], wb[2][8];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const lds_t* ra = &(sA + buf * kBuf)[(wr * 64 + x * 32 + rl) * kLdsStride + g * 8];
      const lds_t* rb = &(sB + buf * kBuf)[(wc * 64 + x * 32 + rl) * kLdsStride + g * 8];
      const uint4 a0 = lds_ld4(ra);
      const uint4 a1 = lds_ld4(ra + 4);
      const uint4 b0 = lds_ld4(rb);
      const uint4 b1 = lds_ld4(rb + 4);
      wa[x][0] = a0.x; wa[x][1] = a0.y; wa[x][2] = a0.z; wa[x][3] = a0.w;
      wa[x][4] = a1.x; wa[x][5] = a1.y; wa[x][6] = a1.z; wa[x][7] = a1.w;
      wb[x][0] = b0.x; wb[x][1] = b0.y; wb[x][2] = b0.z; wb[x][3] = b0.w;
      wb[x][4] = b1.x; wb[x][5] = b1.y; wb[x][6] = b1.z; wb[x][7] = b1.w;
    }
    Fp4Feat fa[2], fb[2];
    fa[0] = fp4_expand(wa[0][0], wa[0][1], false);
    fa[1] = fp4_expand(wa[1][0], wa[1][1], false);
    fb[0] = fp4_expand(wb[0][0], wb[0][1], true);
    fb[1] = fp4_expand(wb[1][0], wb[1][1], true);
#pragma unroll
    for (int s = 0; s < kKW / 4; ++s) {
      Fp4Feat na[2], nb[2];
      if (s + 1 < kKW / 4) {
        na[0] = fp4_expand(wa[0][2 * s + 2], wa[0][2 * s + 3], false);
        na[1] = fp4_expand(wa[1][2 * s + 2], wa[1][2 * s + 3], false);
        nb[0] = fp4_expand(wb[0][2 * s + 2], wb[0][2 * s + 3], true);
        nb[1] = fp4_expand(wb[1][2 * s + 2], wb[1][2 * s + 3], true);
      }
      fp4_step(acc, fa, fb);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
      }
      if (s + 1 < kKW / 4) {
        fa[0] = na[0]; fa[1] = na[1];
        fb[0] = nb[0]; fb[1] = nb[1];
      }
    }
    if (k + 1 < nchunks) lstore(buf ^ 1);
    __syncthreads();
  }
  fp4_epilogue(acc, o, I, J, wr, wc, lane);
}

// Pipelined fp4 tile (variant 8, the default): ibs_mfma_tile_pipe's
// schedule on the fp4 matrix cores, with a cheaper Gram set than
// ibs_fp4_tile.  One MFMA lane takes two 2-bit words (32 variants) per step,
// so a chunk is four steps; the fetch and LDS store of chunk k + 2 happen at
// step 1, the reads of chunk k + 1 at steps 2 (words 0-3) and 3 (words 4-7).
//
// Grams: features m = [called], w = +1 homozygote / -1 heterozygote,
// a1 = [homozygous A1], a2 = [homozygous A2] (all 0 when missing), the same
// on both sides:
//   N = G(m, m),  IBS1 = (N - G(w, w)) / 2,  IBS0 = G(a2, a1) + G(a1, a2),
// the two products of IBS0 sharing one accumulator.  Of the four-product
// sets that fit three accumulators this one needs the fewest bit operations:
// only w carries a sign.
//
// Expansion of one word w (code j at bits 2j, 2j + 1) into the nibbles of
// its even codes (nibble n = code 2n) and of its odd codes (nibble n = code
// 2n + 1): with X holding each code's high bit and Y its low bit at bit 1 of
// the code's nibble (even: X = w, Y = w << 1; odd: X = w >> 2, Y = w >> 1)
// and K = bit 1 of every nibble,
//   m = K & (X | ~Y),  w = m | (K & X & ~Y) << 2,  a1 = K & ~X & ~Y,
//   a2 = K & X & Y;
// bits 0, 2 of every nibble stay 0 and bit 3 is the sign, so every value is
// 0 or +-1.0 in e2m1: four v_bitop3 and one shift-or per parity of a word.
// The even nibbles of a word fill one dword of a feature and the odd nibbles
// the next; A and B use the same order.
constexpr uint32_t kNibK = 0x22222222u;
constexpr int kB3Mx = 0xa2;   // K & (X | ~Y): S0 = X, S1 = Y, S2 = K
constexpr int kB3Het = 0x20;  // K & X & ~Y
constexpr int kB3Hom = 0x82;  // K & ~(X ^ Y)
constexpr int kB3A1 = 0x02;   // K & ~X & ~Y
constexpr int kB3A2 = 0x80;   // K & X & Y

__device__ __forceinline__ void fp4_parity(uint32_t X, uint32_t Y, uint32_t& m, uint32_t& w,
                                           uint32_t& a1, uint32_t& a2) {
  m = __builtin_amdgcn_bitop3_b32(X, Y, kNibK, kB3Mx);
  const uint32_t het = __builtin_amdgcn_bitop3_b32(X, Y, kNibK, kB3Het);
  w = (het << 2) | m;
  a1 = __builtin_amdgcn_bitop3_b32(X, Y, kNibK, kB3A1);
  a2 = __builtin_amdgcn_bitop3_b32(X, Y, kNibK, kB3A2);
}

// Features of two words, stored in Fp4Feat as m, w, h = a1, c = a2.
__device__ __forceinline__ Fp4Feat fp4_expand2(uint32_t w0, uint32_t w1) {
  Fp4Feat f;
  f.m = (v8i){0}; f.w = (v8i){0}; f.h = (v8i){0}; f.c = (v8i){0};
  const uint32_t ws[2] = {w0, w1};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint32_t m, w, a1, a2;
    fp4_parity(ws[q], ws[q] << 1, m, w, a1, a2);
    f.m[2 * q] = (int)m; f.w[2 * q] = (int)w; f.h[2 * q] = (int)a1; f.c[2 * q] = (int)a2;
    fp4_parity(ws[q] >> 2, ws[q] >> 1, m, w, a1, a2);
    f.m[2 * q + 1] = (int)m; f.w[2 * q + 1] = (int)w; f.h[2 * q + 1] = (int)a1;
    f.c[2 * q + 1] = (int)a2;
  }
  return f;
}

// acc.hc accumulates IBS0 itself here.
__device__ __forceinline__ void fp4_step_opp(Fp4Acc& acc, const Fp4Feat (&fa)[2],
                                             const Fp4Feat (&fb)[2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.m[a][b] = mfma_fp4(fa[a].m, fb[b].m, acc.m[a][b]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.w[a][b] = mfma_fp4(fa[a].w, fb[b].w, acc.w[a][b]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.hc[a][b] = mfma_fp4(fa[a].c, fb[b].h, acc.hc[a][b]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.hc[a][b] = mfma_fp4(fa[a].h, fb[b].c, acc.hc[a][b]);
}

__device__ __forceinline__ void ibs_fp4_tile_pipe(const uint32_t* __restrict__ T, int64_t wp,
                                                  int64_t I, int64_t J, const IbsOut& o,
                                                  lds_t* smem, int64_t c0 = 0, int64_t c1 = -1,
                                                  int32_t* __restrict__ part = nullptr) {
  constexpr int kBuf = kT * kLdsStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int g = lane >> 5;
  const int rl = lane & 31;
  const int lrow = t >> 2;
  const int lq = (t & 3) * 4;
  const uint32_t* pa = T + (I * kT + lrow) * wp + lq;
  const uint32_t* pb = T + (J * kT + lrow) * wp + lq;
  const int64_t half = 64 * wp;
  uint4 ga0, ga1, gb0, gb1;
  auto gload = [&](int64_t kc) {
    ga0 = *reinterpret_cast<const uint4*>(pa + kc);
    ga1 = *reinterpret_cast<const uint4*>(pa + half + kc);
    gb0 = *reinterpret_cast<const uint4*>(pb + kc);
    gb1 = *reinterpret_cast<const uint4*>(pb + half + kc);
  };
  auto lstore = [&](int buf) {
    lds_st4(&(sA + buf * kBuf)[lrow * kLdsStride + lq], ga0);
    lds_st4(&(sA + buf * kBuf)[(lrow + 64) * kLdsStride + lq], ga1);
    lds_st4(&(sB + buf * kBuf)[lrow * kLdsStride + lq], gb0);
    lds_st4(&(sB + buf * kBuf)[(lrow + 64) * kLdsStride + lq], gb1);
  };
  uint32_t wa[2][8], wb[2][8];
  auto lread = [&](int buf, int h) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const lds_t* ra = &(sA + buf * kBuf)[(wr * 64 + x * 32 + rl) * kLdsStride + g * 8 + 4 * h];
      const lds_t* rb = &(sB + buf * kBuf)[(wc * 64 + x * 32 + rl) * kLdsStride + g * 8 + 4 * h];
      const uint4 a = lds_ld4(ra);
      const uint4 b = lds_ld4(rb);
      wa[x][4 * h] = a.x; wa[x][4 * h + 1] = a.y; wa[x][4 * h + 2] = a.z; wa[x][4 * h + 3] = a.w;
      wb[x][4 * h] = b.x; wb[x][4 * h + 1] = b.y; wb[x][4 * h + 2] = b.z; wb[x][4 * h + 3] = b.w;
    }
  };
  Fp4Acc acc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc.m[a][b] = (v16f){0};
      acc.w[a][b] = (v16f){0};
      acc.hc[a][b] = (v16f){0};
    }
  const int64_t nch = (c1 < 0 ? wp / kKW : c1) - c0;
  auto fetch = [&](int64_t c) { gload((c0 + (c < nch ? c : nch - 1)) * kKW); };
  fetch(0);
  lstore(0);
  fetch(1);
  lstore(1);
  fetch(2);
  __syncthreads();
  lread(0, 0);
  lread(0, 1);
  Fp4Feat fa[2], fb[2];
  fa[0] = fp4_expand2(wa[0][0], wa[0][1]);
  fa[1] = fp4_expand2(wa[1][0], wa[1][1]);
  fb[0] = fp4_expand2(wb[0][0], wb[0][1]);
  fb[1] = fp4_expand2(wb[1][0], wb[1][1]);
  for (int64_t k = 0; k < nch; ++k) {
    const int buf = (int)(k & 1);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kKW / 4; ++s) {
      if (s == 1) {
        lstore(buf);                                  // chunk k + 2
        fetch(k + 3);
      }
      if (s == 2) lread(buf ^ 1, 0);                  // words 0-3 of chunk k + 1
      if (s == 3) lread(buf ^ 1, 1);                  // words 4-7
      const int sn = 2 * ((s + 1) & 3);               // next step's first word
      Fp4Feat na[2], nb[2];
      na[0] = fp4_expand2(wa[0][sn], wa[0][sn + 1]);
      na[1] = fp4_expand2(wa[1][sn], wa[1][sn + 1]);
      nb[0] = fp4_expand2(wb[0][sn], wb[0][sn + 1]);
      nb[1] = fp4_expand2(wb[1][sn], wb[1][sn + 1]);
      fp4_step_opp(acc, fa, fb);
      if (s == 1) {
        __builtin_amdgcn_sched_group_barrier(0x200, 4, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 4, 0);
      }
      if (s >= 2) __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
      // seven VALU per MFMA (the expansion is 104 per 16): the unscaled fp4
      // MFMA hides about six, so a more even spread than eight per group
      // leaves less VALU exposed (2% on the whole call)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 7, 0);
      }
      fa[0] = na[0]; fa[1] = na[1];
      fb[0] = nb[0]; fb[1] = nb[1];
    }
  }
  if (part) {   // the raw sums as int32 (exact integers), laid out as ibs_mfma_tile's
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          int32_t* q = part + ((a * 2 + b) * 48 + v) * 256 + t;
          q[0] = (int32_t)acc.m[a][b][v];
          q[16 * 256] = (int32_t)acc.w[a][b][v];
          q[32 * 256] = 2 * (int32_t)acc.hc[a][b][v];   // 2 IBS0, as G_h - G_c
        }
    return;
  }
  fp4_epilogue(acc, o, I, J, wr, wc, lane, 0);
}

// ---- matrix-core path, fp4 operands from the replicated layout ----------------------
// Same Grams and MFMA as above; the operand is the replicated layout (per 8
// variants, HR = high code bits and LR = low code bits at nibble bits 1 and 3,
// LR with ones at bits 0 and 2), so each feature word is ONE three-input bit
// function of (HR, LR, K = bit 1 of every nibble):
//   m = K & (hi | ~lo)                       +1 unless missing
//   w = K & (hi | ~lo)  |  ~K & hi & ~lo     sign at bit 3 for heterozygotes
//   h = K & ~(hi ^ lo)                       homozygotes
//   c = K & ~(hi ^ lo)  |  ~K & ~hi & ~lo    sign for homozygous A1 (A side)
//  -c = K & ~(hi ^ lo)  |  ~K & hi & lo      sign for homozygous A2 (B side)
// Bits 0 and 2 of every nibble evaluate to 0 because LR is 1 there and HR 0.
// A chunk is 256 variants = 64 words per row; one MFMA lane takes 4 groups
// (32 variants) per step.
constexpr int kRC = kIbsRepChunk;
constexpr int kRStride = kRC + 4;

// Truth tables of v_bitop3_b32 (result bit = table[S0*4 + S1*2 + S2]) with
// S0 = HR, S1 = LR, S2 = K; derived from the expressions above.
constexpr int kB3M = 0xa2, kB3W = 0xb2, kB3H = 0x82, kB3C = 0x83, kB3Cn = 0xc2;

__device__ __forceinline__ void rep_features(const uint4& p0, const uint4& p1, bool b_side,
                                             Fp4Feat& f) {
  constexpr uint32_t K = 0x22222222u;
  const uint32_t hr[4] = {p0.x, p0.z, p1.x, p1.z};
  const uint32_t lr[4] = {p0.y, p0.w, p1.y, p1.w};
  f.m = (v8i){0}; f.w = (v8i){0}; f.h = (v8i){0}; f.c = (v8i){0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    f.m[q] = (int)__builtin_amdgcn_bitop3_b32(hr[q], lr[q], K, kB3M);
    f.w[q] = (int)__builtin_amdgcn_bitop3_b32(hr[q], lr[q], K, kB3W);
    f.h[q] = (int)__builtin_amdgcn_bitop3_b32(hr[q], lr[q], K, kB3H);
    f.c[q] = (int)(b_side ? __builtin_amdgcn_bitop3_b32(hr[q], lr[q], K, kB3Cn)
                          : __builtin_amdgcn_bitop3_b32(hr[q], lr[q], K, kB3C));
  }
}

__device__ __forceinline__ void ibs_fp4rep_tile(const uint32_t* __restrict__ R, int64_t rp,
                                                int64_t I, int64_t J, const IbsOut& o,
                                                lds_t* smem) {
  constexpr int kBuf = kT * kRStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int g = lane >> 5;
  const int rl = lane & 31;
  // global -> LDS: 128 rows x 16 uint4 per operand; thread t takes uint4 (t + 256k)
  const uint32_t* baseA = R + I * kT * rp;
  const uint32_t* baseB = R + J * kT * rp;
  uint4 ga[8], gb[8];
  auto gload = [&](int64_t kc) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = t + 256 * k;
      const int64_t off = (int64_t)(e >> 4) * rp + kc + (e & 15) * 4;
      ga[k] = *reinterpret_cast<const uint4*>(baseA + off);
      gb[k] = *reinterpret_cast<const uint4*>(baseB + off);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = t + 256 * k;
      const int off = (e >> 4) * kRStride + (e & 15) * 4;
      lds_st4(&(sA + buf * kBuf)[off], ga[k]);
      lds_st4(&(sB + buf * kBuf)[off], gb[k]);
    }
  };
  Fp4Acc acc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc.m[a][b] = (v16f){0};
      acc.w[a][b] = (v16f){0};
      acc.hc[a][b] = (v16f){0};
    }
  const int64_t nchunks = rp / kRC;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int64_t k = 0; k < nchunks; ++k) {
    const int buf = (int)(k & 1);
    if (k + 1 < nchunks) gload((k + 1) * kRC);
#pragma unroll
    for (int s = 0; s < kRC / 16; ++s) {
      Fp4Feat fa[2], fb[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const lds_t* ra = &(sA + buf * kBuf)[(wr * 64 + x * 32 + rl) * kRStride + g * 32 + s * 8];
        const lds_t* rb = &(sB + buf * kBuf)[(wc * 64 + x * 32 + rl) * kRStride + g * 32 + s * 8];
        rep_features(lds_ld4(ra), lds_ld4(ra + 4),
                     false, fa[x]);
        rep_features(lds_ld4(rb), lds_ld4(rb + 4),
                     true, fb[x]);
      }
      fp4_step(acc, fa, fb);
    }
    if (k + 1 < nchunks) lstore(buf ^ 1);
    __syncthreads();
  }
  fp4_epilogue(acc, o, I, J, wr, wc, lane);
}

// ---- LD ---------------------------------------------------------------------
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

// Emission test for one pair (a < b <= a + window, b < nv checked by the
// caller): marks bit (b - a - 1) of row a and counts it.
__device__ __forceinline__ void ld_mark(const LdScratch& sc, int64_t a, int64_t b, double r2_min,
                                        int64_t n, int64_t sx, int64_t sy, int64_t sxx,
                                        int64_t syy, int64_t sxy) {
  if (ld_r2_reaches(n, sx, sy, sxx, syy, sxy, r2_min)) {
    const int64_t d = b - a - 1;
    atomicOr(&sc.bitmap[a * sc.bm_words + (d >> 5)], 1u << (d & 31));
    atomicAdd(&sc.rowcnt[a], 1u);
  }
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

__device__ __forceinline__ void ld_popc_tile(const uint32_t* __restrict__ P, int64_t words_pad,
                                             int64_t nv, int64_t rows_pad, int64_t I, int64_t J,
                                             int32_t window, double r2_min, const LdScratch& sc,
                                             lds_t* smem) {
  lds_t* const sA = smem;
  lds_t* const sB = smem + kLPW * 3 * kLP;
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
      lds_st4(&sA[row * kLP + col], a);
      lds_st4(&sB[row * kLP + col], b);
    }
    __syncthreads();
#pragma unroll 2
    for (int w = 0; w < kLPW; ++w) {
      const uint4 ap = lds_ld4(&sA[(w * 3 + 0) * kLP + ty * 4]);
      const uint4 aq = lds_ld4(&sA[(w * 3 + 1) * kLP + ty * 4]);
      const uint4 am = lds_ld4(&sA[(w * 3 + 2) * kLP + ty * 4]);
      const uint4 bp = lds_ld4(&sB[(w * 3 + 0) * kLP + tx * 4]);
      const uint4 bq = lds_ld4(&sB[(w * 3 + 1) * kLP + tx * 4]);
      const uint4 bm = lds_ld4(&sB[(w * 3 + 2) * kLP + tx * 4]);
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

__device__ __forceinline__ void ld_mfma_tile(const uint32_t* __restrict__ D, int64_t wn,
                                             int64_t nv, int64_t I, int64_t J, int32_t window,
                                             double r2_min, const LdScratch& sc, lds_t* smem) {
  constexpr int kBuf = kL * kLStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
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
    lds_st4(&(sA + buf * kBuf)[lrow * kLStride + lq], ga);
    lds_st4(&(sB + buf * kBuf)[lrow * kLStride + lq], gb);
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
      const lds_t* ra = &(sA + buf * kBuf)[(wr * 32 + rl) * kLStride + g * 8];
      const lds_t* rb = &(sB + buf * kBuf)[(wc * 32 + rl) * kLStride + g * 8];
      const uint4 a0 = lds_ld4(ra);
      const uint4 a1 = lds_ld4(ra + 4);
      const uint4 b0 = lds_ld4(rb);
      const uint4 b1 = lds_ld4(rb + 4);
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
  if (!active) return;   // nothing after this point synchronises

  // 32x32 accumulator layout: register v of lane l holds row
  // 8*(v/4) + 4*(l/32) + v%4 and column l%32.
  for (int v = 0; v < 16; ++v) {
    const int64_t a = a_lo + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int64_t b = b_lo + (lane & 31);
    if (!(a < b && b - a <= window && b < nv)) continue;
    ld_mark(sc, a, b, r2_min, s_n[v], s_x[v], s_y[v], s_xx[v], s_yy[v], s_xy[v]);
  }
}


// Pipelined fp4 form of the banded matrix-core tile (the default LD kernel):
// the same six Grams on v_mfma_f32_32x32x64_f8f6f4 with e2m1 operands
// (m, x, h are 0 or +-1, exact; fp32 sums exact below 2^24 samples), and
// the chunk schedule of ibs_fp4_tile_pipe: a chunk of 256 samples is four
// steps of 64 per MFMA lane (two 2-bit words), chunk k + 2 is fetched and
// stored to LDS at step 1 of chunk k, chunk k + 1 is read at steps 2 and 3,
// and its first step expanded during step 3.  Waves without a pair in the
// window run a loop that only stages, with the same barriers.
// Expansion of one parity of a word (see ibs_fp4_tile_pipe for X, Y, K):
//   m = K & (X | ~Y),  h = K & ~(X ^ Y),  x = h | (K & ~X & ~Y) << 2
// (x = -1 for homozygous A1, +1 for homozygous A2, 0 otherwise).
struct Fp4Feat3 {
  v8i m, x, h;
};

__device__ __forceinline__ Fp4Feat3 ld_fp4_expand2(uint32_t w0, uint32_t w1) {
  Fp4Feat3 f;
  f.m = (v8i){0}; f.x = (v8i){0}; f.h = (v8i){0};
  const uint32_t ws[2] = {w0, w1};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const uint32_t X = par ? ws[q] >> 2 : ws[q];
      const uint32_t Y = par ? ws[q] >> 1 : ws[q] << 1;
      const uint32_t h = __builtin_amdgcn_bitop3_b32(X, Y, kNibK, kB3Hom);
      const uint32_t neg = __builtin_amdgcn_bitop3_b32(X, Y, kNibK, kB3A1);
      f.m[2 * q + par] = (int)__builtin_amdgcn_bitop3_b32(X, Y, kNibK, kB3Mx);
      f.h[2 * q + par] = (int)h;
      f.x[2 * q + par] = (int)((neg << 2) | h);
    }
  }
  return f;
}

__device__ __forceinline__ void ld_fp4_tile_pipe(const uint32_t* __restrict__ D, int64_t wn,
                                                 int64_t nv, int64_t I, int64_t J, int32_t window,
                                                 double r2_min, const LdScratch& sc, lds_t* smem) {
  constexpr int kBuf = kL * kLStride;
  lds_t* const sA = smem;
  lds_t* const sB = smem + 2 * kBuf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int g = lane >> 5;
  const int rl = lane & 31;
  const int64_t a_lo = I * kL + wr * 32, b_lo = J * kL + wc * 32;
  const bool active = (b_lo + 31 > a_lo) && (b_lo - (a_lo + 31) <= window) && (b_lo < nv);

  const int lrow = t >> 2;
  const int lq = (t & 3) * 4;
  const uint32_t* pa = D + (I * kL + lrow) * wn + lq;
  const uint32_t* pb = D + (J * kL + lrow) * wn + lq;
  uint4 ga, gb;
  const int64_t nch = wn / kLW;
  auto fetch = [&](int64_t c) {
    const int64_t kc = (c < nch ? c : nch - 1) * kLW;
    ga = *reinterpret_cast<const uint4*>(pa + kc);
    gb = *reinterpret_cast<const uint4*>(pb + kc);
  };
  auto lstore = [&](int buf) {
    lds_st4(&(sA + buf * kBuf)[lrow * kLStride + lq], ga);
    lds_st4(&(sB + buf * kBuf)[lrow * kLStride + lq], gb);
  };
  fetch(0);
  lstore(0);
  fetch(1);
  lstore(1);
  fetch(2);
  __syncthreads();
  if (!active) {
    for (int64_t k = 0; k < nch; ++k) {
      __syncthreads();
      lstore((int)(k & 1));
      fetch(k + 3);
    }
    return;   // nothing after this point synchronises
  }
  uint32_t wa[8], wb[8];
  auto lread = [&](int buf, int h) {
    const uint4 a = lds_ld4(&(sA + buf * kBuf)[(wr * 32 + rl) * kLStride + g * 8 + 4 * h]);
    const uint4 b = lds_ld4(&(sB + buf * kBuf)[(wc * 32 + rl) * kLStride + g * 8 + 4 * h]);
    wa[4 * h] = a.x; wa[4 * h + 1] = a.y; wa[4 * h + 2] = a.z; wa[4 * h + 3] = a.w;
    wb[4 * h] = b.x; wb[4 * h + 1] = b.y; wb[4 * h + 2] = b.z; wb[4 * h + 3] = b.w;
  };
  v16f s_n = (v16f){0}, s_x = (v16f){0}, s_y = (v16f){0};
  v16f s_xx = (v16f){0}, s_yy = (v16f){0}, s_xy = (v16f){0};
  lread(0, 0);
  lread(0, 1);
  Fp4Feat3 fa = ld_fp4_expand2(wa[0], wa[1]), fb = ld_fp4_expand2(wb[0], wb[1]);
  for (int64_t k = 0; k < nch; ++k) {
    const int buf = (int)(k & 1);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kLW / 4; ++s) {
      if (s == 1) {
        lstore(buf);                                  // chunk k + 2
        fetch(k + 3);
      }
      if (s == 2) lread(buf ^ 1, 0);                  // words 0-3 of chunk k + 1
      if (s == 3) lread(buf ^ 1, 1);                  // words 4-7
      const int sn = 2 * ((s + 1) & 3);
      const Fp4Feat3 na = ld_fp4_expand2(wa[sn], wa[sn + 1]);
      const Fp4Feat3 nb = ld_fp4_expand2(wb[sn], wb[sn + 1]);
      s_n = mfma_fp4(fa.m, fb.m, s_n);
      s_x = mfma_fp4(fa.x, fb.m, s_x);
      s_y = mfma_fp4(fa.m, fb.x, s_y);
      s_xx = mfma_fp4(fa.h, fb.m, s_xx);
      s_yy = mfma_fp4(fa.m, fb.h, s_yy);
      s_xy = mfma_fp4(fa.x, fb.x, s_xy);
      if (s == 1) {
        __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
      }
      if (s >= 2) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 7, 0);
      }
      fa = na;
      fb = nb;
    }
  }
  // 32x32 accumulator layout: register v of lane l holds row
  // 8*(v/4) + 4*(l/32) + v%4 and column l%32.
  for (int v = 0; v < 16; ++v) {
    const int64_t a = a_lo + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int64_t b = b_lo + (lane & 31);
    if (!(a < b && b - a <= window && b < nv)) continue;
    ld_mark(sc, a, b, r2_min, (int64_t)(int)s_n[v], (int64_t)(int)s_x[v], (int64_t)(int)s_y[v],
            (int64_t)(int)s_xx[v], (int64_t)(int)s_yy[v], (int64_t)(int)s_xy[v]);
  }
}

// LDS words each body needs.
constexpr int kIbsMfmaSmem = 4 * kT * kLdsStride;
constexpr int kIbsMfmaSimpleSmem = 2 * kT * kLdsStride;
constexpr int kIbsPopcSmem = 2 * kPW * 3 * kP;
constexpr int kLdPopcSmem = 2 * kLPW * 3 * kLP;
constexpr int kLdMfmaSmem = 4 * kL * kLStride;
constexpr int kIbsRepSmem = 4 * kT * kRStride;
constexpr int kMaxTileSmem = kIbsMfmaSmem;
static_assert(kIbsMfmaSimpleSmem <= kMaxTileSmem && kIbsPopcSmem <= kMaxTileSmem &&
              kLdPopcSmem <= kMaxTileSmem && kLdMfmaSmem <= kMaxTileSmem, "LDS budget");

}  // namespace pg
