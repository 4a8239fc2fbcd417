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
#include "pg_internal.h"

namespace pg {

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

__device__ __forceinline__ void store_counts(const IbsOut& o, int64_t i, int64_t j, bool mirror,
                                             uint32_t n, uint32_t z, uint32_t one) {
  if (i >= o.m || j >= o.m) return;
  const uint32_t two = n - z - one;
  if (o.full) {
    const int64_t a = i * o.m + j;
    o.ibs0[a] = z; o.ibs1[a] = one; o.ibs2[a] = two; o.nonmiss[a] = n;
    if (mirror) {
      const int64_t b = j * o.m + i;
      o.ibs0[b] = z; o.ibs1[b] = one; o.ibs2[b] = two; o.nonmiss[b] = n;
    }
  } else if (i < j) {
    const int64_t a = i * o.m - i * (i + 1) / 2 + (j - i - 1);
    o.ibs0[a] = z; o.ibs1[a] = one; o.ibs2[a] = two; o.nonmiss[a] = n;
  }
}

// ---- matrix-core path ---------------------------------------------------------
// Block: 256 threads = 4 waves in a 2x2 grid over a 128x128 tile; each wave
// owns 64x64 = 2x2 blocks of v_mfma_i32_32x32x32_i8.  K runs over variants in
// chunks of 16 words (256 variants) staged through LDS.  Within a chunk, lane
// group g = lane/32 of a 32x32x32 step s reads word 8g + s of its row, i.e.
// the 16 K values of one MFMA lane are the 16 codes of one 2-bit word.
constexpr int kT = kIbsMfmaTile;
constexpr int kKW = kIbsMfmaKWords;
constexpr int kLdsStride = kKW + 4;   // words per LDS row (padding vs. bank conflicts)

__global__ __launch_bounds__(256, 1) void k_ibs_mfma(const uint32_t* __restrict__ T, int64_t wp,
                                                     int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t sA[kT * kLdsStride];
  __shared__ __attribute__((aligned(16))) uint32_t sB[kT * kLdsStride];
  int64_t I, J;
  tri_tile(blockIdx.x, nt, I, J);
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const uint32_t* gA = T + I * kT * wp;
  const uint32_t* gB = T + J * kT * wp;

  v16i acc_m[2][2], acc_w[2][2], acc_hc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      acc_m[a][b] = (v16i){0};
      acc_w[a][b] = (v16i){0};
      acc_hc[a][b] = (v16i){0};
    }

  for (int64_t kc = 0; kc < wp; kc += kKW) {
    for (int h = 0; h < 2; ++h) {
      const int r = (t >> 2) + 64 * h;
      const int q = t & 3;
      const uint4 a = *reinterpret_cast<const uint4*>(gA + r * wp + kc + q * 4);
      const uint4 b = *reinterpret_cast<const uint4*>(gB + r * wp + kc + q * 4);
      *reinterpret_cast<uint4*>(&sA[r * kLdsStride + q * 4]) = a;
      *reinterpret_cast<uint4*>(&sB[r * kLdsStride + q * 4]) = b;
    }
    __syncthreads();
    const int g = lane >> 5;
    const int rl = lane & 31;
#pragma unroll 2
    for (int s = 0; s < kKW / 2; ++s) {
      const int kw = g * (kKW / 2) + s;
      v4i fm_a[2], fw_a[2], fh_a[2], fc_a[2];
      v4i fm_b[2], fw_b[2], fh_b[2], fc_b[2];
      for (int x = 0; x < 2; ++x) {
        uint32_t c[4];
        spread_codes(sA[(wr * 64 + x * 32 + rl) * kLdsStride + kw], c);
        fm_a[x] = lookup(kLutM, c);
        fw_a[x] = lookup(kLutW, c);
        fh_a[x] = lookup(kLutH, c);
        fc_a[x] = lookup(kLutC, c);
        spread_codes(sB[(wc * 64 + x * 32 + rl) * kLdsStride + kw], c);
        fm_b[x] = lookup(kLutM, c);
        fw_b[x] = lookup(kLutW, c);
        fh_b[x] = lookup(kLutH, c);
        fc_b[x] = lookup(kLutCn, c);
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          acc_m[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fm_a[a], fm_b[b], acc_m[a][b], 0, 0, 0);
          acc_w[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fw_a[a], fw_b[b], acc_w[a][b], 0, 0, 0);
          acc_hc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fh_a[a], fh_b[b], acc_hc[a][b], 0, 0, 0);
          acc_hc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fc_a[a], fc_b[b], acc_hc[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }

  // 32x32 accumulator layout: register v of lane l holds row
  // 8*(v/4) + 4*(l/32) + v%4 and column l%32 of the block.
  const bool mirror = (I != J);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 16; ++v) {
        const int64_t i = I * kT + wr * 64 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t j = J * kT + wc * 64 + b * 32 + (lane & 31);
        const uint32_t n = (uint32_t)acc_m[a][b][v];
        const uint32_t z = (uint32_t)acc_hc[a][b][v] >> 1;
        const uint32_t one = (n - (uint32_t)acc_w[a][b][v]) >> 1;
        store_counts(o, i, j, mirror, n, z, one);
      }
}

int launch_ibs_mfma(const uint32_t* T, int64_t wp, const IbsOut& o, hipStream_t st) {
  const int64_t nt = ceil_div(o.m, kT);
  const int64_t blocks = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(k_ibs_mfma, dim3((unsigned)blocks), dim3(256), 0, st, T, wp, nt, o);
  return check_launch("ibs_mfma");
}

// ---- popcount path --------------------------------------------------------------
// Block: 256 threads over a 64x64 tile, 4x4 pairs per thread; K runs over
// 32-variant plane words in chunks of 16 staged through LDS.
constexpr int kP = kIbsPopcTile;
constexpr int kPW = kIbsPopcKWords;

__global__ __launch_bounds__(256) void k_ibs_popc(const uint32_t* __restrict__ P, int64_t rows_pad,
                                                  int64_t words_pad, int64_t nt, IbsOut o) {
  __shared__ __attribute__((aligned(16))) uint32_t sA[kPW * 3 * kP];
  __shared__ __attribute__((aligned(16))) uint32_t sB[kPW * 3 * kP];
  int64_t I, J;
  tri_tile(blockIdx.x, nt, I, J);
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
      *reinterpret_cast<uint4*>(&sA[row * kP + col]) = a;
      *reinterpret_cast<uint4*>(&sB[row * kP + col]) = b;
    }
    __syncthreads();
#pragma unroll 4
    for (int w = 0; w < kPW; ++w) {
      const uint4 ah = *reinterpret_cast<const uint4*>(&sA[(w * 3 + 0) * kP + ty * 4]);
      const uint4 al = *reinterpret_cast<const uint4*>(&sA[(w * 3 + 1) * kP + ty * 4]);
      const uint4 am = *reinterpret_cast<const uint4*>(&sA[(w * 3 + 2) * kP + ty * 4]);
      const uint4 bh = *reinterpret_cast<const uint4*>(&sB[(w * 3 + 0) * kP + tx * 4]);
      const uint4 bl = *reinterpret_cast<const uint4*>(&sB[(w * 3 + 1) * kP + tx * 4]);
      const uint4 bm = *reinterpret_cast<const uint4*>(&sB[(w * 3 + 2) * kP + tx * 4]);
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
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      store_counts(o, I * kP + ty * 4 + r, J * kP + tx * 4 + c, mirror, cn[r][c], cz[r][c],
                   co[r][c]);
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
