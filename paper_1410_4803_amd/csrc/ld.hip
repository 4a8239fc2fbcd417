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
constexpr int kL = kLdTile;
constexpr int kLW = kLdKWords;
constexpr int kLStride = kLW + 4;

__global__ __launch_bounds__(256) void k_ld_mfma(const uint32_t* __restrict__ D, int64_t wn,
                                                 int64_t nv, int64_t n_row_tiles, int64_t n_band,
                                                 int32_t window, double r2_min, LdScratch sc) {
  const int64_t I = (int64_t)blockIdx.x / n_band;
  const int64_t J = I + (int64_t)blockIdx.x % n_band;
  if (J >= n_row_tiles) return;
  __shared__ __attribute__((aligned(16))) uint32_t sA[kL * kLStride];
  __shared__ __attribute__((aligned(16))) uint32_t sB[kL * kLStride];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const uint32_t* gA = D + I * kL * wn;
  const uint32_t* gB = D + J * kL * wn;

  v16i s_n = (v16i){0}, s_x = (v16i){0}, s_y = (v16i){0};
  v16i s_xx = (v16i){0}, s_yy = (v16i){0}, s_xy = (v16i){0};

  for (int64_t kc = 0; kc < wn; kc += kLW) {
    {
      const int r = t >> 2;   // 64 rows x 4 uint4
      const int q = t & 3;
      const uint4 a = *reinterpret_cast<const uint4*>(gA + r * wn + kc + q * 4);
      const uint4 b = *reinterpret_cast<const uint4*>(gB + r * wn + kc + q * 4);
      *reinterpret_cast<uint4*>(&sA[r * kLStride + q * 4]) = a;
      *reinterpret_cast<uint4*>(&sB[r * kLStride + q * 4]) = b;
    }
    __syncthreads();
    const int g = lane >> 5;
    const int rl = lane & 31;
#pragma unroll 2
    for (int s = 0; s < kLW / 2; ++s) {
      const int kw = g * (kLW / 2) + s;
      uint32_t c[4];
      ld_spread(sA[(wr * 32 + rl) * kLStride + kw], c);
      const v4i am = ld_lookup(kLdLutM, c), ax = ld_lookup(kLdLutX, c), ah = ld_lookup(kLdLutH, c);
      ld_spread(sB[(wc * 32 + rl) * kLStride + kw], c);
      const v4i bm = ld_lookup(kLdLutM, c), bx = ld_lookup(kLdLutX, c), bh = ld_lookup(kLdLutH, c);
      s_n = __builtin_amdgcn_mfma_i32_32x32x32_i8(am, bm, s_n, 0, 0, 0);
      s_x = __builtin_amdgcn_mfma_i32_32x32x32_i8(ax, bm, s_x, 0, 0, 0);
      s_y = __builtin_amdgcn_mfma_i32_32x32x32_i8(am, bx, s_y, 0, 0, 0);
      s_xx = __builtin_amdgcn_mfma_i32_32x32x32_i8(ah, bm, s_xx, 0, 0, 0);
      s_yy = __builtin_amdgcn_mfma_i32_32x32x32_i8(am, bh, s_yy, 0, 0, 0);
      s_xy = __builtin_amdgcn_mfma_i32_32x32x32_i8(ax, bx, s_xy, 0, 0, 0);
    }
    __syncthreads();
  }

  for (int v = 0; v < 16; ++v) {
    const int64_t a = I * kL + wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int64_t b = J * kL + wc * 32 + (lane & 31);
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
__global__ __launch_bounds__(1024) void k_ld_scan(const uint32_t* __restrict__ cnt, int64_t nv,
                                                  int64_t* __restrict__ off, int64_t* n_out) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = ceil_div(nv, 1024);
  const int64_t lo = t * chunk;
  const int64_t hi = lo + chunk < nv ? lo + chunk : nv;
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t add = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = lo; i < hi; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) {
    off[nv] = part[1023];
    *n_out = part[1023];
  }
}

// ---- emit: one wave per row --------------------------------------------------------
__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_ld_emit(const uint32_t* __restrict__ D, int64_t wn,
                                                 int64_t nv, int64_t v0, LdScratch sc,
                                                 pg_ld_pair* __restrict__ out, int64_t capacity) {
  const int64_t a = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (a >= nv) return;
  int64_t pos = sc.rowoff[a];
  if (pos >= capacity || sc.rowcnt[a] == 0) return;
  const uint32_t* ra = D + a * wn;
  for (int64_t q = 0; q < sc.bm_words; ++q) {
    uint32_t bits = sc.bitmap[a * sc.bm_words + q];
    while (bits) {
      const int tb = __builtin_ctz(bits);
      bits &= bits - 1;
      if (pos >= capacity) return;
      const int64_t b = a + 1 + q * 32 + tb;
      const uint32_t* rb = D + b * wn;
      int cn = 0, csx = 0, csy = 0, csxx = 0, csyy = 0, csxy = 0;
      for (int64_t w = lane; w < wn; w += 64) {
        const uint32_t xa = ra[w], xb = rb[w];
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
      cn = wave_sum(cn); csx = wave_sum(csx); csy = wave_sum(csy);
      csxx = wave_sum(csxx); csyy = wave_sum(csyy); csxy = wave_sum(csxy);
      if (lane == 0) {
        pg_ld_pair r;
        r.a = (int32_t)(v0 + a);
        r.b = (int32_t)(v0 + b);
        r.n = cn; r.sx = csx; r.sy = csy; r.sxx = csxx; r.syy = csyy; r.sxy = csxy;
        r.r2 = ld_r2(cn, csx, csy, csxx, csyy, csxy);
        out[pos] = r;
      }
      ++pos;
    }
  }
}

int launch_ld_finish(const uint32_t* D, int64_t wn, int64_t nv, int64_t v0, int32_t window,
                     const LdScratch& sc, pg_ld_pair* out, int64_t capacity, int64_t* n_out,
                     hipStream_t st) {
  (void)window;
  hipLaunchKernelGGL(k_ld_scan, dim3(1), dim3(1024), 0, st, sc.rowcnt, nv, sc.rowoff, n_out);
  int rc = check_launch("ld_scan");
  mark_stage(3, st);
  if (rc == PG_OK && capacity > 0) {
    hipLaunchKernelGGL(k_ld_emit, dim3((unsigned)ceil_div(nv, 4)), dim3(256), 0, st, D, wn, nv,
                       v0, sc, out, capacity);
    rc = check_launch("ld_emit");
  }
  mark_stage(4, st);
  return rc;
}

}  // namespace pg
