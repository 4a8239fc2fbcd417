// IBS distance and complete-linkage clustering (section "Identity-by-state
// matrices, complete linkage clustering": an IBS matrix followed by complete
// linkage clustering, timed in Table 2).
//
// Distance (reading; the paper names the statistic but not its formula): the
// proportion of alleles not shared identical by state over the jointly
// non-missing markers, d = (2 IBS0 + IBS1) / (2 N), +inf when N = 0 -- the
// correctly rounded quotient of two integers, so any implementation gets the
// same double.
//
// Clustering: while more than one cluster remains, merge the two clusters
// with the smallest complete-linkage distance (largest member-to-member
// distance); ties go to the smallest (a, b) pair of cluster indices, a
// cluster being indexed by its smallest sample.  Every decision compares
// doubles that are maxima of the input doubles, so the merge sequence is
// exactly determined.
//
// GPU plan: the working matrix D (m x m doubles) lives in the workspace.
// For each active cluster k the cached nearest neighbour among l > k,
// nn[k] = argmin over (D[k][l], l), is kept; the globally closest pair is the
// argmin over k of (nn_d[k], k), which is exactly the lexicographic rule.
// One block runs the m - 1 steps: pick the pair (i, j), fold row and column
// j into i with max(), retire j, then rescan only the rows whose cached
// neighbour could have changed -- row i, rows k < i whose neighbour was i or
// j, and rows i < k < j whose neighbour was j (distances only grow, so no
// other row's minimum moves).  A retired cluster's column and cache entry
// hold NaN, which never wins a minimum, so scans need no activity flags;
// each rescan is done by the whole block with several loads in flight per
// thread.
#include "pg_internal.h"

namespace pg {

__global__ __launch_bounds__(256) void k_ibs_distance(const uint32_t* __restrict__ i0,
                                                      const uint32_t* __restrict__ i1,
                                                      const uint32_t* __restrict__ nm,
                                                      int64_t count, double* __restrict__ d) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t n = nm[e];
    d[e] = n ? __ddiv_rn((double)(2 * (int64_t)i0[e] + i1[e]), (double)(2 * (int64_t)n))
             : __longlong_as_double(0x7ff0000000000000ll);
  }
}

int launch_ibs_distance(const uint32_t* i0, const uint32_t* i1, const uint32_t* nm, int64_t count,
                        double* d, hipStream_t st) {
  if (count <= 0) return PG_OK;
  const int64_t blocks = ceil_div(count, 256) < 65536 ? ceil_div(count, 256) : 65536;
  hipLaunchKernelGGL(k_ibs_distance, dim3((unsigned)blocks), dim3(256), 0, st, i0, i1, nm, count,
                     d);
  return check_launch("ibs_distance");
}

// ---- IBS similarity and the IBD report ---------------------------------------
// Similarity (the --distance ibs value; reading): s = (2 IBS2 + IBS1) / (2 N),
// the correctly rounded quotient of two integers, NaN when N = 0.
__global__ __launch_bounds__(256) void k_ibs_similarity(const uint32_t* __restrict__ i1,
                                                        const uint32_t* __restrict__ i2,
                                                        const uint32_t* __restrict__ nm,
                                                        int64_t count, double* __restrict__ s) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t n = nm[e];
    s[e] = n ? __ddiv_rn((double)(2 * (int64_t)i2[e] + i1[e]), (double)(2 * (int64_t)n))
             : __longlong_as_double(0x7ff8000000000000ll);
  }
}

int launch_ibs_similarity(const uint32_t* i1, const uint32_t* i2, const uint32_t* nm,
                          int64_t count, double* s, hipStream_t st) {
  if (count <= 0) return PG_OK;
  const int64_t blocks = ceil_div(count, 256) < 65536 ? ceil_div(count, 256) : 65536;
  hipLaunchKernelGGL(k_ibs_similarity, dim3((unsigned)blocks), dim3(256), 0, st, i1, i2, nm,
                     count, s);
  return check_launch("ibs_similarity");
}

// IBD report (reading; the paper times it but gives no formulas).  A marker
// whose observed alleles among the selected samples are x copies of A2 and y
// of A1 (n = x + y >= 4) expects, for two samples sharing no allele IBD (four
// alleles drawn without replacement from those n) or one (three drawn),
//   P(IBS0|IBD0) = 2 x(x-1) y(y-1) / n(n-1)(n-2)(n-3),
//   P(IBS1|IBD0) = 4 [x(x-1)(x-2) y + x y(y-1)(y-2)] / n(n-1)(n-2)(n-3),
//   P(IBS2|IBD0) = [x(x-1)(x-2)(x-3) + y(y-1)(y-2)(y-3) + 4 x(x-1) y(y-1)] / n(n-1)(n-2)(n-3),
//   P(IBS1|IBD1) = 2 [x(x-1) y + x y(y-1)] / n(n-1)(n-2),
//   P(IBS2|IBD1) = [x(x-1)(x-2) + y(y-1)(y-2) + x(x-1) y + x y(y-1)] / n(n-1)(n-2).
// These are averaged over the markers with n >= 4 (E00, E10, E20, E11, E21),
// and per pair the IBS0 and IBS1 moment equations give
//   Z0 = min(P0 / E00, 1),  Z1 = (P1 - Z0 E10) / E11 clamped to [0, 1 - Z0],
//   Z2 = (1 - Z0) - Z1,  PI_HAT = 0.5 Z1 + Z2,  with P0 = IBS0 / N, P1 = IBS1 / N.
// Every term is evaluated in IEEE double in the order written (explicit
// round-to-nearest operations, no contraction) and the averages are sums in
// increasing marker order, so the results are the same doubles any
// implementation of these formulas in that order gets.

// One wave per marker row of the variant-major operand D (rows_pad x wn
// words of 16 codes, padding codes missing): counts the calls and A2 alleles,
// then writes the five terms (0 when n < 4) to terms[q * rows_pad + v] and
// whether the marker counts to used[v].
__global__ __launch_bounds__(256) void k_genome_terms(const uint32_t* __restrict__ D, int64_t wn,
                                                      int64_t nv, int64_t rows_pad,
                                                      double* __restrict__ terms,
                                                      uint32_t* __restrict__ used) {
  const int lane = threadIdx.x & 63;
  const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (v >= nv) return;
  const uint32_t* row = D + v * wn;
  int64_t calls = 0, a2 = 0;
  for (int64_t w = lane; w < wn; w += 64) {
    const uint32_t x = row[w];
    const uint32_t lo = x & 0x55555555u, hi = (x >> 1) & 0x55555555u;
    calls += __popc((hi | ~lo) & 0x55555555u);          // codes 00, 10, 11
    a2 += 2 * __popc(hi & lo) + __popc(hi & ~lo);       // 11 twice, 10 once
  }
  for (int d = 32; d > 0; d >>= 1) {
    calls += __shfl_xor(calls, d, 64);
    a2 += __shfl_xor(a2, d, 64);
  }
  if (lane != 0) return;
  double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const bool ok = 2 * calls >= 4;
  if (ok) {
    const double X = (double)a2, Y = (double)(2 * calls - a2), n = (double)(2 * calls);
    const double d4 = __dmul_rn(__dmul_rn(__dmul_rn(n, __dsub_rn(n, 1.0)), __dsub_rn(n, 2.0)),
                                __dsub_rn(n, 3.0));
    const double d3 = __dmul_rn(__dmul_rn(n, __dsub_rn(n, 1.0)), __dsub_rn(n, 2.0));
    const double x2 = __dmul_rn(X, __dsub_rn(X, 1.0)), y2 = __dmul_rn(Y, __dsub_rn(Y, 1.0));
    const double x3 = __dmul_rn(x2, __dsub_rn(X, 2.0)), y3 = __dmul_rn(y2, __dsub_rn(Y, 2.0));
    t[0] = __ddiv_rn(__dmul_rn(__dmul_rn(2.0, x2), y2), d4);
    t[1] = __ddiv_rn(__dmul_rn(4.0, __dadd_rn(__dmul_rn(x3, Y), __dmul_rn(X, y3))), d4);
    t[2] = __ddiv_rn(__dadd_rn(__dadd_rn(__dmul_rn(x3, __dsub_rn(X, 3.0)),
                                         __dmul_rn(y3, __dsub_rn(Y, 3.0))),
                               __dmul_rn(__dmul_rn(4.0, x2), y2)),
                     d4);
    t[3] = __ddiv_rn(__dmul_rn(2.0, __dadd_rn(__dmul_rn(x2, Y), __dmul_rn(X, y2))), d3);
    t[4] = __ddiv_rn(__dadd_rn(__dadd_rn(__dadd_rn(x3, y3), __dmul_rn(x2, Y)), __dmul_rn(X, y2)),
                     d3);
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) terms[q * rows_pad + v] = t[q];
  used[v] = ok ? 1u : 0u;
}

// The five sums and the count K of markers that count, in two levels: each
// run of kSumRun consecutive markers is summed in increasing marker order
// from 0, then the runs' sums are added in increasing run order from 0.
// k_genome_run_sums: one block per run; all threads stage the run's five
// term columns in LDS (coalesced loads), then threads 0..4 each add their
// column in order; a marker that does not count, and the padding past the
// last marker, add +0.0, which leaves a non-negative sum unchanged.  It
// writes part[q * n_runs + r] (q < 5) and the run's count at q = 5.
constexpr int kSumRun = 1024;
constexpr int kSumPer = 5 * kSumRun / 256;      // staged values per thread
__global__ __launch_bounds__(256) void k_genome_run_sums(const double* __restrict__ terms,
                                                         const uint32_t* __restrict__ used,
                                                         int64_t nv, int64_t rows_pad,
                                                         int64_t n_runs,
                                                         double* __restrict__ part) {
  __shared__ double buf[5][kSumRun + 1];
  __shared__ unsigned int kcount;
  const int t = threadIdx.x;
  const int64_t r = blockIdx.x, c0 = r * kSumRun;
  const int64_t len = nv - c0 < kSumRun ? nv - c0 : kSumRun;
  if (t == 0) kcount = 0;
  double v[kSumPer];
#pragma unroll
  for (int u = 0; u < kSumPer; ++u) {
    const int i = t + 256 * u, q = i / kSumRun, j = i % kSumRun;
    v[u] = j < len ? terms[q * rows_pad + c0 + j] : 0.0;
  }
  unsigned int K = 0;
  for (int64_t j = t; j < len; j += 256) K += used[c0 + j];
#pragma unroll
  for (int u = 0; u < kSumPer; ++u) {
    const int i = t + 256 * u;
    buf[i / kSumRun][i % kSumRun] = v[u];
  }
  __syncthreads();
  if (K) atomicAdd(&kcount, K);
  if (t < 5) {
    const double* col = buf[t];
    double S = 0.0;
    for (int j = 0; j < len; j += 32) {
      double b[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) b[u] = col[j + u];
#pragma unroll
      for (int u = 0; u < 32; ++u) S = __dadd_rn(S, b[u]);
    }
    part[t * n_runs + r] = S;
  }
  __syncthreads();
  if (t == 0) part[5 * n_runs + r] = (double)kcount;
}

// out = {S00, S10, S20, S11, S21, K}: threads 0..4 add the runs' sums of
// their column in run order; thread 5 adds the counts (integers, exact).
__global__ __launch_bounds__(64) void k_genome_total(const double* __restrict__ part,
                                                     int64_t n_runs, double* __restrict__ out) {
  const int t = threadIdx.x;
  if (t > 5) return;
  double S = 0.0;
  for (int64_t r = 0; r < n_runs; ++r) S = __dadd_rn(S, part[t * n_runs + r]);
  out[t] = S;
}

__global__ __launch_bounds__(256) void k_genome_pairs(const double* __restrict__ sums,
                                                      const uint32_t* __restrict__ i0,
                                                      const uint32_t* __restrict__ i1,
                                                      const uint32_t* __restrict__ nm,
                                                      int64_t count, double* __restrict__ z0,
                                                      double* __restrict__ z1,
                                                      double* __restrict__ z2,
                                                      double* __restrict__ pi) {
  const double K = sums[5];
  const double E00 = __ddiv_rn(sums[0], K), E10 = __ddiv_rn(sums[1], K);
  const double E11 = __ddiv_rn(sums[3], K);
  const bool ok = K > 0.0 && E00 != 0.0 && E11 != 0.0;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (!ok || nm[e] == 0) {
      z0[e] = z1[e] = z2[e] = pi[e] = nan;
      continue;
    }
    const double N = (double)nm[e];
    const double p0 = __ddiv_rn((double)i0[e], N), p1 = __ddiv_rn((double)i1[e], N);
    double a = __ddiv_rn(p0, E00);
    if (a > 1.0) a = 1.0;
    double b = __ddiv_rn(__dsub_rn(p1, __dmul_rn(a, E10)), E11);
    if (b < 0.0) b = 0.0;
    if (b > __dsub_rn(1.0, a)) b = __dsub_rn(1.0, a);
    const double c = __dsub_rn(__dsub_rn(1.0, a), b);
    z0[e] = a;
    z1[e] = b;
    z2[e] = c;
    pi[e] = __dadd_rn(__dmul_rn(0.5, b), c);
  }
}

int launch_genome(const uint32_t* D, int64_t wn, int64_t nv, int64_t rows_pad, double* terms,
                  uint32_t* used, double* sums, const uint32_t* i0, const uint32_t* i1,
                  const uint32_t* nm, int64_t count, double* z0, double* z1, double* z2,
                  double* pi, hipStream_t st) {
  hipLaunchKernelGGL(k_genome_terms, dim3((unsigned)ceil_div(nv, 4)), dim3(256), 0, st, D, wn, nv,
                     rows_pad, terms, used);
  int rc = check_launch("genome_terms");
  if (rc != PG_OK) return rc;
  const int64_t n_runs = genome_runs(nv);
  double* part = sums + 8;
  hipLaunchKernelGGL(k_genome_run_sums, dim3((unsigned)n_runs), dim3(256), 0, st, terms, used, nv,
                     rows_pad, n_runs, part);
  rc = check_launch("genome_run_sums");
  if (rc != PG_OK) return rc;
  hipLaunchKernelGGL(k_genome_total, dim3(1), dim3(64), 0, st, part, n_runs, sums);
  rc = check_launch("genome_total");
  mark_stage(1, st);
  if (rc != PG_OK || count <= 0) return rc;
  const int64_t blocks = ceil_div(count, 256) < 65536 ? ceil_div(count, 256) : 65536;
  hipLaunchKernelGGL(k_genome_pairs, dim3((unsigned)blocks), dim3(256), 0, st, sums, i0, i1, nm,
                     count, z0, z1, z2, pi);
  return check_launch("genome_pairs");
}

// (value, index) minimum with the smaller index on equal values.
__device__ __forceinline__ void take_min(double& bv, int& bi, double v, int i) {
  if (v < bv || (v == bv && (unsigned)i < (unsigned)bi)) {
    bv = v;
    bi = i;
  }
}

__device__ __forceinline__ void wave_min(double& v, int& i) {
  for (int d = 32; d > 0; d >>= 1) {
    const double ov = __shfl_xor(v, d, 64);
    const int oi = __shfl_xor(i, d, 64);
    take_min(v, i, ov, oi);
  }
}

constexpr uint64_t kNaN = 0x7ff8000000000000ull;

__global__ __launch_bounds__(256) void k_nn_init(const double* __restrict__ D, int64_t m,
                                                 double* nn_d, int* nn_j) {
  const int lane = threadIdx.x & 63;
  for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; k < m;
       k += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    double bv = __longlong_as_double(0x7ff0000000000000ll);
    int bi = -1;
    const double* row = D + k * m;
    for (int64_t l = k + 1 + lane; l < m; l += 64) take_min(bv, bi, row[l], (int)l);
    wave_min(bv, bi);
    if (lane == 0) {
      nn_d[k] = bi >= 0 ? bv : __longlong_as_double(kNaN);
      nn_j[k] = bi;
    }
  }
}

constexpr int kCT = 1024;
constexpr int kCW = kCT / 64;   // waves
constexpr int kCU = 4;          // loads in flight per thread in the argmin and the fold
constexpr int kCR = 8;          // loads in flight per thread in row rescans

__global__ __launch_bounds__(kCT) void k_cluster(double* __restrict__ D, int64_t m,
                                                 double* __restrict__ nn_d, int* __restrict__ nn_j,
                                                 pg_merge* __restrict__ merges) {
  __shared__ double s_v[kCW];
  __shared__ int s_i[kCW];
  __shared__ int s_rows[kCT];
  __shared__ int s_nrows;
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  const double nan = __longlong_as_double(kNaN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t t = 0; t + 1 < m; ++t) {
    // (a) the globally closest pair: argmin over k of (nn_d[k], k); retired
    // rows and rows without a neighbour hold NaN
    double bv = inf;
    int bi = -1;
    for (int64_t k0 = tid; k0 < m; k0 += kCT * kCU) {
      double v[kCU];
#pragma unroll
      for (int u = 0; u < kCU; ++u) v[u] = k0 + u * kCT < m ? nn_d[k0 + u * kCT] : nan;
#pragma unroll
      for (int u = 0; u < kCU; ++u) take_min(bv, bi, v[u], (int)(k0 + u * kCT));
    }
    wave_min(bv, bi);
    if (lane == 0) {
      s_v[wave] = bv;
      s_i[wave] = bi;
    }
    __syncthreads();
    double hv = s_v[0];
    int i = s_i[0];
    for (int w = 1; w < kCW; ++w) take_min(hv, i, s_v[w], s_i[w]);
    if (i < 0) break;   // unreachable: two active clusters always pair
    const int j = nn_j[i];
    if (tid == 0) {
      merges[t].a = i;
      merges[t].b = j;
      merges[t].height = hv;
      s_nrows = 0;
    }
    // (b) fold j into i: D[i][k] = D[k][i] = max(D[i][k], D[j][k]) for the
    // active k (a retired k has NaN in row i); retire j: its column and its
    // cache entry become NaN
    const double* ri = D + (int64_t)i * m;
    const double* rj = D + (int64_t)j * m;
    for (int64_t k0 = tid; k0 < m; k0 += kCT * kCU) {
      double a[kCU], b[kCU];
#pragma unroll
      for (int u = 0; u < kCU; ++u) {
        const int64_t k = k0 + u * kCT;
        a[u] = k < m ? ri[k] : nan;
        b[u] = k < m ? rj[k] : nan;
      }
#pragma unroll
      for (int u = 0; u < kCU; ++u) {
        const int64_t k = k0 + u * kCT;
        if (k >= m || k == j || a[u] != a[u]) continue;
        if (k != i) {
          const double v = a[u] > b[u] ? a[u] : b[u];
          D[(int64_t)i * m + k] = v;
          D[k * m + i] = v;
        }
        D[k * m + j] = nan;
      }
    }
    __syncthreads();
    if (tid == 0) nn_d[j] = nan;
    // (c) active rows (cache entry not NaN) whose neighbour may have moved
    for (int64_t k = tid; k < j; k += kCT) {
      const double dk = nn_d[k];
      if (dk != dk) continue;
      const int nk = nn_j[k];
      if (k == i || (k < i && (nk == i || nk == j)) || (k > i && nk == j)) {
        const int slot = atomicAdd(&s_nrows, 1);
        if (slot < kCT) s_rows[slot] = (int)k;
      }
    }
    __syncthreads();
    const int nrows = s_nrows;
    // (d) rescan them: groups of g waves per row, kCW / g rows at a time
    // (more rows than the list holds: walk every row below j, g = 1)
    const bool listed = nrows <= kCT;
    const int64_t nscan = listed ? nrows : j;
    int g = kCW;
    while (g > 1 && (int64_t)(kCW / g) < nscan) g >>= 1;
    const int groups = kCW / g, grp = wave / g, gt = tid - grp * g * 64;
    for (int64_t r0 = 0; r0 < nscan; r0 += groups) {
      const int64_t rr = r0 + grp;
      int k = -1;
      if (rr < nscan) {
        if (listed) {
          k = s_rows[rr];
        } else {
          const int kk = (int)rr;
          const double dk = nn_d[kk];
          const int nk = nn_j[kk];
          if (dk == dk && (kk == i || (kk < i && (nk == i || nk == j)) || (kk > i && nk == j)))
            k = kk;
        }
      }
      double v = inf;
      int l = -1;
      if (k >= 0) {
        const double* row = D + (int64_t)k * m;
        for (int64_t c0 = k + 1 + gt; c0 < m; c0 += (int64_t)g * 64 * kCR) {
          double x[kCR];
#pragma unroll
          for (int u = 0; u < kCR; ++u) {
            const int64_t c = c0 + (int64_t)u * g * 64;
            x[u] = c < m ? row[c] : nan;
          }
#pragma unroll
          for (int u = 0; u < kCR; ++u) take_min(v, l, x[u], (int)(c0 + (int64_t)u * g * 64));
        }
      }
      wave_min(v, l);
      __syncthreads();   // s_v / s_i free (their last readers are past here)
      if (lane == 0) {
        s_v[wave] = v;
        s_i[wave] = l;
      }
      __syncthreads();
      if (k >= 0 && gt == 0) {
        double rv = s_v[grp * g];
        int rl = s_i[grp * g];
        for (int w = 1; w < g; ++w) take_min(rv, rl, s_v[grp * g + w], s_i[grp * g + w]);
        nn_d[k] = rl >= 0 ? rv : nan;
        nn_j[k] = rl;
      }
    }
    __syncthreads();
  }
}

// ---- the merge loop as two launches per merge (large cohorts) ---------------
// The same steps as k_cluster, each spread over the chip.  k_cl_fold: every
// block finds the pair itself (the argmin over the cached neighbours, the
// same in every block; a block that already sees j retired by another block
// still finds i, since i != j), block 0 records the merge, and each thread
// folds sample k = its global index: j into i, j retired, and k appended to
// the list of rows to rescan when its neighbour may have moved.  k_cl_rescan
// (a block per listed row) rescans them.  The list's length for merge t is
// cnt[t % 2]; merge t clears cnt[(t + 1) % 2], whose last reader was merge
// t - 1's rescan, so the host only enqueues.
constexpr int kClT = 1024;
constexpr int kClScanBlocks = 64;

__global__ __launch_bounds__(kClT) void k_cl_fold(double* __restrict__ D, int64_t m,
                                                 double* __restrict__ nn_d,
                                                 const int* __restrict__ nn_j, int64_t t,
                                                 pg_merge* __restrict__ merges,
                                                 int* __restrict__ cnt, int* __restrict__ rows) {
  __shared__ double s_v[kClT / 64];
  __shared__ int s_i[kClT / 64];
  __shared__ int s_pair[2];
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  const double nan = __longlong_as_double(kNaN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double bv = inf;
  int bi = -1;
  for (int64_t k0 = tid; k0 < m; k0 += kClT * kCU) {
    double v[kCU];
#pragma unroll
    for (int u = 0; u < kCU; ++u) v[u] = k0 + u * kClT < m ? nn_d[k0 + u * kClT] : nan;
#pragma unroll
    for (int u = 0; u < kCU; ++u) take_min(bv, bi, v[u], (int)(k0 + u * kClT));
  }
  wave_min(bv, bi);
  if (lane == 0) {
    s_v[wave] = bv;
    s_i[wave] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    double hv = s_v[0];
    int pi = s_i[0];
    for (int w = 1; w < kClT / 64; ++w) take_min(hv, pi, s_v[w], s_i[w]);
    const int pj = pi >= 0 ? nn_j[pi] : -1;
    s_pair[0] = pi;
    s_pair[1] = pj;
    if (blockIdx.x == 0) {
      if (pi >= 0) {   // always: two active clusters always pair
        merges[t].a = pi;
        merges[t].b = pj;
        merges[t].height = hv;
      }
      cnt[(t + 1) & 1] = 0;
    }
  }
  __syncthreads();
  const int i = s_pair[0], j = s_pair[1];
  const int64_t k = (int64_t)blockIdx.x * kClT + tid;
  if (i < 0 || k >= m) return;
  // fold: D[i][k] = D[k][i] = max(D[i][k], D[j][k]) for the active k (a
  // retired k has NaN in row i); retire j: its column becomes NaN
  const double a = D[(int64_t)i * m + k];
  if (k != j && a == a) {
    if (k != i) {
      const double b = D[(int64_t)j * m + k];
      const double v = a > b ? a : b;
      D[(int64_t)i * m + k] = v;
      D[k * m + i] = v;
    }
    D[k * m + j] = nan;
  }
  if (k == j) nn_d[j] = nan;
  // active rows below j whose cached neighbour may have moved (their cache
  // entries are not touched by this kernel, except j's, which is not listed)
  if (k < j) {
    const double dk = nn_d[k];
    const int nk = nn_j[k];
    if (dk == dk && (k == i || (k < i && (nk == i || nk == j)) || (k > i && nk == j)))
      rows[atomicAdd(&cnt[t & 1], 1)] = (int)k;
  }
}

__global__ __launch_bounds__(kClT) void k_cl_rescan(const double* __restrict__ D, int64_t m,
                                                    double* __restrict__ nn_d,
                                                    int* __restrict__ nn_j, int64_t t,
                                                    const int* __restrict__ cnt,
                                                    const int* __restrict__ rows) {
  __shared__ double s_v[kClT / 64];
  __shared__ int s_i[kClT / 64];
  const int nrows = cnt[t & 1];
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  const double nan = __longlong_as_double(kNaN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int r = blockIdx.x; r < nrows; r += gridDim.x) {   // block-uniform
    const int64_t k = rows[r];
    const double* row = D + k * m;
    double v = inf;
    int l = -1;
    for (int64_t c0 = k + 1 + tid; c0 < m; c0 += (int64_t)kClT * kCR) {
      double x[kCR];
#pragma unroll
      for (int u = 0; u < kCR; ++u) {
        const int64_t c = c0 + (int64_t)u * kClT;
        x[u] = c < m ? row[c] : nan;
      }
#pragma unroll
      for (int u = 0; u < kCR; ++u) take_min(v, l, x[u], (int)(c0 + (int64_t)u * kClT));
    }
    wave_min(v, l);
    __syncthreads();   // s_v / s_i free (the previous row's reader is done)
    if (lane == 0) {
      s_v[wave] = v;
      s_i[wave] = l;
    }
    __syncthreads();
    if (tid == 0) {
      double rv = s_v[0];
      int rl = s_i[0];
      for (int w = 1; w < kClT / 64; ++w) take_min(rv, rl, s_v[w], s_i[w]);
      nn_d[k] = rl >= 0 ? rv : nan;
      nn_j[k] = rl;
    }
  }
}

int launch_ibs_cluster(const uint32_t* i0, const uint32_t* i1, const uint32_t* nm, int64_t m,
                       double* D, double* nn_d, int* nn_j, int* ctl, int* rows,
                       pg_merge* merges, hipStream_t st) {
  int rc = launch_ibs_distance(i0, i1, nm, m * m, D, st);
  if (rc != PG_OK) return rc;
  const int64_t blocks = ceil_div(m, 4) < 65536 ? ceil_div(m, 4) : 65536;
  hipLaunchKernelGGL(k_nn_init, dim3((unsigned)blocks), dim3(256), 0, st, D, m, nn_d, nn_j);
  rc = check_launch("cluster_init");
  mark_stage(1, st);
  if (rc != PG_OK || m < 2) return rc;
  if (m < kClusterSplitMin) {
    hipLaunchKernelGGL(k_cluster, dim3(1), dim3(kCT), 0, st, D, m, nn_d, nn_j, merges);
    rc = check_launch("cluster");
  } else {
    const unsigned fold_blocks = (unsigned)ceil_div(m, kClT);
    rc = fill_u32(reinterpret_cast<uint32_t*>(ctl), 2, 0u, st);   // the two list lengths
    for (int64_t t = 0; t + 1 < m && rc == PG_OK; ++t) {
      hipLaunchKernelGGL(k_cl_fold, dim3(fold_blocks), dim3(kClT), 0, st, D, m, nn_d, nn_j, t,
                         merges, ctl, rows);
      hipLaunchKernelGGL(k_cl_rescan, dim3(kClScanBlocks), dim3(kClT), 0, st, D, m, nn_d, nn_j, t,
                         ctl, rows);
      rc = check_launch("cluster_step");
    }
  }
  mark_stage(2, st);
  return rc;
}

}  // namespace pg
