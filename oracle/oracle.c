/*
 * CPU oracle for the pairwise genotype statistics of Chang et al.,
 * "Second-generation PLINK: rising to the challenge of larger and richer
 * datasets" (GigaScience 2015; arXiv 1410.4803).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the library never does, and this file
 * shares no code, header or table with it.
 *
 * Everything works on unpacked genotype codes (one int8 per call), never on
 * packed words or bit tricks:
 *   code 0 = homozygous A1, 1 = missing, 2 = heterozygous, 3 = homozygous A2
 * (PLINK 1 binary .bed code table; the paper states only that calls are packed
 * 2-bit elements, section "Bitwise parallelism").
 *
 * OpenMP parallelises the outer loop over pairs only; each pair's sum is the
 * textbook loop in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MISSING 1

/*
 * Unpack a .bed payload.  Row v of `bed` starts at v*bytes_per_variant; the
 * call of sample k is (byte[k/4] >> 2*(k%4)) & 3.  Bits past sample n-1 are
 * ignored.  If `mask` is non-NULL (V rows of ceil(n/64) uint64, bit k%64 of
 * word k/64), a set bit marks the call missing as well.
 * Output: sample_major ? codes[k*V + v] : codes[v*n + k].
 */
void oracle_unpack(const uint8_t* bed, int64_t n, int64_t V, int64_t bytes_per_variant,
                   const uint64_t* mask, int sample_major, int8_t* codes) {
  const int64_t wpv = (n + 63) / 64;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < V; ++v) {
    const uint8_t* row = bed + v * bytes_per_variant;
    for (int64_t k = 0; k < n; ++k) {
      int code = (row[k / 4] >> (2 * (k % 4))) & 3;
      if (mask && ((mask[v * wpv + k / 64] >> (k % 64)) & 1ULL)) code = MISSING;
      if (sample_major)
        codes[k * V + v] = (int8_t)code;
      else
        codes[v * n + k] = (int8_t)code;
    }
  }
}

/* Number of A2 alleles carried by a non-missing call. */
static int dosage(int code) {
  if (code == 0) return 0; /* homozygous A1 */
  if (code == 2) return 1; /* heterozygous */
  return 2;                /* code 3, homozygous A2 */
}

/*
 * Identity-by-state counts of one sample pair (section "Bitwise parallelism",
 * the per-marker loop PLINK 1.07 used): markers where either call is missing
 * are skipped; at the others the two samples share 2, 1 or 0 alleles
 * identical by state.  The number of shared alleles is 2 - |dosage_i -
 * dosage_j|.  out = {IBS0, IBS1, IBS2, jointly non-missing}.
 * a and b point at the two samples' V codes (sample-major rows).
 */
static void ibs_pair(const int8_t* a, const int8_t* b, int64_t V, uint32_t out[4]) {
  uint32_t ibs[3] = {0, 0, 0}, nonmiss = 0;
  for (int64_t v = 0; v < V; ++v) {
    if (a[v] == MISSING || b[v] == MISSING) continue;
    nonmiss += 1;
    const int d = abs(dosage(a[v]) - dosage(b[v]));
    ibs[2 - d] += 1;
  }
  out[0] = ibs[0];
  out[1] = ibs[1];
  out[2] = ibs[2];
  out[3] = nonmiss;
}

/*
 * IBS counts for a list of pairs.  codes_sm: sample-major codes (n rows of V).
 * out: npairs x 4 (IBS0, IBS1, IBS2, N).
 */
void oracle_ibs_pairs(const int8_t* codes_sm, int64_t n, int64_t V, const int64_t* pi,
                      const int64_t* pj, int64_t npairs, uint32_t* out) {
  (void)n;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < npairs; ++p)
    ibs_pair(codes_sm + pi[p] * V, codes_sm + pj[p] * V, V, out + 4 * p);
}

/*
 * The whole IBS matrix.  full != 0: n x n row-major, diagonal included.
 * full == 0: strict upper triangle, row-major, entry (i,j), i<j, at
 * i*n - i*(i+1)/2 + (j-i-1).  Four separate arrays.
 */
void oracle_ibs_matrix(const int8_t* codes_sm, int64_t n, int64_t V, int full, uint32_t* ibs0,
                       uint32_t* ibs1, uint32_t* ibs2, uint32_t* nonmiss) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = full ? 0 : i + 1; j < n; ++j) {
      uint32_t c[4];
      ibs_pair(codes_sm + i * V, codes_sm + j * V, V, c);
      const int64_t idx = full ? i * n + j : i * n - i * (i + 1) / 2 + (j - i - 1);
      ibs0[idx] = c[0];
      ibs1[idx] = c[1];
      ibs2[idx] = c[2];
      nonmiss[idx] = c[3];
    }
  }
}

/* x value of a non-missing call (section "Bit population count"): -1 for one
 * homozygote, 0 for the heterozygote, +1 for the other homozygote.  The paper
 * names the homozygotes minor/major; with fixed A1/A2 labels this uses
 * -1 = homozygous A1 and +1 = homozygous A2 (r^2 does not depend on it). */
static int xval(int code) {
  if (code == 0) return -1;
  if (code == 2) return 0;
  return 1;
}

/*
 * The six sums behind r for one variant pair (section "Bit population
 * count"): over S_xy, the samples where neither call is missing,
 * n = |S_xy|, Sx = sum x, Sy = sum y, Sxx = sum x^2, Syy = sum y^2,
 * Sxy = sum x*y.  xa, xb: the two variants' n codes (variant-major rows).
 */
static void ld_sums(const int8_t* xa, const int8_t* xb, int64_t n, int64_t s[6]) {
  int64_t cnt = 0, sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
  for (int64_t k = 0; k < n; ++k) {
    if (xa[k] == MISSING || xb[k] == MISSING) continue;
    const int64_t x = xval(xa[k]), y = xval(xb[k]);
    cnt += 1;
    sx += x;
    sy += y;
    sxx += x * x;
    syy += y * y;
    sxy += x * y;
  }
  s[0] = cnt; s[1] = sx; s[2] = sy; s[3] = sxx; s[4] = syy; s[5] = sxy;
}

/*
 * r^2 from the six sums, in double precision, following the paper's
 * expression for r with missing data: with means over S_xy,
 *   r = (Sxy/|S_xy| - xbar*ybar) / sqrt((x2bar - xbar^2)(y2bar - ybar^2)),
 * then r^2 = r*r.  Undefined (NaN) when |S_xy| = 0 or a variance is 0.
 */
double oracle_r2(const int64_t s[6]) {
  if (s[0] == 0) return NAN;
  const double cnt = (double)s[0];
  const double xbar = (double)s[1] / cnt, ybar = (double)s[2] / cnt;
  const double x2bar = (double)s[3] / cnt, y2bar = (double)s[4] / cnt;
  const double varx = x2bar - xbar * xbar, vary = y2bar - ybar * ybar;
  if (varx == 0.0 || vary == 0.0) return NAN;
  const double r = ((double)s[5] / cnt - xbar * ybar) / sqrt(varx * vary);
  return r * r;
}

/* Sums and r^2 for a list of variant pairs.  codes_vm: variant-major codes
 * (V rows of n).  sums: npairs x 6; r2: npairs. */
void oracle_ld_pairs(const int8_t* codes_vm, int64_t n, int64_t V, const int64_t* pa,
                     const int64_t* pb, int64_t npairs, int64_t* sums, double* r2) {
  (void)V;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t p = 0; p < npairs; ++p) {
    ld_sums(codes_vm + pa[p] * n, codes_vm + pb[p] * n, n, sums + 6 * p);
    r2[p] = oracle_r2(sums + 6 * p);
  }
}

/* One emitted LD record: 64 bytes. */
typedef struct {
  int32_t a, b;
  int64_t n, sx, sy, sxx, syy, sxy;
  double r2;
} oracle_ld_record;

/*
 * All variant pairs a < b <= a + window with first index a in [a_begin, a_end)
 * and b < V, in (a, b) order; a pair is kept when its r^2 >= r2_min (an
 * undefined r^2 is never kept).  Writes at most `capacity` records and returns
 * the number of kept pairs.
 */
int64_t oracle_ld_window(const int8_t* codes_vm, int64_t n, int64_t V, int64_t a_begin,
                         int64_t a_end, int64_t window, double r2_min, oracle_ld_record* out,
                         int64_t capacity) {
  const int64_t rows = a_end - a_begin;
  if (rows <= 0) return 0;
  int64_t* per_row = (int64_t*)calloc((size_t)rows + 1, sizeof(int64_t));
  if (!per_row) return -1;
  /* pass 1: how many pairs each row keeps */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t a = a_begin + r;
    int64_t kept = 0;
    for (int64_t b = a + 1; b <= a + window && b < V; ++b) {
      int64_t s[6];
      ld_sums(codes_vm + a * n, codes_vm + b * n, n, s);
      const double r2 = oracle_r2(s);
      if (r2 >= r2_min) ++kept;
    }
    per_row[r + 1] = kept;
  }
  for (int64_t r = 0; r < rows; ++r) per_row[r + 1] += per_row[r];
  const int64_t total = per_row[rows];
  /* pass 2: write the records in order */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t a = a_begin + r;
    int64_t pos = per_row[r];
    if (pos >= capacity) continue;
    for (int64_t b = a + 1; b <= a + window && b < V && pos < capacity; ++b) {
      int64_t s[6];
      ld_sums(codes_vm + a * n, codes_vm + b * n, n, s);
      const double r2 = oracle_r2(s);
      if (!(r2 >= r2_min)) continue;
      oracle_ld_record* o = out + pos++;
      o->a = (int32_t)a;
      o->b = (int32_t)b;
      o->n = s[0]; o->sx = s[1]; o->sy = s[2]; o->sxx = s[3]; o->syy = s[4]; o->sxy = s[5];
      o->r2 = r2;
    }
  }
  free(per_row);
  return total;
}

int oracle_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * r^2 of the library's emission test, used where a floating-point value
 * decides an integer result (LD pruning): from the exact integer
 *   cov = n*Sxy - Sx*Sy,  vx = n*Sxx - Sx^2,  vy = n*Syy - Sy^2
 * (the paper's r with missing data, multiplied through by n^2), evaluated as
 * (cov*cov) / (vx*vy) with IEEE double operations, clamped to 1; NaN when
 * n, vx or vy is 0.  Both sides take the pruning decision on this double.
 */
double oracle_r2_counts(const int64_t s[6]) {
  const int64_t n = s[0];
  const int64_t cov = n * s[5] - s[1] * s[2];
  const int64_t vx = n * s[3] - s[1] * s[1];
  const int64_t vy = n * s[4] - s[2] * s[2];
  if (n == 0 || vx == 0 || vy == 0) return NAN;
  const double num = (double)cov * (double)cov;
  const double den = (double)vx * (double)vy;
  const double r2 = num / den;
  return r2 > 1.0 ? 1.0 : r2;
}

/*
 * Minor allele frequency of one variant over its non-missing calls
 * (dosage counts A2 alleles): min(A2, 2n - A2) / 2n, and 0 with no
 * non-missing call.
 */
static double variant_maf(const int8_t* x, int64_t n) {
  int64_t calls = 0, a2 = 0;
  for (int64_t k = 0; k < n; ++k) {
    if (x[k] == MISSING) continue;
    calls += 1;
    a2 += dosage(x[k]);
  }
  if (calls == 0) return 0.0;
  const int64_t minor = a2 < 2 * calls - a2 ? a2 : 2 * calls - a2;
  return (double)minor / (double)(2 * calls);
}

/*
 * LD-based pruning, the --indep-pairwise operation the paper times (section
 * "Linkage disequilibrium-based variant pruning", Table 4), which it names but
 * does not spell out.  The reading implemented here:
 *  - windows of `window` consecutive variants start at 0, step, 2*step, ...;
 *    the last one is the first that reaches the end;
 *  - in each window, pairs a < b of variants that are still kept are visited
 *    in increasing a, then increasing b; when r^2 > r2_max (the double of
 *    oracle_r2_counts; an undefined r^2 never triggers) the variant with the
 *    lower minor allele frequency is dropped, the later one (b) on a tie;
 *  - a dropped variant stays dropped.
 * keep[v] = 1 for the variants that remain; returns their number.
 * r^2 of every pair closer than `window` is computed first (in parallel);
 * the greedy pass itself is the sequential loop above.
 */
int64_t oracle_ld_prune(const int8_t* codes_vm, int64_t n, int64_t V, int64_t window,
                        int64_t step, double r2_max, uint8_t* keep) {
  const int64_t span = window - 1;  /* largest b - a inside one window */
  double* r2 = (double*)malloc((size_t)(V * (span > 0 ? span : 1)) * sizeof(double));
  double* maf = (double*)malloc((size_t)V * sizeof(double));
  if (!r2 || !maf) {
    free(r2);
    free(maf);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < V; ++a) {
    maf[a] = variant_maf(codes_vm + a * n, n);
    for (int64_t d = 1; d <= span; ++d) {
      double v = NAN;
      if (a + d < V) {
        int64_t s[6];
        ld_sums(codes_vm + a * n, codes_vm + (a + d) * n, n, s);
        v = oracle_r2_counts(s);
      }
      r2[a * span + d - 1] = v;
    }
  }
  for (int64_t v = 0; v < V; ++v) keep[v] = 1;
  for (int64_t start = 0; start < V; start += step) {
    const int64_t end = start + window < V ? start + window : V;
    for (int64_t a = start; a < end; ++a) {
      if (!keep[a]) continue;
      for (int64_t b = a + 1; b < end; ++b) {
        if (!keep[b]) continue;
        if (!(r2[a * span + (b - a) - 1] > r2_max)) continue;
        if (maf[a] < maf[b]) {
          keep[a] = 0;
          break;
        }
        keep[b] = 0;
      }
    }
    if (end == V) break;
  }
  int64_t kept = 0;
  for (int64_t v = 0; v < V; ++v) kept += keep[v];
  free(r2);
  free(maf);
  return kept;
}

/*
 * Genomic relationship matrix (section "Partial sum lookup": the weighted
 * distance built from per-marker increments, with the GCTA relationship
 * increments as its example), the paper's first-draft algorithm: per marker,
 * a table of the increments of every genotype pair; per sample pair, the
 * table entries summed over markers, where a marker with a missing call adds
 * nothing and is not counted in that pair's denominator.
 *
 * Reading.  x = number of A2 alleles (0, 1, 2) and p = the A2 frequency over
 * the marker's non-missing calls; the increment of genotypes (x, y) is
 *   (x - 2p)(y - 2p) / (2p(1 - p)).
 * The paper states the cases with major/minor labels and the minor allele
 * frequency; counting either allele gives the same value as long as x and p
 * refer to the same allele.  Markers with no non-missing call or with p equal
 * to 0 or 1 (increments undefined) are left out of every pair.
 * A[i,j] = sum of increments / N[i,j], N[i,j] = markers counted for the
 * pair; NaN when N[i,j] = 0.  The diagonal uses the same increments with
 * i = j.  full != 0: n x n row-major; else strict upper triangle as in
 * oracle_ibs_matrix.  abs_sum (optional, same layout): the sum of the
 * increments' absolute values, for error bounds.
 */
/* Fills the per-marker increment tables of the relationship matrix (see
 * oracle_grm) and the markers' used flags. */
static void grm_tables(const int8_t* codes_sm, int64_t n, int64_t V, double* inc, uint8_t* used) {
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < V; ++v) {
    int64_t calls = 0, a2 = 0;
    for (int64_t k = 0; k < n; ++k) {
      const int8_t c = codes_sm[k * V + v];
      if (c == MISSING) continue;
      calls += 1;
      a2 += dosage(c);
    }
    used[v] = calls > 0 && a2 > 0 && a2 < 2 * calls;
    const double p = used[v] ? (double)a2 / (double)(2 * calls) : 0.0;
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y)
        inc[v * 9 + x * 3 + y] =
            used[v] ? ((double)x - 2.0 * p) * ((double)y - 2.0 * p) / (2.0 * p * (1.0 - p)) : 0.0;
  }
}

/* One pair's sum over markers of the table entries (markers left out or with
 * a missing call skipped). */
static void grm_pair(const int8_t* ci, const int8_t* cj, int64_t V, const double* inc,
                     const uint8_t* used, double* A, uint32_t* N, double* abs_sum) {
  double sum = 0.0, asum = 0.0;
  uint32_t cnt = 0;
  for (int64_t v = 0; v < V; ++v) {
    if (!used[v] || ci[v] == MISSING || cj[v] == MISSING) continue;
    const double t = inc[v * 9 + dosage(ci[v]) * 3 + dosage(cj[v])];
    sum += t;
    asum += fabs(t);
    cnt += 1;
  }
  *A = cnt ? sum / (double)cnt : NAN;
  *N = cnt;
  if (abs_sum) *abs_sum = asum;
}

void oracle_grm(const int8_t* codes_sm, int64_t n, int64_t V, int full, double* A, uint32_t* N,
                double* abs_sum) {
  /* per-marker increment tables, indexed [marker][dosage_i][dosage_j] */
  double* inc = (double*)malloc((size_t)V * 9 * sizeof(double));
  uint8_t* used = (uint8_t*)malloc((size_t)V);
  if (!inc || !used) {
    free(inc);
    free(used);
    return;
  }
  grm_tables(codes_sm, n, V, inc, used);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = full ? 0 : i + 1; j < n; ++j) {
      const int64_t idx = full ? i * n + j : i * n - i * (i + 1) / 2 + (j - i - 1);
      grm_pair(codes_sm + i * V, codes_sm + j * V, V, inc, used, A + idx, N + idx,
               abs_sum ? abs_sum + idx : NULL);
    }
  }
  free(inc);
  free(used);
}

/* The relationship matrix entries of a list of sample pairs (pi[k], pj[k]). */
void oracle_grm_pairs(const int8_t* codes_sm, int64_t n, int64_t V, const int64_t* pi,
                      const int64_t* pj, int64_t npairs, double* A, uint32_t* N, double* abs_sum) {
  double* inc = (double*)malloc((size_t)V * 9 * sizeof(double));
  uint8_t* used = (uint8_t*)malloc((size_t)V);
  if (!inc || !used) {
    free(inc);
    free(used);
    return;
  }
  grm_tables(codes_sm, n, V, inc, used);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < npairs; ++k)
    grm_pair(codes_sm + pi[k] * V, codes_sm + pj[k] * V, V, inc, used, A + k, N + k,
             abs_sum + k);
  free(inc);
  free(used);
}

/*
 * IBS distance between two samples (the --distance / --cluster input the
 * paper times in Table 2; it names the statistic but not its formula).
 * Reading: the proportion of alleles not shared identical by state over the
 * jointly non-missing markers, d = (2*IBS0 + IBS1) / (2*N), i.e. one minus
 * the IBS similarity (IBS2 + IBS1/2) / N; +infinity when N = 0.  Both counts
 * are integers, so d is their correctly rounded quotient.
 */
void oracle_ibs_distance(const uint32_t* ibs0, const uint32_t* ibs1, const uint32_t* nonmiss,
                         int64_t count, double* d) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < count; ++e)
    d[e] = nonmiss[e] ? (double)(2 * (int64_t)ibs0[e] + ibs1[e]) / (double)(2 * (int64_t)nonmiss[e])
                      : INFINITY;
}

/*
 * IBS similarity, the value --distance ibs reports (section "Identity-by-state
 * matrices, complete linkage clustering" names it without a formula).
 * Reading: the proportion of alleles shared identical by state over the
 * jointly non-missing markers, s = (IBS2 + IBS1/2) / N = (2*IBS2 + IBS1) /
 * (2*N), the correctly rounded quotient of the two integers; NaN when N = 0.
 */
void oracle_ibs_similarity(const uint32_t* ibs1, const uint32_t* ibs2, const uint32_t* nonmiss,
                           int64_t count, double* s) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < count; ++e)
    s[e] = nonmiss[e] ? (double)(2 * (int64_t)ibs2[e] + ibs1[e]) / (double)(2 * (int64_t)nonmiss[e])
                      : NAN;
}

/*
 * Expected IBS given IBD at one marker (the IBD report, --genome /
 * --Z-genome, that Table 2 times after the IBS matrix; the paper gives no
 * formulas, so this is the method-of-moments reading stated here).  The
 * marker's observed alleles are x copies of A2 and y of A1 (n = x + y >= 4).
 * Two samples that share no allele IBD carry four alleles drawn without
 * replacement from these n; with one allele IBD, three (the shared one and
 * one more each).  Counting the ordered draws:
 *   t[0] = P(IBS0 | IBD0) = 2 x(x-1) y(y-1) / n(n-1)(n-2)(n-3)
 *          (opposite homozygotes);
 *   t[1] = P(IBS1 | IBD0) = 4 [x(x-1)(x-2) y + x y(y-1)(y-2)] / n(n-1)(n-2)(n-3)
 *          (a homozygote and a heterozygote);
 *   t[2] = P(IBS2 | IBD0) = [x(x-1)(x-2)(x-3) + y(y-1)(y-2)(y-3)
 *          + 4 x(x-1) y(y-1)] / n(n-1)(n-2)(n-3)  (the same genotype);
 *   t[3] = P(IBS1 | IBD1) = 2 [x(x-1) y + x y(y-1)] / n(n-1)(n-2)
 *          (the two non-shared alleles differ);
 *   t[4] = P(IBS2 | IBD1) = [x(x-1)(x-2) + y(y-1)(y-2) + x(x-1) y
 *          + x y(y-1)] / n(n-1)(n-2);
 * and P(IBS2 | IBD2) = 1.  Evaluated in double exactly as written (products
 * left to right, the sums in the order shown, then one division).
 */
void oracle_genome_terms(int64_t x, int64_t y, double t[5]) {
  const double X = (double)x, Y = (double)y, n = (double)(x + y);
  const double d4 = n * (n - 1.0) * (n - 2.0) * (n - 3.0);
  const double d3 = n * (n - 1.0) * (n - 2.0);
  const double x2 = X * (X - 1.0), y2 = Y * (Y - 1.0);
  const double x3 = x2 * (X - 2.0), y3 = y2 * (Y - 2.0);
  t[0] = 2.0 * x2 * y2 / d4;
  t[1] = 4.0 * (x3 * Y + X * y3) / d4;
  t[2] = (x3 * (X - 3.0) + y3 * (Y - 3.0) + 4.0 * x2 * y2) / d4;
  t[3] = 2.0 * (x2 * Y + X * y2) / d3;
  t[4] = (x3 + y3 + x2 * Y + X * y2) / d3;
}

/*
 * The means of the five terms above over the markers of codes_vm
 * (variant-major, V rows of n codes) with at least 4 observed alleles among
 * these samples: E = {E00, E10, E20, E11, E21} and the number K of such
 * markers.  Each sum is formed in two levels: the terms of each run of
 * GENOME_RUN consecutive markers are added in increasing marker order,
 * starting from 0, then the runs' sums in increasing run order, starting
 * from 0; each mean is its sum divided by K.
 */
#define GENOME_RUN 1024
void oracle_genome_means(const int8_t* codes_vm, int64_t n, int64_t V, double E[5], int64_t* Kout) {
  double S[5] = {0, 0, 0, 0, 0}, R[5] = {0, 0, 0, 0, 0};
  int64_t K = 0;
  for (int64_t v = 0; v < V; ++v) {
    int64_t calls = 0, a2 = 0;
    for (int64_t k = 0; k < n; ++k) {
      const int8_t c = codes_vm[v * n + k];
      if (c == MISSING) continue;
      calls += 1;
      a2 += dosage(c);
    }
    if (2 * calls >= 4) {
      double t[5];
      oracle_genome_terms(a2, 2 * calls - a2, t);
      for (int q = 0; q < 5; ++q) R[q] += t[q];
      K += 1;
    }
    if ((v + 1) % GENOME_RUN == 0 || v == V - 1) {   /* the run ends */
      for (int q = 0; q < 5; ++q) {
        S[q] += R[q];
        R[q] = 0.0;
      }
    }
  }
  for (int q = 0; q < 5; ++q) E[q] = S[q] / (double)K;
  *Kout = K;
}

/*
 * The IBD report for IBS counts over the samples and variants of codes_vm:
 * the means E00, E10, E11 and K of oracle_genome_means, then for each of
 * `count` pairs with jointly non-missing count N:
 *   P0 = IBS0 / N,  P1 = IBS1 / N,
 *   Z0 = min(P0 / E00, 1),
 *   Z1 = (P1 - Z0 E10) / E11, clamped to [0, 1 - Z0],
 *   Z2 = (1 - Z0) - Z1,   PI_HAT = 0.5 Z1 + Z2
 * (the IBS0 and IBS1 moment equations; Z0 + Z1 + Z2 = 1).  All four are NaN
 * when N = 0, K = 0, E00 = 0 or E11 = 0.
 */
void oracle_genome(const int8_t* codes_vm, int64_t n, int64_t V, const uint32_t* ibs0,
                   const uint32_t* ibs1, const uint32_t* nonmiss, int64_t count, double* z0,
                   double* z1, double* z2, double* pi_hat) {
  double E[5];
  int64_t K = 0;
  oracle_genome_means(codes_vm, n, V, E, &K);
  const double E00 = E[0], E10 = E[1];
  const double E11 = E[3];
  const int ok = K > 0 && E00 != 0.0 && E11 != 0.0;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < count; ++e) {
    if (!ok || nonmiss[e] == 0) {
      z0[e] = z1[e] = z2[e] = pi_hat[e] = NAN;
      continue;
    }
    const double N = (double)nonmiss[e];
    const double p0 = (double)ibs0[e] / N, p1 = (double)ibs1[e] / N;
    double a = p0 / E00;
    if (a > 1.0) a = 1.0;
    double b = (p1 - a * E10) / E11;
    if (b < 0.0) b = 0.0;
    if (b > 1.0 - a) b = 1.0 - a;
    const double c = (1.0 - a) - b;
    z0[e] = a;
    z1[e] = b;
    z2[e] = c;
    pi_hat[e] = 0.5 * b + c;
  }
}

/*
 * Complete-linkage agglomerative clustering of m samples from their m x m
 * distance matrix (section "Identity-by-state matrices, complete linkage
 * clustering").  Plain definition: while more than one cluster remains,
 * merge the two clusters whose largest member-to-member distance is
 * smallest; ties go to the pair with the smallest first, then second,
 * cluster index.  A cluster is indexed by its smallest sample index.
 * merges[t] = {a, b, height} for step t (a < b, the two clusters' indices;
 * the merged cluster is a).  O(m^3); dist is not modified.
 */
typedef struct {
  int32_t a, b;
  double height;
} oracle_merge;

int oracle_cluster_complete(const double* dist, int64_t m, oracle_merge* merges) {
  double* d = (double*)malloc((size_t)(m * m) * sizeof(double));
  uint8_t* active = (uint8_t*)malloc((size_t)m);
  if (!d || !active) {
    free(d);
    free(active);
    return -1;
  }
  memcpy(d, dist, (size_t)(m * m) * sizeof(double));
  for (int64_t i = 0; i < m; ++i) active[i] = 1;
  for (int64_t t = 0; t + 1 < m; ++t) {
    int64_t bi = -1, bj = -1;
    double best = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      if (!active[i]) continue;
      for (int64_t j = i + 1; j < m; ++j) {
        if (!active[j]) continue;
        if (bi < 0 || d[i * m + j] < best) {
          best = d[i * m + j];
          bi = i;
          bj = j;
        }
      }
    }
    merges[t].a = (int32_t)bi;
    merges[t].b = (int32_t)bj;
    merges[t].height = best;
    /* complete linkage: the merged cluster's distance to k is the larger of
     * the two */
    for (int64_t k = 0; k < m; ++k) {
      if (!active[k] || k == bi || k == bj) continue;
      const double v = d[bi * m + k] > d[bj * m + k] ? d[bi * m + k] : d[bj * m + k];
      d[bi * m + k] = v;
      d[k * m + bi] = v;
    }
    active[bj] = 0;
  }
  free(d);
  free(active);
  return 0;
}
