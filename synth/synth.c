/*
 * Seeded synthetic genotype generators that write PLINK 1 binary (.bed)
 * payloads: variant-major rows, 2-bit codes, four samples per byte, sample k
 * of a row at bits 2*(k%4) of byte k/4.  Code 0 = homozygous A1, 1 = missing,
 * 2 = heterozygous, 3 = homozygous A2.  No 3-byte file header is written.
 *
 * This module only draws inputs.  It holds none of the pairwise statistics
 * (IBS counts, LD sums); both the CPU oracle and the GPU library consume its
 * output, and neither links against the other.
 *
 * Random numbers: xoshiro256** (Blackman and Vigna, "Scrambled linear
 * pseudorandom number generators", 2018/2021), each stream seeded with four
 * consecutive outputs of SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), as those authors recommend.
 * Every (purpose, index) pair gets its own stream, so results do not depend on
 * the number of OpenMP threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SPLITMIX_GAMMA 0x9E3779B97F4A7C15ULL

static uint64_t splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += SPLITMIX_GAMMA);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xoshiro;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t xo_next(xoshiro* r) {
  const uint64_t result = rotl64(r->s[1] * 5, 7) * 9;
  const uint64_t t = r->s[1] << 17;
  r->s[2] ^= r->s[0];
  r->s[3] ^= r->s[1];
  r->s[1] ^= r->s[2];
  r->s[0] ^= r->s[3];
  r->s[2] ^= t;
  r->s[3] = rotl64(r->s[3], 45);
  return result;
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double xo_unif(xoshiro* r) { return (double)(xo_next(r) >> 11) * 0x1.0p-53; }

/* Stream purposes; the stream key mixes seed, purpose and index. */
enum { ST_HWE_VARIANT = 1, ST_FOUNDER = 2, ST_HAPLO = 3, ST_MISSING = 4, ST_PAD = 5, ST_MASK = 6 };

static xoshiro xo_stream(uint64_t seed, uint64_t purpose, uint64_t index) {
  uint64_t st = seed ^ (purpose * 0xD1B54A32D192ED03ULL) ^ (index * 0xAEF17502108EF2D9ULL);
  /* burn one output so nearby keys decorrelate before seeding */
  (void)splitmix64_next(&st);
  xoshiro r;
  for (int i = 0; i < 4; ++i) r.s[i] = splitmix64_next(&st);
  return r;
}

static inline int64_t bytes_per_row(int64_t n) { return (n + 3) / 4; }

static void put_code(uint8_t* row, int64_t k, int code) {
  row[k >> 2] |= (uint8_t)(code << (2 * (k & 3)));
}

/* Fill the unused high bits of each row's last byte with random bits when
 * garbage_pad is set (consumers must ignore them), else leave them zero. */
static void fill_padding(uint8_t* bed, int64_t n, int64_t V, int64_t bpv, uint64_t seed, int garbage_pad) {
  if (!garbage_pad || (n & 3) == 0) return;
  const int used_bits = 2 * (int)(n & 3);
  const uint8_t pad_mask = (uint8_t)(0xFFu << used_bits);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < V; ++v) {
    xoshiro r = xo_stream(seed, ST_PAD, (uint64_t)v);
    bed[v * bpv + (n >> 2)] |= (uint8_t)(xo_next(&r) & pad_mask);
  }
}

/*
 * Hardy-Weinberg panel.  Per variant: A1 frequency q ~ U[q_lo, q_hi].  Per
 * call: u ~ U[0,1); homA1 if u < q^2, het if u < q^2 + 2q(1-q), else homA2.
 * Then, independently per call, the call is set missing with probability miss.
 * bed must hold V * ceil(n/4) bytes.
 */
int synth_hwe(int64_t n, int64_t V, double q_lo, double q_hi, double miss, uint64_t seed,
              int garbage_pad, uint8_t* bed) {
  if (n <= 0 || V <= 0 || !bed || q_lo < 0 || q_hi > 1 || q_lo > q_hi || miss < 0 || miss > 1) return -1;
  const int64_t bpv = bytes_per_row(n);
  memset(bed, 0, (size_t)(V * bpv));
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < V; ++v) {
    xoshiro r = xo_stream(seed, ST_HWE_VARIANT, (uint64_t)v);
    const double q = q_lo + (q_hi - q_lo) * xo_unif(&r);
    const double p_hom1 = q * q, p_het_cum = q * q + 2.0 * q * (1.0 - q);
    uint8_t* row = bed + v * bpv;
    for (int64_t k = 0; k < n; ++k) {
      const double u = xo_unif(&r);
      int code = (u < p_hom1) ? 0 : (u < p_het_cum) ? 2 : 3;
      if (xo_unif(&r) < miss) code = 1;
      put_code(row, k, code);
    }
  }
  fill_padding(bed, n, V, bpv, seed, garbage_pad);
  return 0;
}

/*
 * Founder-mosaic panel (linkage decays with distance).  F founder haplotypes:
 * at candidate variant c, founder f carries allele A2 with probability p_c,
 * p_c ~ U[0.05, 0.95].  Each sample has two haplotypes; each starts on a
 * uniformly drawn founder and, at every following candidate, with probability
 * switch_p jumps to a uniformly drawn founder (possibly the same one).  The
 * copied allele flips with probability mu.  Genotype = number of A2 alleles
 * (0 -> homA1, 1 -> het, 2 -> homA2).  Candidates whose sample minor allele
 * frequency (before missingness) is below maf_min are dropped, and candidates
 * are drawn until exactly V pass.  Last, each call is set missing with
 * probability miss.  Returns the number of candidates drawn, or -1.
 */
int64_t synth_mosaic(int64_t n, int64_t V, int F, double switch_p, double mu, double maf_min,
                     double miss, uint64_t seed, int garbage_pad, uint8_t* bed) {
  if (n <= 0 || V <= 0 || !bed || F <= 0 || F > 255 || switch_p < 0 || switch_p > 1 || mu < 0 ||
      mu > 1 || miss < 0 || miss > 1)
    return -1;
  const int64_t bpv = bytes_per_row(n);
  const int64_t H = 2 * n;
  const int64_t CH = 2048; /* candidates per chunk */
  memset(bed, 0, (size_t)(V * bpv));

  uint8_t* founder = (uint8_t*)malloc((size_t)H);       /* current founder per haplotype */
  xoshiro* hr = (xoshiro*)malloc(sizeof(xoshiro) * (size_t)H);
  uint8_t* fall = (uint8_t*)malloc((size_t)(CH * F));   /* founder alleles, [c][f] */
  uint8_t* hall = (uint8_t*)malloc((size_t)(CH * H));   /* haplotype alleles, [c][h] */
  uint8_t* keep = (uint8_t*)malloc((size_t)CH);
  int64_t* dest = (int64_t*)malloc(sizeof(int64_t) * (size_t)CH);
  if (!founder || !hr || !fall || !hall || !keep || !dest) {
    free(founder); free(hr); free(fall); free(hall); free(keep); free(dest);
    return -1;
  }
  for (int64_t h = 0; h < H; ++h) {
    hr[h] = xo_stream(seed, ST_HAPLO, (uint64_t)h);
    founder[h] = (uint8_t)(xo_unif(&hr[h]) * F);
  }

  int64_t kept = 0, cand = 0;
  while (kept < V) {
    /* founder alleles for this chunk */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < CH; ++c) {
      xoshiro r = xo_stream(seed, ST_FOUNDER, (uint64_t)(cand + c));
      const double p = 0.05 + 0.90 * xo_unif(&r);
      for (int f = 0; f < F; ++f) fall[c * F + f] = (uint8_t)(xo_unif(&r) < p);
    }
    /* haplotype walks: sequential over candidates, parallel over haplotypes */
#pragma omp parallel for schedule(static)
    for (int64_t h = 0; h < H; ++h) {
      xoshiro r = hr[h];
      uint8_t f = founder[h];
      for (int64_t c = 0; c < CH; ++c) {
        if ((cand + c) > 0 && xo_unif(&r) < switch_p) f = (uint8_t)(xo_unif(&r) * F);
        uint8_t a = fall[c * F + f];
        if (xo_unif(&r) < mu) a ^= 1u;
        hall[c * H + h] = a;
      }
      hr[h] = r;
      founder[h] = f;
    }
    /* minor-allele-frequency filter */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < CH; ++c) {
      int64_t alt = 0;
      for (int64_t h = 0; h < H; ++h) alt += hall[c * H + h];
      const double fr = (double)alt / (double)H;
      const double maf = fr < 0.5 ? fr : 1.0 - fr;
      keep[c] = (uint8_t)(maf >= maf_min);
    }
    for (int64_t c = 0; c < CH; ++c) {
      dest[c] = (keep[c] && kept < V) ? kept : -1;
      if (dest[c] >= 0) ++kept;
    }
    /* genotypes, then missingness keyed by the output variant index */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < CH; ++c) {
      if (dest[c] < 0) continue;
      const int64_t v = dest[c];
      xoshiro r = xo_stream(seed, ST_MISSING, (uint64_t)v);
      uint8_t* row = bed + v * bpv;
      for (int64_t k = 0; k < n; ++k) {
        const int s = hall[c * H + 2 * k] + hall[c * H + 2 * k + 1];
        int code = (s == 0) ? 0 : (s == 1) ? 2 : 3;
        if (xo_unif(&r) < miss) code = 1;
        put_code(row, k, code);
      }
    }
    cand += CH;
  }
  free(founder); free(hr); free(fall); free(hall); free(keep); free(dest);
  fill_padding(bed, n, V, bpv, seed, garbage_pad);
  return cand;
}

/*
 * Optional missing-call bitmask: V rows of ceil(n/64) little-endian uint64
 * words, bit (k%64) of word k/64 set means sample k is missing at that
 * variant.  Each bit is set with probability rate; bits past n stay zero.
 */
int synth_missing_mask(int64_t n, int64_t V, double rate, uint64_t seed, uint64_t* mask) {
  if (n <= 0 || V <= 0 || !mask || rate < 0 || rate > 1) return -1;
  const int64_t wpv = (n + 63) / 64;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < V; ++v) {
    xoshiro r = xo_stream(seed, ST_MASK, (uint64_t)v);
    uint64_t* row = mask + v * wpv;
    for (int64_t w = 0; w < wpv; ++w) row[w] = 0;
    for (int64_t k = 0; k < n; ++k)
      if (xo_unif(&r) < rate) row[k >> 6] |= 1ULL << (k & 63);
  }
  return 0;
}

/* First outputs of the two published generators, for self-tests. */
uint64_t synth_splitmix64_first(uint64_t state) { return splitmix64_next(&state); }
uint64_t synth_xoshiro_first(uint64_t s0, uint64_t s1, uint64_t s2, uint64_t s3) {
  xoshiro r = {{s0, s1, s2, s3}};
  return xo_next(&r);
}
