// Internal declarations shared by the libpg sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pg.h"

namespace pg {

// Records a failure message for pg_last_error() and returns `status`.
int fail(int status, const char* fmt, ...);
// Checks the last HIP launch error; returns PG_OK or PG_EDEVICE.
int check_launch(const char* what);
// Records the caller's stage event k (pg_profile_events) on `st`, if set.
void mark_stage(int k, hipStream_t st);
// Fills n words with v by a kernel (no memset node, so graph replays are safe).
int fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// The caller's selection of a genotype matrix: which rows (variants) and
// which samples, with the optional missing mask folded into the codes.
struct Sel {
  const uint8_t* bed;      // variant-major .bed payload
  int64_t bpv;             // row stride in bytes
  const uint64_t* mask;    // optional missing mask, wpm words per row
  int64_t wpm;
  const int32_t* idx;      // optional sample list
  int64_t n;               // samples per row of the matrix
  int64_t m;               // selected samples
  int64_t v0;              // first selected variant
  int64_t nv;              // selected variants
};

// 2-bit .bed code of selected sample k at selected variant v (both local);
// positions past the selection, and list entries outside [0, n), read as 1
// (missing).
__device__ __forceinline__ uint32_t code_at(const Sel& s, int64_t v, int64_t k) {
  if (v >= s.nv || k >= s.m) return 1u;
  const int64_t row = s.v0 + v;
  const int64_t smp = s.idx ? (int64_t)s.idx[k] : k;
  if (smp < 0 || smp >= s.n) return 1u;
  uint32_t c = (s.bed[row * s.bpv + (smp >> 2)] >> (2 * (smp & 3))) & 3u;
  if (s.mask && ((s.mask[row * s.wpm + (smp >> 6)] >> (smp & 63)) & 1ull)) c = 1u;
  return c;
}

// Sixteen codes of one word, all positions "missing".
constexpr uint32_t kAllMissing16 = 0x55555555u;

// 2-bit word (16 codes) -> the three indicator masks at the even bit positions.
__device__ __forceinline__ void masks_of_word(uint32_t x, uint32_t& p, uint32_t& q, uint32_t& m) {
  const uint32_t lo = x & 0x55555555u, hi = (x >> 1) & 0x55555555u;
  p = lo & hi;                       // homA2
  q = ~(lo | hi) & 0x55555555u;      // homA1
  m = ~(lo & ~hi) & 0x55555555u;     // not code 01
}

// In-place transpose of a 16x16 matrix of 2-bit elements: element (r, c) at
// bits 2c of x[r] moves to bits 2r of x[c].  Recursive block swap: exchange
// the off-diagonal halves, then transpose each half-size block.
__device__ __forceinline__ void transpose16_2bit(uint32_t x[16]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t t = ((x[r] >> 16) ^ x[r + 8]) & 0x0000FFFFu;
    x[r] ^= t << 16;
    x[r + 8] ^= t;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if ((r & 4) == 0) {
      const uint32_t t = ((x[r] >> 8) ^ x[r + 4]) & 0x00FF00FFu;
      x[r] ^= t << 8;
      x[r + 4] ^= t;
    }
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if ((r & 2) == 0) {
      const uint32_t t = ((x[r] >> 4) ^ x[r + 2]) & 0x0F0F0F0Fu;
      x[r] ^= t << 4;
      x[r + 2] ^= t;
    }
#pragma unroll
  for (int r = 0; r < 16; r += 2) {
    const uint32_t t = ((x[r] >> 2) ^ x[r + 1]) & 0x33333333u;
    x[r] ^= t << 2;
    x[r + 1] ^= t;
  }
}

// ---- layout kernels (layout.hip) -------------------------------------------
// Sample-major 2-bit words: T[i*wp + w] holds codes of variants 16w..16w+15
// of selected sample i (code of variant 16w+t at bits 2t); rows_pad x wp.
int launch_sample_major_2bit(const Sel& s, uint32_t* T, int64_t rows_pad, int64_t wp,
                             hipStream_t st);
// Replicated fp4 operand (matrix-core variant 4): per sample, per group of 8
// variants, words HR (high code bits at nibble bits 1 and 3) and LR (low code
// bits at nibble bits 1 and 3, ones at bits 0 and 2); rp words per row.
int launch_sample_major_rep(const Sel& s, uint32_t* R, int64_t rows_pad, int64_t rp,
                            hipStream_t st);
// Sample-major bit planes for the popcount IBS path: for 32-variant word w,
// plane p (0 = high code bit, 1 = low code bit, 2 = non-missing) of sample i
// at P[(w*3 + p)*rows_pad + i]; words_pad words.
int launch_ibs_planes(const Sel& s, uint32_t* P, int64_t rows_pad, int64_t words_pad,
                      hipStream_t st);
// The same layout (without a sample list) for several operands in one
// launch: one job per operand, blocks [block_begin, block_begin +
// sample_major_job_blocks(rows_pad, wp)) of the launch lay it out.
struct LayoutJob {
  Sel s;
  uint32_t* T;
  int64_t rows_pad, wp, block_begin;
  int aligned;   // rows_dword_aligned(s)
};
bool rows_dword_aligned(const Sel& s);
int64_t sample_major_job_blocks(int64_t rows_pad, int64_t wp);
// jobs: device array of n_jobs jobs in increasing block_begin.
int launch_sample_major_jobs(const LayoutJob* jobs, int n_jobs, int64_t total_blocks,
                             hipStream_t st);
// Variant-major 2-bit words over the selected samples: D[v*wn + w] holds
// codes of samples 16w..16w+15 of selected variant v; rows_pad x wn.
int launch_variant_major_2bit(const Sel& s, uint32_t* D, int64_t rows_pad, int64_t wn,
                              hipStream_t st);

// Variant-major bit planes for the popcount LD path: for 32-sample word w,
// plane p (0 = homozygous A2, 1 = homozygous A1, 2 = non-missing) of selected
// variant v at P[(w*3 + p)*rows_pad + v]; words_pad words.
int launch_ld_planes(const Sel& s, uint32_t* P, int64_t rows_pad, int64_t words_pad,
                     hipStream_t st);

// ---- IBS ------------------------------------------------------------------
struct IbsOut {
  uint32_t* ibs0;
  uint32_t* ibs1;
  uint32_t* ibs2;
  uint32_t* nonmiss;
  int64_t m;     // matrix order
  int full;      // PG_FULL or PG_TRI_UPPER
  int u16;       // the arrays hold uint16 counts (PG_COUNTS_U16)
};
// out_layout of an IBS call: the layout and the count width; PG_EINVAL for
// an unknown layout or flag, or 16-bit counts over 65,536 variants or more.
int ibs_out_layout(int out_layout, int64_t nv, int& layout, int& u16);

constexpr int kIbsMfmaTile = 128;     // samples per tile side
constexpr int kIbsMfmaKWords = 16;    // 2-bit words per K chunk (256 variants)
constexpr int kIbsVariantFp4 = 3;     // matrix-core variant with fp4 operands
constexpr int kIbsVariantFp4Rep = 4;  // fp4 operands from the replicated layout
constexpr int kIbsVariantW8 = 5;      // eight waves of 64x32 (6: without scheduling hints)
constexpr int kIbsVariantPipe = 7;    // int8, chunk boundaries pipelined
constexpr int kIbsVariantFp4Pipe = 8; // fp4 operands, chunk boundaries pipelined (the default)
constexpr int kIbsVariantR1 = 9;      // int8, unpipelined, scheduling hints
constexpr int kIbsVariants = 10;      // variant codes 1 .. kIbsVariants - 1 are defined
// fp4 operands accumulate in fp32, exact while every sum stays below 2^24
constexpr int64_t kFp4MaxVariants = (int64_t)1 << 24;
constexpr int kIbsRepChunk = 64;      // replicated words per K chunk (256 variants)
constexpr int kIbsPopcTile = 64;
constexpr int kIbsPopcKWords = 16;    // 32-bit plane words per K chunk

// Operand plan of an IBS call: resolved path and variant, operand rows and K
// words, workspace bytes.
struct IbsPlan {
  int path;
  int variant;
  int64_t rows_pad, words;
  int64_t off_part;   // K-split sums of the default matrix-core kernel (-1: none)
  int64_t bytes;
};
// The plan of the default matrix-core kernel for a selection (abi.hip).
int plan_ibs_default(const Sel& s, IbsPlan& p);

// The path PG_PATH_AUTO resolves to for an IBS matrix of m samples and nv
// variants (abi.hip).
int ibs_auto_path(int64_t m, int64_t nv);
// The path PG_PATH_AUTO resolves to for LD windows (abi.hip).
int ld_auto_path(int64_t m, int64_t nv, int32_t window);

// Static scratch of pg_ibs_matrix_noalloc (abi.hip): its size, and its
// device address on the current device (looked up once per device).
constexpr int64_t kNoAllocScratchBytes = (int64_t)64 << 20;
constexpr int kMaxDevices = 64;
int noalloc_scratch(void** ptr);

// `part`: workspace of ibs_part_bytes() for the default kernel's K split
// (nullptr: never split).
int launch_ibs_mfma(const uint32_t* T, int64_t wp, const IbsOut& o, int variant, hipStream_t st,
                    int32_t* part = nullptr);
// K split of a tile kernel that runs one block per CU on the 256 CUs: each
// of `tiles` tiles has `chunks` K chunks, split into n_split ranges of cps
// chunks (cps >= min_cps, n_split <= max_split, tiles * n_split <= 2,048).
// The time in chunk units is ceil(tiles * n_split / 256) * cps (rounds of the
// CUs times the chunks per block) plus, when split, reduce_cost per tile and
// range (reading its partial sums back); the split steps to more ranges only
// where that saves 5%.  Grids of 512 tiles or more (two rounds and up) are
// left to the tail split below.
inline void split_ranges(int64_t tiles, int64_t chunks, int64_t min_cps, int64_t max_split,
                         double reduce_cost, int64_t& n_split, int64_t& cps) {
  n_split = 1;
  cps = chunks;
  if (tiles < 1 || tiles >= 512 || chunks < 2 * min_cps) return;
  double best = (double)ceil_div(tiles, 256) * (double)chunks;
  for (int64_t want = 2; want <= max_split && want * tiles <= 2048; ++want) {
    const int64_t c = ceil_div(chunks, want);
    if (c < min_cps) break;
    const int64_t n = ceil_div(chunks, c);
    const double cost = (double)ceil_div(tiles * n, 256) * (double)c + reduce_cost * tiles * n;
    if (cost < 0.95 * best) {
      best = cost;
      n_split = n;
      cps = c;
    }
  }
}

// K split of the default IBS matrix-core kernel (chunks of 256 variants, at
// least two per range, at most 32 ranges).  The ranges park their raw sums
// (192 int32 per thread of the 256) in the workspace and a second kernel
// adds them in range order.  n_split == 1: no split.  A block takes about
// 2.5 us per chunk and reading one range's 196,608 bytes back about 0.05 us
// of the whole chip's time: 0.02 chunks.
inline void ibs_split(int64_t rows_pad, int64_t wp, int64_t& n_split, int64_t& cps) {
  const int64_t nt = rows_pad / kIbsMfmaTile;
  split_ranges(nt * (nt + 1) / 2, wp / kIbsMfmaKWords, 2, 32, 0.02, n_split, cps);
}
// Tail split of the whole-tile launch (grids too large for ibs_split).  The
// tiles, in the banded order without empty positions, are cut into 8
// contiguous runs of equal length (+-1), one per XCD; the head of each run
// -- `head` tiles, whole rounds of the XCD's 32 CUs -- runs whole tiles, and
// the rest of the run (at most rmax tiles) runs as n_split K ranges of cps
// chunks each, whose raw sums a reduce kernel adds in range order.
// tail == false: no tail split.
struct IbsTail {
  bool tail = false;
  int64_t head = 0, rmax = 0, n_split = 1, cps = 0;
  int64_t start[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // run x = [start[x], start[x + 1])
};
IbsTail ibs_tail_plan(int64_t rows_pad, int64_t wp);
inline int64_t ibs_part_bytes(int64_t rows_pad, int64_t wp) {
  int64_t n_split, cps;
  ibs_split(rows_pad, wp, n_split, cps);
  const int64_t nt = rows_pad / kIbsMfmaTile;
  if (n_split > 1) return n_split * (nt * (nt + 1) / 2) * 192 * 256 * 4;
  const IbsTail t = ibs_tail_plan(rows_pad, wp);
  return t.tail ? 8 * t.rmax * t.n_split * 192 * 256 * 4 : 0;
}
int launch_ibs_fp4rep(const uint32_t* R, int64_t rp, const IbsOut& o, hipStream_t st);
int launch_ibs_popc(const uint32_t* P, int64_t rows_pad, int64_t words_pad, const IbsOut& o,
                    hipStream_t st);

// ---- LD -------------------------------------------------------------------
constexpr int kLdTile = 64;           // variants per tile side
constexpr int kLdKWords = 16;         // 2-bit words per K chunk (256 samples)

struct LdScratch {
  uint32_t* bitmap;    // rows_pad x bm_words, bit (b-a-1) of row a
  int64_t bm_words;
  uint32_t* rowcnt;    // rows_pad
  int64_t* rowoff;     // rows_pad + 1
  int64_t* bsum;       // ld_scan_blocks(rows) per-block sums
};
// Number of per-block partial sums the row-offset scan needs.
int ld_scan_blocks(int64_t nv);

constexpr int kLdPopcKWords = 16;     // 32-bit plane words per K chunk

// Missing-call correction path (ldsparse.hip): per-variant missing-call
// lists (cap entries per variant, a multiple of 8), counts and totals
// {c, sum x, sum x^2, 0}, and per 64-variant group the total and largest
// count.  A tile (I, J) takes the path when ld_tile_sparse holds.
struct LdSparse {
  uint32_t* lists;     // rows_pad x cap entries (sample indices, increasing)
  int4* vst;           // rows_pad
  int64_t* gsum;       // rows_pad / 64
  int* gmax;           // rows_pad / 64
  uint32_t* groups_ok; // 1 word: groups whose diagonal tile qualifies
  uint32_t min_groups; // the path is on when groups_ok reaches this
  int cap;
  int64_t budget;      // largest missing-call total of a tile's two groups
  // optional sampled gate: the statistics pass (and with it the path) runs
  // only while *gate, the missing calls counted over a sample of the
  // variants, is at most gate_max
  uint64_t* gate;
  uint64_t gate_max;
  int64_t gate_stride; // every gate_stride-th variant is sampled
};
__device__ inline bool ld_tile_sparse(const int64_t* gsum, const int* gmax,
                                      const uint32_t* groups_ok, uint32_t min_groups, int64_t I,
                                      int64_t J, int cap, int64_t budget) {
  return *groups_ok >= min_groups && gmax[I] <= cap && gmax[J] <= cap &&
         gsum[I] + gsum[J] <= budget;
}
// Slot length of the missing-call lists for m selected samples.
inline int ld_sparse_cap(int64_t m) {
  int64_t c = round_up(ceil_div(m, 16), 8);
  if (c < 64) c = 64;
  if (c > 65528) c = 65528;
  return (int)c;
}

// Clears the emission bitmap and row counts (stage 1 ends after this).
int ld_clear(const LdScratch& sc, int64_t rows_pad, hipStream_t st);
// Dense pair kernel over the band; with `sp`, tiles the correction path
// takes are skipped (and stage 2 is left to that path).  fp4: the pipelined
// fp4 tile (exact below 2^24 samples), else the int8 tile.
int launch_ld_mfma(const uint32_t* D, int64_t wn, int64_t nv, int64_t rows_pad, int32_t window,
                   double r2_min, const LdScratch& sc, hipStream_t st,
                   const LdSparse* sp = nullptr, bool fp4 = true);
// Kernel variants of the LD matrix-core path: 0 (default) the pipelined fp4
// tile, or the int8 tile (1) when sums could reach 2^24 (m >= 2^24).
constexpr int kLdVariantFp4 = 0;
constexpr int kLdVariantInt8 = 1;
// Correction path, first part: lists, counts and totals from D
// (variant-major, wn words), the group statistics and groups_ok.
int launch_ld_sparse_stats(const uint32_t* D, int64_t wn, int64_t m, int64_t nv,
                           int64_t rows_pad, const LdSparse& sp, hipStream_t st);
// The sample-major operand of the corrections, transposed from D in strips
// of 64 variants: word w (0-3) of strip s at sample k is T[(s * t_rows + k) *
// 4 + w] (t_rows = round_up(m, 128); tw words of 16 variants per sample, a
// multiple of 4); nothing when the path is off.
int launch_ld_transpose(const uint32_t* D, int64_t rows_pad, int64_t wn, uint32_t* T,
                        int64_t t_rows, int64_t tw, const LdSparse& sp, hipStream_t st);
// Second part: the dense kernel on the tiles this path leaves, then the
// correction kernel with D for the Gram and T (the strips above, built after
// the first part) for the corrections.  With `dbg`,
// the dense kernel is not run and each pair of a correction tile writes its
// record to dbg[a * window + (b - a - 1)] (a, b local; the record holds
// v0 + a, v0 + b) instead of the emission test.
int launch_ld_sparse(const uint32_t* D, int64_t wn, const uint32_t* T, int64_t t_rows, int64_t m,
                     int64_t nv, int64_t rows_pad, int32_t window, double r2_min,
                     const LdScratch& sc, const LdSparse& sp, hipStream_t st,
                     pg_ld_pair* dbg = nullptr, int64_t v0 = 0);
int launch_ld_popc(const uint32_t* P, int64_t words_pad, int64_t nv, int64_t rows_pad,
                   int32_t window, double r2_min, const LdScratch& sc, hipStream_t st);
// Row-offset scan, *n_out, and the emit kernel.  X is the operand the pair
// kernel used: 2-bit words (rows x words) or bit planes (planes == true).
// `marks` records stage events 3 and 4 (one-problem calls only).
int launch_ld_finish(const uint32_t* X, bool planes, int64_t words, int64_t rows_pad, int64_t nv,
                     int64_t v0, const LdScratch& sc, pg_ld_pair* out, int64_t capacity,
                     int64_t* n_out, hipStream_t st, bool marks = true);

// ---- LD pruning (prune.hip) -------------------------------------------------
// Per selected variant: {minor allele count, non-missing calls (at least 1)}
// over the selected samples, from the operand of the LD pair kernel.
int launch_variant_stats(const uint32_t* X, bool planes, int64_t words, int64_t rows_pad,
                         int64_t nv, int2* stats, hipStream_t st);
// The greedy pass over the windows, from the pair kernel's bitmap of pairs
// with r^2 above the threshold (bitmap window = window - 1); `drop` is
// scratch of the bitmap's size for the drop side of every marked pair.
// `cc`: scratch for cc_capacity uint16 per-cell counts.  When the call's
// (window, row) cells, padded to whole passes, fit, they are counted
// grid-wide first; otherwise (or with cc NULL) the pass counts in its own
// block.
int launch_prune_greedy(const LdScratch& sc, const int2* stats, uint32_t* drop, uint16_t* cc,
                        int64_t cc_capacity, int64_t nv, int64_t window, int64_t step,
                        uint8_t* keep, int64_t* n_kept, hipStream_t st);
constexpr int64_t kPruneMaxWindow = 1 << 16;
// Most per-cell counts kept in scratch (128 MiB of uint16).
constexpr int64_t kPruneCountCellsMax = (int64_t)1 << 26;
// Count scratch a pruning plan reserves: enough for any step, capped.
int64_t prune_count_capacity(int64_t nv, int64_t window);

// ---- relationship matrix (grm.hip) -------------------------------------------
// Per-marker z tables and the fp64 matrix-core Gram over the sample-major
// 2-bit operand T (rows_pad multiple of 128, wp multiple of 4 words).
// `part` holds the K-split partial sums and counts (grm_part_bytes).
// waves: 4 (64 x 64 each), 8 (32 x 64) or 16 (32 x 32) waves per 128 x 128
// tile.
int launch_grm(const Sel& s, const uint32_t* T, int64_t rows_pad, int64_t wp, double* ztab,
               uint32_t* used2, double* part, double* grm, uint32_t* n_used, int full,
               int waves, hipStream_t st);
// K split of the relationship-matrix kernel (chunks of 128 variants, at
// least eight per range, at most 16 ranges; about 19 us per chunk, so a
// range's 196,608 bytes of partial sums cost 0.003 chunks to read back).
inline void grm_split(int64_t rows_pad, int64_t wp, int64_t& n_split, int64_t& cps) {
  const int64_t nt = rows_pad / 128;
  split_ranges(nt * (nt + 1) / 2, wp / 8, 8, 16, 0.003, n_split, cps);
}
inline int64_t grm_part_bytes(int64_t rows_pad, int64_t wp) {
  int64_t n_split, cps;
  grm_split(rows_pad, wp, n_split, cps);
  const int64_t nt = rows_pad / 128;
  return n_split > 1 ? n_split * (nt * (nt + 1) / 2) * 128 * 128 * (8 + 4) : 0;
}

// ---- IBS distance and clustering (cluster.hip) ------------------------------
int launch_ibs_distance(const uint32_t* i0, const uint32_t* i1, const uint32_t* nm, int64_t count,
                        double* d, hipStream_t st);
int launch_ibs_similarity(const uint32_t* i1, const uint32_t* i2, const uint32_t* nm,
                          int64_t count, double* s, hipStream_t st);
// IBD report from the variant-major operand D of the selection (rows_pad x
// wn words): terms 5 x rows_pad doubles, used rows_pad words, sums
// genome_sums_doubles(nv) doubles of workspace (the six totals, padded to 8,
// then six per run of 1,024 markers); then `count` pairs of IBS counts.
// Stage 1 ends after the per-marker averages.
inline int64_t genome_runs(int64_t nv) { return nv > 0 ? (nv + 1023) / 1024 : 1; }
inline int64_t genome_sums_doubles(int64_t nv) { return 8 + 6 * genome_runs(nv); }
int launch_genome(const uint32_t* D, int64_t wn, int64_t nv, int64_t rows_pad, double* terms,
                  uint32_t* used, double* sums, const uint32_t* i0, const uint32_t* i1,
                  const uint32_t* nm, int64_t count, double* z0, double* z1, double* z2,
                  double* pi, hipStream_t st);
// D: m x m doubles; nn_d: m doubles; nn_j: m ints; ctl: 4 ints (the first two
// count the rows to rescan); rows: m ints.  From kClusterSplitMin samples on,
// each merge runs as two launches over the chip (the pair and the fold; the
// rescans) instead of one block's loop.
constexpr int64_t kClusterSplitMin = 3200;
int launch_ibs_cluster(const uint32_t* i0, const uint32_t* i1, const uint32_t* nm, int64_t m,
                       double* D, double* nn_d, int* nn_j, int* ctl, int* rows,
                       pg_merge* merges, hipStream_t st);

// r^2 from exact sums, as documented in pg.h; shared by every LD path so that
// the emission decision and the emitted value are the same double.
// Integer route of ld_r2 for sums beyond 2^26 (kept out of line: rare).
__device__ __noinline__ double ld_r2_wide(int64_t n, int64_t sx, int64_t sy, int64_t sxx,
                                          int64_t syy, int64_t sxy) {
  const int64_t c = n * sxy - sx * sy;
  const int64_t va = n * sxx - sx * sx;
  const int64_t vb = n * syy - sy * sy;
  if (n == 0 || va == 0 || vb == 0) return __longlong_as_double(0x7ff8000000000000ll);
  const double num = __dmul_rn((double)c, (double)c);
  const double den = __dmul_rn((double)va, (double)vb);
  const double r2 = __ddiv_rn(num, den);
  return r2 > 1.0 ? 1.0 : r2;
}

__device__ __forceinline__ double ld_r2(int64_t n, int64_t sx, int64_t sy, int64_t sxx,
                                        int64_t syy, int64_t sxy) {
  if (n >= ((int64_t)1 << 26)) return ld_r2_wide(n, sx, sy, sxx, syy, sxy);
  // every sum is at most n in magnitude, so each product is below 2^52 and
  // each difference below 2^53: all exact in double, the same values as the
  // integer route, without 64-bit integer multiplies
  const double dn = (double)(int)n, dx = (double)(int)sx, dy = (double)(int)sy;
  const double c = __dsub_rn(__dmul_rn(dn, (double)(int)sxy), __dmul_rn(dx, dy));
  const double va = __dsub_rn(__dmul_rn(dn, (double)(int)sxx), __dmul_rn(dx, dx));
  const double vb = __dsub_rn(__dmul_rn(dn, (double)(int)syy), __dmul_rn(dy, dy));
  if (n == 0 || va == 0.0 || vb == 0.0) return __longlong_as_double(0x7ff8000000000000ll);
  const double r2 = __ddiv_rn(__dmul_rn(c, c), __dmul_rn(va, vb));
  return r2 > 1.0 ? 1.0 : r2;
}

// ld_r2(...) >= r2_min, the emission test, with the division skipped for
// pairs whose quotient is clearly below r2_min: if c^2 < fl(fl(r2_min * den)
// * (1 - 2^-50)) then c^2 / den < r2_min (1 - 2^-51), whose rounding is still
// below r2_min, so the test fails exactly as the full evaluation would.
// NaN r2 (n, va or vb zero) never passes.
//
// Before that, a cheaper test rejects most pairs: below 2^15 samples every
// sum is below 2^15 in magnitude, so c, va and vb are exact in int32 (each
// product below 2^30).  In float each conversion and product is within
// 2^-24 relative (nine roundings in all), so fl(c)^2 < fl(fl(r2_min) *
// fl(va) fl(vb)) (1 - 2^-16) implies c^2 / (va vb) < r2_min (1 - 2^-17),
// which the double route also rounds below r2_min.  NaN and infinite
// products compare false and fall through.
__device__ __forceinline__ bool ld_r2_reaches(int64_t n, int64_t sx, int64_t sy, int64_t sxx,
                                              int64_t syy, int64_t sxy, double r2_min) {
  if (n < (1 << 15) && r2_min > 0.0) {
    const int32_t ni = (int32_t)n, x = (int32_t)sx, y = (int32_t)sy;
    const float c = (float)(ni * (int32_t)sxy - x * y);
    const float va = (float)(ni * (int32_t)sxx - x * x);
    const float vb = (float)(ni * (int32_t)syy - y * y);
    if (c * c < (float)r2_min * (va * vb) * (1.0f - 0x1p-16f)) return false;
  }
  if (n >= ((int64_t)1 << 26)) return ld_r2_wide(n, sx, sy, sxx, syy, sxy) >= r2_min;
  const double dn = (double)(int)n, dx = (double)(int)sx, dy = (double)(int)sy;
  const double c = __dsub_rn(__dmul_rn(dn, (double)(int)sxy), __dmul_rn(dx, dy));
  const double va = __dsub_rn(__dmul_rn(dn, (double)(int)sxx), __dmul_rn(dx, dx));
  const double vb = __dsub_rn(__dmul_rn(dn, (double)(int)syy), __dmul_rn(dy, dy));
  if (n == 0 || va == 0.0 || vb == 0.0) return false;
  const double num = __dmul_rn(c, c), den = __dmul_rn(va, vb);
  if (num < __dmul_rn(__dmul_rn(r2_min, den), 1.0 - 0x1p-50)) return false;
  const double r2 = __ddiv_rn(num, den);
  return (r2 > 1.0 ? 1.0 : r2) >= r2_min;
}

}  // namespace pg
