/*
 * pg -- pairwise genotype statistics on AMD MI355X (gfx950).
 *
 * C ABI of libpg.so.  The library computes, on the GPU, the two pairwise
 * kernels that PLINK 1.9 accelerates with word-level bit operations (Chang et
 * al., "Second-generation PLINK", GigaScience 2015, arXiv 1410.4803), and the
 * analyses the paper times on top of them:
 *
 *  - identity-by-state: for every sample pair, the number of markers where
 *    the two samples share 2, 1 or 0 alleles identical by state, and the
 *    number of markers where neither call is missing (section "Bitwise
 *    parallelism", the per-marker IBS loop and its XOR / mask / popcount
 *    replacement);
 *  - linkage disequilibrium: for every variant pair within a window, the six
 *    sums n, Sx, Sy, Sxx, Syy, Sxy over the samples where neither call is
 *    missing, and r^2 (section "Bit population count", the expression for r
 *    with missing data);
 *  - LD-based pruning, --indep-pairwise (section "Linkage disequilibrium-based
 *    variant pruning", Table 4);
 *  - the genomic relationship matrix (section "Partial sum lookup", Table 3);
 *  - the IBS distance and complete-linkage clustering on it (section
 *    "Identity-by-state matrices, complete linkage clustering", Table 2);
 *  - batched execution of many IBS / LD problems in persistent launches.
 *
 * Input is the PLINK 1 binary genotype payload (.bed without its 3-byte
 * header): variant-major rows of 2-bit codes, four calls per byte, sample k of
 * a row at bits 2*(k%4) of byte k/4:
 *     0 = homozygous A1, 1 = missing, 2 = heterozygous, 3 = homozygous A2.
 * Bits past the last sample of a row are ignored.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers, allocated and owned by the
 *    caller.  The library keeps no pointer after a call returns and never
 *    allocates device memory: scratch space is the caller's `workspace`, of
 *    at least the size the matching *_workspace_bytes call reports.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL means
 *    the default stream).  Outputs are valid after the stream synchronises.
 *  - Argument errors are detected on the host before anything is enqueued and
 *    return PG_EINVAL (or PG_ENOMEM for a short workspace); a failed launch
 *    returns PG_EDEVICE.  The library never aborts and never prints;
 *    pg_last_error() describes the last failure of the calling thread.
 *  - Calls on different streams may run concurrently; they share no state.
 */
#ifndef PG_H
#define PG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PG_VERSION 1

enum pg_status {
  PG_OK = 0,
  PG_EINVAL = -1,       /* invalid argument */
  PG_ENOMEM = -2,       /* workspace smaller than required */
  PG_EDEVICE = -3,      /* HIP runtime or launch failure */
  PG_EUNSUPPORTED = -4  /* valid request this build cannot serve */
};

/* Static text for a status code. */
const char* pg_status_str(int status);
/* Detail of the calling thread's last failure ("" if none). */
const char* pg_last_error(void);
/* PG_VERSION of the built library. */
int pg_version(void);

/*
 * Stage timing, for measurement.  After this call, every pg_* compute call
 * made by the calling thread records events[0] on its stream before its first
 * kernel and events[k] after its k-th stage, for k < n_events:
 *   pg_ibs_matrix: stage 1 = operand layout, stage 2 = pair kernel;
 *   pg_ld_window:  stage 1 = operand layout and scratch clearing,
 *                  stage 2 = banded pair kernel, 3 = scan, 4 = emit;
 *   pg_ld_prune, pg_grm_matrix, pg_ibs_cluster, pg_batch_launch: as
 *                  documented at each of them.
 * events are hipEvent_t handles created and owned by the caller; they must
 * stay valid while set.  NULL (or n_events = 0) turns recording off.
 * Returns PG_EINVAL for n_events < 0 or > 16.
 */
int pg_profile_events(void* const* events, int n_events);

/* A genotype matrix resident in device memory. */
typedef struct pg_genotypes {
  const uint8_t* bed;          /* variant-major .bed payload (device) */
  int64_t n_samples;           /* samples per variant row, >= 1 */
  int64_t n_variants;          /* rows, >= 1, < 2^31 */
  int64_t bytes_per_variant;   /* row stride in bytes, >= ceil(n_samples/4);
                                  0 means ceil(n_samples/4) */
  const uint64_t* missing_mask;/* optional (NULL = none), device: n_variants
                                  rows of ceil(n_samples/64) uint64; bit k%64 of
                                  word k/64 set => call of sample k is treated
                                  as missing, in addition to code 1 */
} pg_genotypes;

/* IBS output layouts. */
enum pg_layout {
  PG_TRI_UPPER = 0, /* strict upper triangle, row-major: pair (i,j), i<j, at
                       index i*m - i*(i+1)/2 + (j-i-1); m(m-1)/2 entries */
  PG_FULL = 1       /* m x m row-major, both halves and the diagonal */
};
/* Flag OR-ed into the `out_layout` of pg_ibs_matrix (and of an IBS
 * pg_problem): the four count arrays are uint16 instead of uint32 (pass
 * uint16_t arrays through the uint32_t* parameters).  Every count is at most
 * the number of selected variants, so it is allowed only when
 * v_end - v_begin < 65,536 (PG_EINVAL otherwise).  Halves the output: for
 * result copies to the host, as a server sends them. */
#define PG_COUNTS_U16 0x100

/* Kernel path.  The low 8 bits of a `path` argument select the path; bits
 * 8-15 select a kernel variant of that path (0 = the library's default; the
 * tuner tries the others).  Unknown variants fall back to the default. */
enum pg_path {
  PG_PATH_AUTO = 0, /* library picks per shape (pg_resolve_path): the
                       matrix-core path (variant 0), except for LD windows
                       of at least 500 over at least 5,000 samples outside
                       batches, where it is PG_PATH_SPARSE with the sampled
                       gate (variant bit 8): the correction path runs only
                       if the missing calls counted over about 4,096
                       sampled variants average at most its tile budget,
                       and the matrix-core kernel takes every tile
                       otherwise.  Batches resolve AUTO to the matrix-core
                       path. */
  PG_PATH_POPC = 1, /* bit planes + popcount on the vector ALUs */
  PG_PATH_MFMA = 2, /* 2-bit codes expanded to indicator features (values
                       0, +-1) and contracted on the matrix cores.  Default
                       kernels (variant 0): fp4 (e2m1) operands with fp32
                       sums, exact below 2^24 summed terms; beyond that
                       (IBS: 2^24 variants, LD: 2^24 samples) int8 operands
                       with int32 sums.  IBS variants: 1 int8 without
                       scheduling hints, 2 unpipelined reference, 3 fp4
                       unpipelined, 4 fp4 from a replicated operand, 5/6
                       eight waves, 7 int8 pipelined, 8 fp4 pipelined (the
                       default), 9 int8 with hints, unpipelined.  LD
                       variants: 1 the int8 tile.  All give identical
                       counts. */
  PG_PATH_SPARSE = 3 /* LD only: sum x_a x_b on the int8 matrix cores, the
                       other five sums from per-variant totals corrected at
                       the other variant's missing calls (section "Bit
                       population count": without missing calls only
                       sum x_a x_b varies per pair).  A tile of 64 x 64
                       variants runs the PG_PATH_MFMA kernel instead when
                       one of its variants has more missing calls than a
                       list slot holds (max(64, ceil(m/16) rounded up to a
                       multiple of 8), at most 65,528, for m selected
                       samples) or its 128 variants have more than 3m/8 in
                       all, and every tile does unless a quarter of the
                       64-variant groups pass these tests on their own
                       (then the extra sample-major operand pays).  Exact
                       like the other paths; not available in batches.
                       Variant bits: 1 drops the last two rules; 8 adds
                       the sampled gate of PG_PATH_AUTO; 2
                       (pg_ld_window only) is a
                       diagnostic that implies 1: no
                       emission; every pair (a, b) of a tile the path takes
                       (under variant 1's rule) gets the kernel's own record
                       at out[(a - v_begin) * window + (b - a - 1)], other
                       slots are left as they were, capacity must be at
                       least (v_end - v_begin) * window and *n_out receives
                       that product. */
};

/*
 * The kernel path and variant (path | variant << 8) that a call of `kind`
 * (PG_KIND_IBS or PG_KIND_LD) with the given `path` argument runs for m
 * selected samples, nv selected variants and (LD) `window`: PG_PATH_AUTO
 * and variant 0 resolve here exactly as the compute calls resolve them.
 */
int pg_resolve_path(int kind, int64_t m, int64_t nv, int32_t window, int path, int* resolved);

/*
 * Sample selection and variant range (shared by the IBS and LD calls):
 *   sample_idx  optional device int32 array of n_sel indices into
 *               [0, n_samples); output rows/columns follow its order and
 *               duplicates are allowed.  NULL selects all samples in order,
 *               and n_sel must then be 0 or n_samples.  The array lives in
 *               device memory and is not read on the host, so its entries
 *               are not validated: an entry outside [0, n_samples) selects
 *               a sample whose every call is missing (all its counts are 0).
 *   v_begin, v_end  variant range [v_begin, v_end); 0, 0 selects all.
 */

/* Workspace bytes pg_ibs_matrix needs for this shape and path: the operand
 * layout, plus, for the default matrix-core kernel, the raw sums of the
 * variant ranges its tiles are split into (196,608 bytes per tile and
 * range): on cohorts of fewer than 512 tiles of 128 samples every tile is
 * split (at most 2,048 tile ranges); on larger ones only the tiles of the
 * last, partial round of the CUs are (at most 8 x 32 tiles x 8 ranges). */
int pg_ibs_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin, int64_t v_end,
                           int path, size_t* bytes);

/*
 * Identity-by-state matrix over the selected samples (m of them) and
 * variants.  For each output pair (i, j), over the selected variants where
 * neither call is missing:
 *   nonmiss = number of such variants,
 *   ibs2 = same genotype, ibs0 = opposite homozygotes, ibs1 = the rest
 * (ibs0 + ibs1 + ibs2 == nonmiss).  The diagonal of PG_FULL holds
 * ibs2 = nonmiss = the sample's non-missing count, ibs0 = ibs1 = 0.
 * Outputs are four caller-owned uint32 device arrays of m*m (PG_FULL) or
 * m(m-1)/2 (PG_TRI_UPPER) entries (uint16 with PG_COUNTS_U16); counts are
 * exact.  The consumers below (distance, similarity, clustering, IBD report)
 * take the uint32 form.  With zero entries
 * (one sample, PG_TRI_UPPER) the call validates its arguments, enqueues
 * nothing and the output pointers may be NULL.
 * Section "Bitwise parallelism".
 */
int pg_ibs_matrix(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                  int64_t v_begin, int64_t v_end, int out_layout, int path, uint32_t* ibs0,
                  uint32_t* ibs1, uint32_t* ibs2, uint32_t* nonmiss, void* workspace,
                  size_t workspace_bytes, void* stream);

/*
 * pg_ibs_matrix without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, outputs and results are those
 * of pg_ibs_matrix; the scratch space is instead a static device array of
 * PG_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on every device it
 * runs on until the process ends, so the call allocates nothing.  A call
 * whose workspace would exceed it (pg_ibs_workspace_bytes) returns
 * PG_EUNSUPPORTED before enqueueing anything.  Every call on one device uses
 * the same array: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.
 */
#define PG_NOALLOC_SCRATCH_BYTES (64ull << 20)
int pg_ibs_matrix_noalloc(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                          int64_t v_begin, int64_t v_end, int out_layout, int path,
                          uint32_t* ibs0, uint32_t* ibs1, uint32_t* ibs2, uint32_t* nonmiss,
                          void* stream);
/* The static scratch size of pg_ibs_matrix_noalloc, in bytes. */
int pg_noalloc_scratch_bytes(size_t* bytes);

/* One emitted LD pair: 64 bytes. a < b are absolute variant indices. */
typedef struct pg_ld_pair {
  int32_t a, b;
  int64_t n, sx, sy, sxx, syy, sxy;
  double r2;
} pg_ld_pair;

/* Workspace bytes pg_ld_window needs for this shape, window and path. */
int pg_ld_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin, int64_t v_end,
                          int32_t window, int path, size_t* bytes);

/*
 * LD within a window over the selected samples and variants.  For every
 * variant pair a < b <= a + window inside [v_begin, v_end), with x = -1 / 0 /
 * +1 for homozygous A1 / heterozygous / homozygous A2 and S the samples where
 * neither call is missing: n = |S|, sx = sum x_a, sy = sum x_b, sxx = sum x_a^2,
 * syy = sum x_b^2, sxy = sum x_a x_b (exact), and
 *   r2 = c*c / (va*vb),  c = n*sxy - sx*sy, va = n*sxx - sx^2, vb = n*syy - sy^2,
 * evaluated in IEEE double from the exact integers (products, then one
 * division, no contraction), clamped to <= 1; r2 is NaN when n == 0 or
 * va*vb == 0.  This equals the square of r in section "Bit population count"
 * (numerator and denominator multiplied by n^2).
 * A pair is emitted iff r2 >= r2_min (NaN never).  Emitted pairs are written
 * to `out` in increasing (a, b) order; *n_out (device int64) receives the total
 * number of emitted pairs.  If that exceeds `capacity`, only the first
 * `capacity` pairs (in the same order) are written; the call still succeeds,
 * and the caller may retry with a larger buffer.
 * path: PG_PATH_POPC, PG_PATH_MFMA (AUTO) or PG_PATH_SPARSE; all give
 * identical records.
 */
int pg_ld_window(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                 int64_t v_begin, int64_t v_end, int32_t window, double r2_min, pg_ld_pair* out,
                 int64_t capacity, int64_t* n_out, int path, void* workspace,
                 size_t workspace_bytes, void* stream);

/* ---- LD-based pruning ------------------------------------------------------
 *
 * The --indep-pairwise operation (section "Linkage disequilibrium-based
 * variant pruning", timed in Table 4; the paper does not spell out its greedy
 * order, so the order below is this library's reading):
 *  - windows of `window` consecutive selected variants start at 0, step,
 *    2*step, ...; the last window is the first one that reaches the end of
 *    the range;
 *  - inside each window, pairs a < b of variants not yet dropped are visited
 *    in increasing a, then increasing b; when r2 > r2_threshold (r2 exactly as
 *    pg_ld_window defines it; NaN never exceeds), the variant with the lower
 *    minor allele frequency is dropped, and b when the two are equal;
 *  - a dropped variant stays dropped.
 * Minor allele frequency of a variant: min(A2, 2n - A2) / 2n over its n
 * non-missing calls among the selected samples (A2 counts A2 alleles;
 * 0 when n = 0); frequencies are compared exactly, as rationals.
 */

/* Workspace bytes pg_ld_prune needs for this shape, window and path. */
int pg_prune_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin,
                             int64_t v_end, int32_t window, int path, size_t* bytes);

/*
 * Greedy LD pruning over the selected samples and variants.
 *   window        variants per window, 2 <= window <= 65536
 *   step          window shift in variants, 1 <= step <= window
 *   r2_threshold  pairs with r2 strictly above it trigger a drop (not NaN)
 *   keep          device uint8 array of v_end - v_begin flags: 1 = kept,
 *                 0 = dropped; entry v belongs to variant v_begin + v
 *   n_kept        optional device int64: number of kept variants
 *   path          PG_PATH_MFMA, PG_PATH_POPC or PG_PATH_SPARSE selects the
 *                 pair kernels that evaluate r2 (all give identical results)
 * Stages for pg_profile_events: 1 = operand layout and scratch clearing,
 * 2 = banded pair kernel, 3 = allele counts, 4 = greedy pass.
 */
int pg_ld_prune(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                int64_t v_begin, int64_t v_end, int32_t window, int32_t step,
                double r2_threshold, uint8_t* keep, int64_t* n_kept, int path,
                void* workspace, size_t workspace_bytes, void* stream);

/* ---- genomic relationship matrix -----------------------------------------
 *
 * The weighted distance of section "Partial sum lookup", with the GCTA
 * relationship increments the paper gives as its example.  Reading: x = the
 * number of A2 alleles of a call (0, 1, 2) and p = the marker's A2 frequency
 * over its non-missing calls among the selected samples; the increment of a
 * pair of calls is (x - 2p)(y - 2p) / (2p(1-p)) (the paper's major/minor
 * case table gives the same value when x and p count the same allele).  A
 * marker where either call is missing adds nothing and is not counted in the
 * pair's denominator; a marker with no call or with p = 0 or 1 is left out of
 * every pair.  For samples i, j of the selection:
 *   N[i,j] = markers counted,  A[i,j] = (sum of increments) / N[i,j]
 * (NaN when N[i,j] = 0).  The diagonal uses the same increments with i = j.
 * The sums are formed in IEEE double (fp64 matrix cores, increments factored
 * as z_i z_j with z = (x - 2p) / sqrt(2p(1-p))); they match a sequential
 * double sum of the per-pair increments to within the rounding of a length-V
 * double dot product (about V * 2^-53 times the sum of |increments|).
 */

/* Workspace bytes pg_grm_matrix needs for this shape: the operand, the
 * per-marker tables, and, on cohorts of fewer than 512 tiles of 128 samples,
 * the partial sums and counts of the variant ranges each tile is split into
 * (196,608 bytes per tile and range). */
int pg_grm_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin,
                           int64_t v_end, size_t* bytes);

/*
 * Relationship matrix over the selected samples and variants.
 *   out_layout  PG_FULL (m x m, diagonal included) or PG_TRI_UPPER
 *   path        PG_PATH_AUTO or PG_PATH_MFMA (fp64 matrix cores); bits 8-15
 *               select the kernel variant: 0 the library's default (= 2),
 *               1 four waves of 64 x 64 per 128 x 128 tile, 2 eight waves of
 *               32 x 64, 3 sixteen waves of 32 x 32 (all give the same sums)
 *   grm         device double array of the layout's size (A)
 *   n_used      device uint32 array of the same size (N)
 * Stages for pg_profile_events: 1 = operand layout and per-marker tables,
 * 2 = pair kernel.
 */
int pg_grm_matrix(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                  int64_t v_begin, int64_t v_end, int out_layout, int path, double* grm,
                  uint32_t* n_used, void* workspace, size_t workspace_bytes, void* stream);

/* ---- IBS distance and complete-linkage clustering ------------------------
 *
 * Consumers of the IBS counts (section "Identity-by-state matrices, complete
 * linkage clustering"; Table 2 times an IBS matrix followed by clustering).
 * The paper names the statistic but not its formula; the reading here:
 *   d(i,j) = (2*IBS0 + IBS1) / (2*N)
 * the proportion of alleles not shared identical by state over the jointly
 * non-missing markers (one minus the IBS similarity (IBS2 + IBS1/2) / N),
 * computed as the correctly rounded quotient of the two integers; +inf when
 * N = 0.
 */

/* One merge of the clustering: clusters a < b (each indexed by its smallest
 * sample index) merge at complete-linkage distance `height`; the merged
 * cluster keeps index a. */
typedef struct pg_merge {
  int32_t a, b;
  double height;
} pg_merge;

/* Elementwise IBS distance of `count` entries of pg_ibs_matrix output (any
 * layout): dist[e] from ibs0[e], ibs1[e], nonmiss[e].  Device arrays. */
int pg_ibs_distance(const uint32_t* ibs0, const uint32_t* ibs1, const uint32_t* nonmiss,
                    int64_t count, double* dist, void* stream);

/* Workspace bytes pg_ibs_cluster needs for m samples (an m x m double
 * working matrix plus per-sample state). */
int pg_cluster_workspace_bytes(int64_t m, size_t* bytes);

/*
 * Complete-linkage agglomerative clustering of m samples on the IBS
 * distance, from full-layout (m x m) pg_ibs_matrix output.  While more than
 * one cluster remains, the two clusters with the smallest complete-linkage
 * distance (largest member-to-member distance) merge; ties go to the pair
 * with the smallest a, then the smallest b.  merges (device, m - 1 records)
 * receives the merge sequence in order; the result is exactly determined by
 * the counts.  Below 3,200 samples one block runs the merge loop; from
 * 3,200 on, each merge is two kernel launches over the chip (the stream
 * receives 2 (m - 1) launches).  Stages for pg_profile_events: 1 =
 * distances and nearest neighbours, 2 = the merge loop.
 */
int pg_ibs_cluster(const uint32_t* ibs0, const uint32_t* ibs1, const uint32_t* nonmiss,
                   int64_t m, pg_merge* merges, void* workspace, size_t workspace_bytes,
                   void* stream);

/*
 * IBS similarity and the IBD report (--distance ibs and --Z-genome; the
 * paper times the IBD report in Table 2 without giving its formulas).
 *
 * Similarity, elementwise over `count` entries of pg_ibs_matrix output (any
 * layout): sim[e] = (2*IBS2 + IBS1) / (2*N), the correctly rounded quotient
 * of the two integers; NaN when N = 0.  Device arrays.
 */
int pg_ibs_similarity(const uint32_t* ibs1, const uint32_t* ibs2, const uint32_t* nonmiss,
                      int64_t count, double* sim, void* stream);

/* Workspace bytes pg_ibs_genome needs for this selection (sample_idx is not
 * read: only n_sel matters, 0 = all samples). */
int pg_genome_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin,
                              int64_t v_end, size_t* bytes);

/*
 * IBD estimates by the method of moments, from IBS counts over the same
 * samples and variant range (g, sample_idx, n_sel, v_begin, v_end mean what
 * they mean for pg_ibs_matrix and must be the ones the counts came from).
 * Reading:
 *   per marker with n = 2 * (called samples) >= 4 observed alleles, x of
 *   them A2 and y = n - x A1, the IBS probabilities of two samples that
 *   share no allele IBD (four alleles drawn without replacement) or one
 *   (three drawn):
 *     P(IBS0|IBD0) = 2 x(x-1) y(y-1) / [n(n-1)(n-2)(n-3)]
 *     P(IBS1|IBD0) = 4 [x(x-1)(x-2) y + x y(y-1)(y-2)] / [n(n-1)(n-2)(n-3)]
 *     P(IBS1|IBD1) = 2 [x(x-1) y + x y(y-1)] / [n(n-1)(n-2)]
 *   averaged over those markers (E00, E10, E11; the mean is the sum in
 *   increasing marker order divided by their number);
 *   per entry e with N = nonmiss[e] > 0, P0 = ibs0[e]/N, P1 = ibs1[e]/N:
 *     z0 = min(P0 / E00, 1)
 *     z1 = (P1 - z0 E10) / E11, clamped to [0, 1 - z0]
 *     z2 = (1 - z0) - z1,   pi_hat = 0.5 z1 + z2
 *   NaN in all four outputs when N = 0, when no marker has n >= 4, or when
 *   E00 or E11 is zero.
 * Every operation is an IEEE double operation in the order written, so the
 * results are exactly determined by the counts and the genotypes.
 * ibs0, ibs1, nonmiss: `count` entries of pg_ibs_matrix output (any layout);
 * z0, z1, z2, pi_hat: `count` doubles each (device).  Errors: PG_EINVAL for
 * a bad selection or NULL pointer, PG_ENOMEM for a short workspace.
 * Stages for pg_profile_events: 1 = per-marker terms and their averages,
 * 2 = per-pair estimates.
 */
int pg_ibs_genome(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                  int64_t v_begin, int64_t v_end, const uint32_t* ibs0, const uint32_t* ibs1,
                  const uint32_t* nonmiss, int64_t count, double* z0, double* z1, double* z2,
                  double* pi_hat, void* workspace, size_t workspace_bytes, void* stream);

/* ---- diagnostics -----------------------------------------------------------
 *
 * Measured throughput of the units the kernels are bound by, on the current
 * device, as context for the published peaks:
 *   out[0]  int8 matrix cores, TOP/s (v_mfma_i32_32x32x32_i8, 2 ops per MAC)
 *   out[1]  fp64 matrix cores, TFLOP/s (v_mfma_f64_16x16x4_f64)
 *   out[2]  vector popcount-add, T lane-ops/s (v_bcnt_u32_b32)
 *   out[3]  HBM device-to-device copy, GB/s counting bytes read + written
 * Each probe is timed with HIP events on the default stream after a warm-up
 * run; the call returns when all are done.  `workspace` (device) needs at
 * least 4 MiB + 64 MiB; the copy uses the rest of it (split in two halves).
 */
int pg_peak_rates(void* workspace, size_t workspace_bytes, double* out);

/* ---- batching ------------------------------------------------------------
 *
 * Many independent problems (IBS matrices and LD windows over different
 * cohorts, sample lists and ranges) in persistent kernel launches, one per
 * kind of tile body (IBS; LD matrix-core; LD popcount).  Each
 * problem's arguments mean exactly what they mean for pg_ibs_matrix /
 * pg_ld_window, and its outputs are identical to a separate call with the
 * same path.  Kernel variants in a batch: IBS matrix-core problems run the
 * pipelined fp4 tile (the default) or the pipelined int8 tile (variant 7),
 * any other IBS variant runs the default; LD matrix-core problems run the
 * fp4 tile (the default) or the int8 tile (variant 1).  Usage:
 *   pg_batch_plan -> pg_batch_workspace_bytes -> (allocate) -> pg_batch_upload
 *   -> pg_batch_launch (any number of times; or pg_batch_capture once and
 *   pg_graph_launch many times) -> pg_plan_free.
 * Between launches the caller may change the genotype data in place but not
 * any pointer or shape recorded in the plan.  Concurrent launches of one plan
 * on one workspace race.
 */
enum pg_kind { PG_KIND_IBS = 0, PG_KIND_LD = 1 };

typedef struct pg_problem {
  int kind;                     /* PG_KIND_IBS or PG_KIND_LD */
  int path;                     /* as the `path` of the one-problem calls */
  pg_genotypes g;
  const int32_t* sample_idx;    /* selection, as for the one-problem calls */
  int64_t n_sel;
  int64_t v_begin, v_end;
  /* IBS outputs */
  int out_layout;
  uint32_t *ibs0, *ibs1, *ibs2, *nonmiss;
  /* LD arguments and outputs */
  int32_t window;
  double r2_min;
  pg_ld_pair* out;
  int64_t capacity;
  int64_t* n_out;
} pg_problem;

typedef struct pg_plan pg_plan;   /* host-side plan; owns no device memory */

/* Validates the problems (any failure names the problem) and builds the
 * schedule: the tiles of all problems in one list, grouped by tile body and
 * with the longest tiles first within a group.  *plan must be released with
 * pg_plan_free. */
int pg_batch_plan(const pg_problem* probs, int n_probs, pg_plan** plan);
/* Device workspace the plan needs: every problem's operand layout and LD
 * scratch, the tile table and the tile counter. */
int pg_batch_workspace_bytes(const pg_plan* plan, size_t* bytes);
/* Number of tiles in the list and the largest persistent grid size
 * (informational). */
int pg_batch_tiles(const pg_plan* plan, int64_t* total_tiles, int* grid);
/* Writes the tile table into `workspace` (a host-to-device copy on `stream`,
 * waited for before returning) and creates the plan's second stream and two
 * events (default priority; released by pg_plan_free).  Launches must use
 * this same workspace. */
int pg_batch_upload(pg_plan* plan, void* workspace, size_t workspace_bytes, void* stream);
/* Enqueues the whole batch behind the work already on `stream`, in two
 * concurrent branches: the IBS problems (layouts, persistent kernel) on
 * `stream`, the LD problems (layouts, persistent kernels, scans and emits)
 * on the plan's second stream, joined back into `stream` before the call's
 * work counts as done there.  Kernels and event waits only, so it may be
 * captured into a HIP graph.  Stage events (pg_profile_events, on `stream`):
 * 1 = the IBS branch done, 2 = both branches done. */
int pg_batch_launch(const pg_plan* plan, void* workspace, size_t workspace_bytes, void* stream);
void pg_plan_free(pg_plan* plan);

/* Captures pg_batch_launch into an instantiated HIP graph (*graph_exec is a
 * hipGraphExec_t).  `stream` must not be the default stream. */
int pg_batch_capture(const pg_plan* plan, void* workspace, size_t workspace_bytes, void* stream,
                     void** graph_exec);
/* Replays a captured graph on `stream`. */
int pg_graph_launch(void* graph_exec, void* stream);
/* Releases a captured graph (NULL is ignored). */
int pg_graph_destroy(void* graph_exec);

#ifdef __cplusplus
}
#endif

#endif /* PG_H */
