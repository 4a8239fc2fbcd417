// C ABI of libpg.so: argument validation, workspace carving and dispatch.
// Every check runs on the host before any launch; see include/pg.h for the
// contract of each entry point.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "pg_internal.h"

namespace pg {

static thread_local char g_last_error[512] = "";

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return status;
}

static thread_local hipEvent_t g_events[16];
static thread_local int g_n_events = 0;

void mark_stage(int k, hipStream_t st) {
  if (k < g_n_events && g_events[k]) (void)hipEventRecord(g_events[k], st);
}

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return PG_OK;
}

// ---- static scratch of pg_ibs_matrix_noalloc ----------------------------------
// One array per device, held until the process ends.  In host code its name
// is only a stand-in: kernels get the device address hipGetSymbolAddress
// returns for the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(PG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(PG_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PG_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return PG_OK;
}

namespace {

constexpr int64_t kAlign = 256;
constexpr int64_t kMaxIndex = (int64_t)1 << 31;

struct Carve {
  int64_t off = 0;
  int64_t take(int64_t bytes) {
    const int64_t o = off;
    off = round_up(off + bytes, kAlign);
    return o;
  }
};

// Validates the matrix, the selection and the range; fills `s`.
// `list` says whether a sample list is given (the workspace queries pass no
// pointer, only its length).
int make_sel(const pg_genotypes* g, bool list, const int32_t* idx, int64_t n_sel,
             int64_t v_begin, int64_t v_end, Sel& s) {
  if (!g) return fail(PG_EINVAL, "genotypes is NULL");
  if (!g->bed) return fail(PG_EINVAL, "bed is NULL");
  if (g->n_samples < 1 || g->n_samples >= kMaxIndex)
    return fail(PG_EINVAL, "n_samples %lld outside [1, 2^31)", (long long)g->n_samples);
  if (g->n_variants < 1 || g->n_variants >= kMaxIndex)
    return fail(PG_EINVAL, "n_variants %lld outside [1, 2^31)", (long long)g->n_variants);
  const int64_t min_bpv = ceil_div(g->n_samples, 4);
  const int64_t bpv = g->bytes_per_variant == 0 ? min_bpv : g->bytes_per_variant;
  if (bpv < min_bpv)
    return fail(PG_EINVAL, "bytes_per_variant %lld < ceil(n_samples/4) = %lld",
                (long long)bpv, (long long)min_bpv);
  int64_t m = g->n_samples;
  if (list) {
    if (n_sel < 1 || n_sel >= kMaxIndex)
      return fail(PG_EINVAL, "n_sel %lld outside [1, 2^31) with a sample list", (long long)n_sel);
    m = n_sel;
  } else if (n_sel != 0 && n_sel != g->n_samples) {
    return fail(PG_EINVAL, "n_sel must be 0 or n_samples without a sample list");
  }
  int64_t vb = v_begin, ve = v_end;
  if (vb == 0 && ve == 0) ve = g->n_variants;
  if (vb < 0 || ve > g->n_variants || vb >= ve)
    return fail(PG_EINVAL, "variant range [%lld, %lld) invalid for %lld variants", (long long)vb,
                (long long)ve, (long long)g->n_variants);
  s.bed = g->bed;
  s.bpv = bpv;
  s.mask = g->missing_mask;
  s.wpm = ceil_div(g->n_samples, 64);
  s.idx = idx;
  s.n = g->n_samples;
  s.m = m;
  s.v0 = vb;
  s.nv = ve - vb;
  return PG_OK;
}


// PG_PATH_AUTO.  Measured whole-call times (the sweep mode of bench.py):
// the pipelined fp4 matrix-core kernel wins every IBS shape of 64 to 10,000
// samples x 5,000 to 100,000 variants, the popcount kernel coming closest
// at 64 samples (0.087 vs 0.081 ms).  For LD the missing-call correction
// path wins on data with few missing calls from 5,000 samples and windows
// of 500 (up to 1.52x at 20,000 samples, window 1,000) and the dense fp4
// kernel everywhere else, so the missing rate decides: there AUTO takes the
// correction path behind a sampled gate (kLdGated) that counts the missing
// calls of about 4,096 variants and leaves the path off, for the cost of
// that count, unless a tile would hold few enough of them on average.
int ibs_auto_path(int64_t m, int64_t nv) {
  (void)m;
  (void)nv;
  return PG_PATH_MFMA;
}

int ld_auto_path(int64_t m, int64_t nv, int32_t window) {
  (void)nv;
  return m >= 5000 && window >= 500 ? PG_PATH_SPARSE : PG_PATH_MFMA;
}

// Variant bits of the correction path: every tile whose lists fit (1), the
// diagnostic records (2, implies 1), the sampled gate (8; what AUTO sets).
constexpr int kLdAllTiles = 1, kLdDiag = 2, kLdGated = 8;
constexpr int64_t kLdGateSamples = 4096;   // variants the gate samples (about)

// Resolves the kernel variant: 0 (or an undefined code) is the default, the
// pipelined fp4 kernel; fp4 variants fall back to the pipelined int8 kernel
// when a sum could reach 2^24.
int resolve_ibs_variant(int variant, int64_t nv) {
  if (variant <= 0 || variant >= kIbsVariants) variant = kIbsVariantFp4Pipe;
  const bool fp4 = variant == kIbsVariantFp4 || variant == kIbsVariantFp4Rep ||
                   variant == kIbsVariantFp4Pipe;
  if (fp4 && nv >= kFp4MaxVariants) variant = kIbsVariantPipe;
  return variant;
}

int plan_ibs(const Sel& s, int path_arg, IbsPlan& p) {
  int path = path_arg & 0xFF;
  if (path_arg < 0 || (path_arg >> 16) != 0) return fail(PG_EINVAL, "bad path argument %d", path_arg);
  if (path == PG_PATH_AUTO) path = ibs_auto_path(s.m, s.nv);
  if (path != PG_PATH_MFMA && path != PG_PATH_POPC)
    return fail(PG_EINVAL, "unknown path %d", path);
  p.path = path;
  p.variant = path == PG_PATH_MFMA ? resolve_ibs_variant((path_arg >> 8) & 0xFF, s.nv)
                                   : (path_arg >> 8) & 0xFF;
  if (path == PG_PATH_MFMA && p.variant == kIbsVariantFp4Rep) {
    p.rows_pad = round_up(s.m, kIbsMfmaTile);
    p.words = round_up(s.nv, 4 * kIbsRepChunk) / 4;     // 2 words per 8 variants
    p.bytes = p.rows_pad * p.words * 4;
  } else if (path == PG_PATH_MFMA) {
    p.rows_pad = round_up(s.m, kIbsMfmaTile);
    p.words = round_up(ceil_div(s.nv, 16), kIbsMfmaKWords);
    p.bytes = p.rows_pad * p.words * 4;
  } else {
    p.rows_pad = round_up(s.m, kIbsPopcTile);
    p.words = round_up(ceil_div(s.nv, 32), kIbsPopcKWords);
    p.bytes = 3 * p.rows_pad * p.words * 4;
  }
  const int64_t nt = p.rows_pad / (path == PG_PATH_MFMA ? kIbsMfmaTile : kIbsPopcTile);
  if (nt * (nt + 1) / 2 + 2 * nt >= kMaxIndex) return fail(PG_EUNSUPPORTED, "too many samples for one call");
  p.off_part = -1;
  // the pipelined kernels split small cohorts' K range (ibs_split)
  const bool pipelined = path == PG_PATH_MFMA &&
      (p.variant == kIbsVariantPipe || p.variant == kIbsVariantFp4Pipe);
  if (pipelined && ibs_part_bytes(p.rows_pad, p.words) > 0) {
    p.off_part = round_up(p.bytes, 256);
    p.bytes = p.off_part + ibs_part_bytes(p.rows_pad, p.words);
  }
  return PG_OK;
}

struct LdPlan {
  int path, variant;
  int64_t rows_pad, words, bm_words;
  int64_t off_D, off_bm, off_cnt, off_off, off_bsum, bytes;
  // correction path: sample-major operand (t_rows x t_words), lists, stats
  int64_t t_rows, t_words, off_T, off_lists, off_vst, off_gsum, off_gmax, off_any;
  int cap;
};

int plan_ld(const Sel& s, int32_t window, int path_arg, LdPlan& p) {
  if (window < 1) return fail(PG_EINVAL, "window %d < 1", (int)window);
  if (path_arg < 0 || (path_arg >> 16) != 0) return fail(PG_EINVAL, "bad path argument %d", path_arg);
  int path = path_arg & 0xFF;
  p.variant = (path_arg >> 8) & 0xFF;
  if (path == PG_PATH_AUTO) {
    path = ld_auto_path(s.m, s.nv, window);
    if (path == PG_PATH_SPARSE) p.variant |= kLdGated;
  }
  if (path != PG_PATH_MFMA && path != PG_PATH_POPC && path != PG_PATH_SPARSE)
    return fail(PG_EINVAL, "unknown path %d", path);
  p.path = path;
  // matrix-core kernel: fp4 by default (exact below 2^24 samples), int8 as
  // variant 1 or beyond that
  if (path == PG_PATH_MFMA && (p.variant != kLdVariantInt8 && s.m < kFp4MaxVariants))
    p.variant = kLdVariantFp4;
  else if (path == PG_PATH_MFMA)
    p.variant = kLdVariantInt8;
  p.rows_pad = round_up(s.nv, kLdTile);
  p.bm_words = ceil_div(window, 32);
  int64_t operand_bytes;
  if (path == PG_PATH_MFMA || path == PG_PATH_SPARSE) {
    p.words = round_up(ceil_div(s.m, 16), kLdKWords);
    operand_bytes = p.rows_pad * p.words * 4;
  } else {
    p.words = round_up(ceil_div(s.m, 32), kLdPopcKWords);
    operand_bytes = 3 * p.words * p.rows_pad * 4;
  }
  Carve c;
  p.off_D = c.take(operand_bytes);
  p.off_bm = c.take(p.rows_pad * p.bm_words * 4);
  p.off_cnt = c.take(p.rows_pad * 4);
  p.off_off = c.take((p.rows_pad + 1) * 8);
  p.off_bsum = c.take((int64_t)ld_scan_blocks(p.rows_pad) * 8);
  if (path == PG_PATH_SPARSE) {
    p.t_rows = round_up(s.m, kIbsMfmaTile);
    p.t_words = round_up(ceil_div(s.nv, 16), kIbsMfmaKWords);
    p.cap = ld_sparse_cap(s.m);
    p.off_T = c.take(p.t_rows * p.t_words * 4);
    p.off_lists = c.take(p.rows_pad * p.cap * 4);
    p.off_vst = c.take(p.rows_pad * 16);
    p.off_gsum = c.take(p.rows_pad / kLdTile * 8);
    p.off_gmax = c.take(p.rows_pad / kLdTile * 4);
    p.off_any = c.take(16);   // groups_ok, then the gate's 64-bit count at +8
  }
  p.bytes = c.off;
  return PG_OK;
}


// Band tiles take the correction path when their two 64-variant groups hold
// at most 3m/8 missing calls (m selected samples), and only once a quarter
// of the groups have a diagonal tile that does, so that the sample-major
// operand is worth building.  Measured on 5,000 samples x 500,000 variants,
// window 1,000, every tile forced onto the correction kernel: 4.1 ms without
// missing calls, 5.4 ms at 0.25% (0.32m per tile), 6.1 ms at 0.5% (0.64m),
// 7.3 ms at 1%, against 6.1-6.2 ms for the pipelined fp4 dense kernel.  Per
// tile the two cost the same near 0.6m; the rule stops at 3m/8 so that the
// tiles' savings also pay for building T and the longer statistics pass
// (0.7 ms together at this size).
int64_t ld_sparse_budget(const LdPlan& p, int64_t m) {
  return p.variant & (kLdAllTiles | kLdDiag) ? INT64_MAX : 3 * m / 8;
}
uint32_t ld_sparse_min_groups(const LdPlan& p) {
  const int64_t g = p.rows_pad / kLdTile;
  return p.variant & (kLdAllTiles | kLdDiag) ? 1u : (uint32_t)(g < 4 ? 1 : g / 4);
}

// Operand layouts and the pair kernels of an LD plan, up to the emission
// bitmap (stage events 1 and 2).
int ld_pairs(const Sel& s, const LdPlan& p, char* ws, int32_t window, double r2_min,
             const LdScratch& sc, hipStream_t st, pg_ld_pair* dbg = nullptr) {
  uint32_t* D = (uint32_t*)(ws + p.off_D);
  int rc;
  if (p.path == PG_PATH_POPC) {
    rc = launch_ld_planes(s, D, p.rows_pad, p.words, st);
    if (rc == PG_OK) rc = ld_clear(sc, p.rows_pad, st);
    mark_stage(1, st);
    if (rc != PG_OK) return rc;
    return launch_ld_popc(D, p.words, s.nv, p.rows_pad, window, r2_min, sc, st);
  }
  rc = launch_variant_major_2bit(s, D, p.rows_pad, p.words, st);
  if (rc == PG_OK) rc = ld_clear(sc, p.rows_pad, st);
  if (p.path == PG_PATH_MFMA) {
    mark_stage(1, st);
    if (rc != PG_OK) return rc;
    return launch_ld_mfma(D, p.words, s.nv, p.rows_pad, window, r2_min, sc, st, nullptr,
                          p.variant == kLdVariantFp4);
  }
  LdSparse sp{(uint32_t*)(ws + p.off_lists), (int4*)(ws + p.off_vst), (int64_t*)(ws + p.off_gsum),
              (int*)(ws + p.off_gmax), (uint32_t*)(ws + p.off_any), ld_sparse_min_groups(p),
              p.cap, ld_sparse_budget(p, s.m), nullptr, 0, 1};
  if (p.variant & kLdGated) {
    // on when the sampled variants' mean, times the 128 variants of a tile,
    // is within the tile budget: count <= budget * n_samp / 128
    sp.gate = (uint64_t*)(ws + p.off_any + 8);
    sp.gate_stride = s.nv > kLdGateSamples ? s.nv / kLdGateSamples : 1;
    const int64_t n_samp = ceil_div(s.nv, sp.gate_stride);
    sp.gate_max = sp.budget == INT64_MAX
                      ? UINT64_MAX
                      : (uint64_t)(sp.budget / (2 * kLdTile) * n_samp +
                                   sp.budget % (2 * kLdTile) * n_samp / (2 * kLdTile));
  }
  uint32_t* T = (uint32_t*)(ws + p.off_T);
  if (rc == PG_OK) rc = launch_ld_sparse_stats(D, p.words, s.m, s.nv, p.rows_pad, sp, st);
  // the sample-major operand only when the path is on
  if (rc == PG_OK) rc = launch_ld_transpose(D, p.rows_pad, p.words, T, p.t_rows, p.t_words, sp, st);
  mark_stage(1, st);
  if (rc != PG_OK) return rc;
  return launch_ld_sparse(D, p.words, T, p.t_rows, s.m, s.nv, p.rows_pad, window, r2_min, sc, sp,
                          st, dbg, s.v0);
}

struct PrunePlan {
  LdPlan ld;
  int64_t off_stats, off_drop, count_cells, off_cc, bytes;
};

// The LD plan for the pair kernel (largest distance window - 1) plus the
// per-variant allele counts.
int plan_prune(const Sel& s, int32_t window, int32_t step, int path_arg, PrunePlan& p) {
  if (window < 2 || window > kPruneMaxWindow)
    return fail(PG_EINVAL, "window %d outside [2, %lld]", (int)window, (long long)kPruneMaxWindow);
  if (step < 1 || step > window) return fail(PG_EINVAL, "step %d outside [1, window]", (int)step);
  int rc = plan_ld(s, window - 1, path_arg, p.ld);
  if (rc != PG_OK) return rc;
  Carve c;
  c.off = p.ld.bytes;
  p.off_stats = c.take(p.ld.rows_pad * (int64_t)sizeof(int2));
  p.off_drop = c.take(p.ld.rows_pad * p.ld.bm_words * 4);
  p.count_cells = prune_count_capacity(s.nv, window);   // independent of step
  p.off_cc = c.take(p.count_cells * 2);
  p.bytes = c.off;
  return PG_OK;
}

struct GrmPlan {
  int64_t rows_pad, words;
  int64_t off_T, off_z, off_used, off_part, bytes;
};

int plan_grm(const Sel& s, GrmPlan& p) {
  p.rows_pad = round_up(s.m, 128);
  p.words = round_up(ceil_div(s.nv, 16), 16);
  const int64_t nt = p.rows_pad / 128;
  if (nt * (nt + 1) / 2 >= kMaxIndex) return fail(PG_EUNSUPPORTED, "too many samples for one call");
  Carve c;
  p.off_T = c.take(p.rows_pad * p.words * 4);
  p.off_z = c.take(p.words * 16 * 4 * 8);
  p.off_used = c.take(p.words * 4);
  p.off_part = c.take(grm_part_bytes(p.rows_pad, p.words));
  p.bytes = c.off;
  return PG_OK;
}

}  // namespace

int plan_ibs_default(const Sel& s, IbsPlan& p) { return plan_ibs(s, PG_PATH_MFMA, p); }

int ibs_out_layout(int out_layout, int64_t nv, int& layout, int& u16) {
  layout = out_layout & ~PG_COUNTS_U16;
  u16 = (out_layout & PG_COUNTS_U16) ? 1 : 0;
  if (layout != PG_FULL && layout != PG_TRI_UPPER)
    return fail(PG_EINVAL, "unknown layout %d", out_layout);
  if (u16 && nv >= 65536)
    return fail(PG_EINVAL, "16-bit counts need fewer than 65,536 variants (%lld selected)",
                (long long)nv);
  return PG_OK;
}

int batch_validate_ibs(const pg_problem& q, Sel& s, int& path, int& variant, int64_t& rows_pad,
                       int64_t& words) {
  int rc = make_sel(&q.g, q.sample_idx != nullptr, q.sample_idx, q.n_sel, q.v_begin, q.v_end, s);
  if (rc != PG_OK) return rc;
  int layout, u16;
  rc = ibs_out_layout(q.out_layout, s.nv, layout, u16);
  if (rc != PG_OK) return rc;
  const int64_t entries = layout == PG_FULL ? s.m * s.m : s.m * (s.m - 1) / 2;
  if (entries > 0 && (!q.ibs0 || !q.ibs1 || !q.ibs2 || !q.nonmiss))
    return fail(PG_EINVAL, "an output pointer is NULL");
  IbsPlan p;
  rc = plan_ibs(s, q.path, p);
  if (rc != PG_OK) return rc;
  path = p.path;
  variant = p.variant;
  rows_pad = p.rows_pad;
  words = p.words;
  return PG_OK;
}

int batch_validate_ld(const pg_problem& q, Sel& s, int& path, int& variant, int64_t& rows_pad,
                      int64_t& words, int64_t& bm_words) {
  int rc = make_sel(&q.g, q.sample_idx != nullptr, q.sample_idx, q.n_sel, q.v_begin, q.v_end, s);
  if (rc != PG_OK) return rc;
  if (!q.n_out) return fail(PG_EINVAL, "n_out is NULL");
  if (q.capacity < 0) return fail(PG_EINVAL, "capacity < 0");
  if (q.capacity > 0 && !q.out) return fail(PG_EINVAL, "out is NULL with capacity > 0");
  LdPlan p;
  // AUTO in a batch: the matrix-core path (the correction path is not hosted)
  const int path_arg = (q.path & 0xFF) == PG_PATH_AUTO ? (q.path & ~0xFF) | PG_PATH_MFMA : q.path;
  rc = plan_ld(s, q.window, path_arg, p);
  if (rc != PG_OK) return rc;
  if (p.path == PG_PATH_SPARSE)
    return fail(PG_EUNSUPPORTED, "the missing-call correction path is not available in batches");
  path = p.path;
  variant = p.variant;
  rows_pad = p.rows_pad;
  words = p.words;
  bm_words = p.bm_words;
  return PG_OK;
}

}  // namespace pg

using namespace pg;

extern "C" {

const char* pg_status_str(int status) {
  switch (status) {
    case PG_OK: return "ok";
    case PG_EINVAL: return "invalid argument";
    case PG_ENOMEM: return "workspace too small";
    case PG_EDEVICE: return "device error";
    case PG_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* pg_last_error(void) { return g_last_error; }

int pg_version(void) { return PG_VERSION; }

int pg_profile_events(void* const* events, int n_events) {
  if (n_events < 0 || n_events > 16) return fail(PG_EINVAL, "n_events %d outside [0, 16]", n_events);
  g_n_events = events ? n_events : 0;
  for (int k = 0; k < g_n_events; ++k) g_events[k] = (hipEvent_t)events[k];
  return PG_OK;
}

int pg_ibs_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin, int64_t v_end,
                           int path, size_t* bytes) {
  if (!bytes) return fail(PG_EINVAL, "bytes is NULL");
  Sel s;
  int rc = make_sel(g, n_sel > 0, nullptr, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  IbsPlan p;
  rc = plan_ibs(s, path, p);
  if (rc != PG_OK) return rc;
  *bytes = (size_t)p.bytes;
  return PG_OK;
}

}  // extern "C"

namespace {

// Body of pg_ibs_matrix and pg_ibs_matrix_noalloc: `workspace` is the
// caller's buffer or the library's static scratch array.
int ibs_matrix_run(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                   int64_t v_begin, int64_t v_end, int out_layout, int path, uint32_t* ibs0,
                   uint32_t* ibs1, uint32_t* ibs2, uint32_t* nonmiss, void* workspace,
                   size_t workspace_bytes, void* stream, bool noalloc) {
  g_last_error[0] = 0;
  Sel s;
  int rc = make_sel(g, sample_idx != nullptr, sample_idx, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  int layout, u16;
  rc = ibs_out_layout(out_layout, s.nv, layout, u16);
  if (rc != PG_OK) return rc;
  const int64_t entries = layout == PG_FULL ? s.m * s.m : s.m * (s.m - 1) / 2;
  if (entries == 0) return PG_OK;  // one sample, triangle layout: nothing to write
  if (!ibs0 || !ibs1 || !ibs2 || !nonmiss) return fail(PG_EINVAL, "an output pointer is NULL");
  IbsPlan p;
  rc = plan_ibs(s, path, p);
  if (rc != PG_OK) return rc;
  if (noalloc) {
    // without room for the K split's sums, the unsplit kernel (same sums)
    if (p.bytes > kNoAllocScratchBytes && p.off_part >= 0 && p.off_part <= kNoAllocScratchBytes) {
      p.bytes = p.off_part;
      p.off_part = -1;
    }
    if (p.bytes > kNoAllocScratchBytes)
      return fail(PG_EUNSUPPORTED,
                  "pg_ibs_matrix_noalloc: %lld scratch bytes needed for %lld samples x %lld "
                  "variants, more than the static array's %lld; call pg_ibs_matrix with a "
                  "workspace instead",
                  (long long)p.bytes, (long long)s.m, (long long)s.nv,
                  (long long)kNoAllocScratchBytes);
    rc = noalloc_scratch(&workspace);
    if (rc != PG_OK) return rc;
    workspace_bytes = (size_t)kNoAllocScratchBytes;
  }
  if ((int64_t)workspace_bytes < p.bytes || (!workspace && p.bytes > 0))
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)p.bytes);
  hipStream_t st = (hipStream_t)stream;
  IbsOut o{ibs0, ibs1, ibs2, nonmiss, s.m, layout == PG_FULL, u16};
  uint32_t* ws = (uint32_t*)workspace;
  mark_stage(0, st);
  if (p.path == PG_PATH_MFMA && p.variant == kIbsVariantFp4Rep) {
    rc = launch_sample_major_rep(s, ws, p.rows_pad, p.words, st);
    mark_stage(1, st);
    if (rc == PG_OK) rc = launch_ibs_fp4rep(ws, p.words, o, st);
  } else if (p.path == PG_PATH_MFMA) {
    rc = launch_sample_major_2bit(s, ws, p.rows_pad, p.words, st);
    mark_stage(1, st);
    int32_t* part = p.off_part >= 0 ? (int32_t*)((char*)workspace + p.off_part) : nullptr;
    if (rc == PG_OK) rc = launch_ibs_mfma(ws, p.words, o, p.variant, st, part);
  } else {
    rc = launch_ibs_planes(s, ws, p.rows_pad, p.words, st);
    mark_stage(1, st);
    if (rc == PG_OK) rc = launch_ibs_popc(ws, p.rows_pad, p.words, o, st);
  }
  mark_stage(2, st);
  return rc;
}

}  // namespace

extern "C" {

int pg_ibs_matrix(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                  int64_t v_begin, int64_t v_end, int out_layout, int path, uint32_t* ibs0,
                  uint32_t* ibs1, uint32_t* ibs2, uint32_t* nonmiss, void* workspace,
                  size_t workspace_bytes, void* stream) {
  return ibs_matrix_run(g, sample_idx, n_sel, v_begin, v_end, out_layout, path, ibs0, ibs1, ibs2,
                        nonmiss, workspace, workspace_bytes, stream, false);
}

int pg_ibs_matrix_noalloc(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                          int64_t v_begin, int64_t v_end, int out_layout, int path,
                          uint32_t* ibs0, uint32_t* ibs1, uint32_t* ibs2, uint32_t* nonmiss,
                          void* stream) {
  return ibs_matrix_run(g, sample_idx, n_sel, v_begin, v_end, out_layout, path, ibs0, ibs1, ibs2,
                        nonmiss, nullptr, 0, stream, true);
}

int pg_noalloc_scratch_bytes(size_t* bytes) {
  if (!bytes) return fail(PG_EINVAL, "bytes is NULL");
  *bytes = (size_t)kNoAllocScratchBytes;
  return PG_OK;
}

int pg_resolve_path(int kind, int64_t m, int64_t nv, int32_t window, int path, int* resolved) {
  if (!resolved) return fail(PG_EINVAL, "resolved is NULL");
  if (m < 1 || m >= kMaxIndex || nv < 1 || nv >= kMaxIndex)
    return fail(PG_EINVAL, "m %lld / nv %lld outside [1, 2^31)", (long long)m, (long long)nv);
  Sel s{};
  s.n = s.m = m;
  s.nv = nv;
  int rc;
  if (kind == PG_KIND_IBS) {
    IbsPlan p;
    rc = plan_ibs(s, path, p);
    if (rc == PG_OK) *resolved = p.path | (p.variant << 8);
  } else if (kind == PG_KIND_LD) {
    LdPlan p;
    rc = plan_ld(s, window, path, p);
    if (rc == PG_OK) *resolved = p.path | (p.variant << 8);
  } else {
    rc = fail(PG_EINVAL, "unknown kind %d", kind);
  }
  return rc;
}

int pg_ld_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin, int64_t v_end,
                          int32_t window, int path, size_t* bytes) {
  if (!bytes) return fail(PG_EINVAL, "bytes is NULL");
  Sel s;
  int rc = make_sel(g, n_sel > 0, nullptr, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  LdPlan p;
  rc = plan_ld(s, window, path, p);
  if (rc != PG_OK) return rc;
  *bytes = (size_t)p.bytes;
  return PG_OK;
}

int pg_ld_window(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                 int64_t v_begin, int64_t v_end, int32_t window, double r2_min, pg_ld_pair* out,
                 int64_t capacity, int64_t* n_out, int path, void* workspace,
                 size_t workspace_bytes, void* stream) {
  g_last_error[0] = 0;
  Sel s;
  int rc = make_sel(g, sample_idx != nullptr, sample_idx, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  if (!n_out) return fail(PG_EINVAL, "n_out is NULL");
  if (capacity < 0) return fail(PG_EINVAL, "capacity < 0");
  if (capacity > 0 && !out) return fail(PG_EINVAL, "out is NULL with capacity > 0");
  LdPlan p;
  rc = plan_ld(s, window, path, p);
  if (rc != PG_OK) return rc;
  if ((int64_t)workspace_bytes < p.bytes || !workspace)
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)p.bytes);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  uint32_t* D = (uint32_t*)(ws + p.off_D);
  LdScratch sc{(uint32_t*)(ws + p.off_bm), p.bm_words, (uint32_t*)(ws + p.off_cnt),
               (int64_t*)(ws + p.off_off), (int64_t*)(ws + p.off_bsum)};
  mark_stage(0, st);
  if (p.path == PG_PATH_SPARSE && (p.variant & kLdDiag)) {
    // diagnostic: the correction kernel's own record of every pair it takes
    const int64_t slots = s.nv * (int64_t)window;
    if (capacity < slots)
      return fail(PG_EINVAL, "capacity %lld < %lld slots of the diagnostic variant",
                  (long long)capacity, (long long)slots);
    rc = ld_pairs(s, p, ws, window, r2_min, sc, st, out);
    if (rc == PG_OK) rc = fill_u32((uint32_t*)n_out, 1, (uint32_t)(slots & 0xFFFFFFFF), st);
    if (rc == PG_OK) rc = fill_u32((uint32_t*)n_out + 1, 1, (uint32_t)(slots >> 32), st);
    return rc;
  }
  rc = ld_pairs(s, p, ws, window, r2_min, sc, st);
  if (rc == PG_OK)
    rc = launch_ld_finish(D, p.path == PG_PATH_POPC, p.words, p.rows_pad, s.nv, s.v0, sc, out,
                          capacity, n_out, st);
  return rc;
}

int pg_prune_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin,
                             int64_t v_end, int32_t window, int path, size_t* bytes) {
  g_last_error[0] = 0;
  if (!bytes) return fail(PG_EINVAL, "bytes is NULL");
  Sel s;
  int rc = make_sel(g, n_sel > 0, nullptr, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  PrunePlan p;
  rc = plan_prune(s, window, window, path, p);
  if (rc != PG_OK) return rc;
  *bytes = (size_t)p.bytes;
  return PG_OK;
}

int pg_ld_prune(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                int64_t v_begin, int64_t v_end, int32_t window, int32_t step,
                double r2_threshold, uint8_t* keep, int64_t* n_kept, int path, void* workspace,
                size_t workspace_bytes, void* stream) {
  g_last_error[0] = 0;
  Sel s;
  int rc = make_sel(g, sample_idx != nullptr, sample_idx, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  if (!keep) return fail(PG_EINVAL, "keep is NULL");
  if (r2_threshold != r2_threshold) return fail(PG_EINVAL, "r2_threshold is NaN");
  PrunePlan p;
  rc = plan_prune(s, window, step, path, p);
  if (rc != PG_OK) return rc;
  if (p.ld.path == PG_PATH_SPARSE && (p.ld.variant & kLdDiag))
    return fail(PG_EINVAL, "variant 2 of the correction path is a pg_ld_window diagnostic");
  if ((int64_t)workspace_bytes < p.bytes || !workspace)
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)p.bytes);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const LdPlan& q = p.ld;
  uint32_t* D = (uint32_t*)(ws + q.off_D);
  LdScratch sc{(uint32_t*)(ws + q.off_bm), q.bm_words, (uint32_t*)(ws + q.off_cnt),
               (int64_t*)(ws + q.off_off), (int64_t*)(ws + q.off_bsum)};
  int2* stats = (int2*)(ws + p.off_stats);
  const bool planes = q.path == PG_PATH_POPC;
  // r2 > t  <=>  r2 >= the next double above t
  const double r2_min = nextafter(r2_threshold, INFINITY);
  mark_stage(0, st);
  rc = ld_pairs(s, q, ws, window - 1, r2_min, sc, st);
  if (rc == PG_OK) rc = launch_variant_stats(D, planes, q.words, q.rows_pad, s.nv, stats, st);
  mark_stage(3, st);
  if (rc == PG_OK)
    rc = launch_prune_greedy(sc, stats, (uint32_t*)(ws + p.off_drop), (uint16_t*)(ws + p.off_cc),
                             p.count_cells, s.nv, window, step, keep, n_kept, st);
  mark_stage(4, st);
  return rc;
}

int pg_grm_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin, int64_t v_end,
                           size_t* bytes) {
  g_last_error[0] = 0;
  if (!bytes) return fail(PG_EINVAL, "bytes is NULL");
  Sel s;
  int rc = make_sel(g, n_sel > 0, nullptr, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  GrmPlan p;
  rc = plan_grm(s, p);
  if (rc != PG_OK) return rc;
  *bytes = (size_t)p.bytes;
  return PG_OK;
}

int pg_grm_matrix(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                  int64_t v_begin, int64_t v_end, int out_layout, int path, double* grm,
                  uint32_t* n_used, void* workspace, size_t workspace_bytes, void* stream) {
  g_last_error[0] = 0;
  Sel s;
  int rc = make_sel(g, sample_idx != nullptr, sample_idx, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  if (out_layout != PG_FULL && out_layout != PG_TRI_UPPER)
    return fail(PG_EINVAL, "unknown layout %d", out_layout);
  if (path < 0 || (path >> 16) != 0 ||
      ((path & 0xFF) != PG_PATH_AUTO && (path & 0xFF) != PG_PATH_MFMA))
    return fail(PG_EINVAL, "bad path argument %d", path);
  const int variant = (path >> 8) & 0xFF;
  const int64_t entries = out_layout == PG_FULL ? s.m * s.m : s.m * (s.m - 1) / 2;
  if (entries > 0 && (!grm || !n_used)) return fail(PG_EINVAL, "an output pointer is NULL");
  GrmPlan p;
  rc = plan_grm(s, p);
  if (rc != PG_OK) return rc;
  if (entries == 0) return PG_OK;
  if ((int64_t)workspace_bytes < p.bytes || !workspace)
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)p.bytes);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  uint32_t* T = (uint32_t*)(ws + p.off_T);
  mark_stage(0, st);
  rc = launch_sample_major_2bit(s, T, p.rows_pad, p.words, st);
  if (rc == PG_OK)
    rc = launch_grm(s, T, p.rows_pad, p.words, (double*)(ws + p.off_z),
                    (uint32_t*)(ws + p.off_used), (double*)(ws + p.off_part), grm, n_used,
                    out_layout == PG_FULL, variant == 1 ? 4 : variant == 3 ? 16 : 8, st);
  return rc;
}

int pg_ibs_distance(const uint32_t* ibs0, const uint32_t* ibs1, const uint32_t* nonmiss,
                    int64_t count, double* dist, void* stream) {
  g_last_error[0] = 0;
  if (count < 0) return fail(PG_EINVAL, "count < 0");
  if (count > 0 && (!ibs0 || !ibs1 || !nonmiss || !dist))
    return fail(PG_EINVAL, "an input or output pointer is NULL");
  return launch_ibs_distance(ibs0, ibs1, nonmiss, count, dist, (hipStream_t)stream);
}

int pg_ibs_similarity(const uint32_t* ibs1, const uint32_t* ibs2, const uint32_t* nonmiss,
                      int64_t count, double* sim, void* stream) {
  g_last_error[0] = 0;
  if (count < 0) return fail(PG_EINVAL, "count < 0");
  if (count > 0 && (!ibs1 || !ibs2 || !nonmiss || !sim))
    return fail(PG_EINVAL, "an input or output pointer is NULL");
  return launch_ibs_similarity(ibs1, ibs2, nonmiss, count, sim, (hipStream_t)stream);
}

namespace {
// Variant-major operand of the selection (rows_pad x wn words), the five
// per-marker term columns, the per-marker flags, the six sums and the runs'
// partial sums.
struct GenomePlan {
  int64_t rows_pad, wn, off_D, off_terms, off_used, off_sums, bytes;
};
void plan_genome(const Sel& s, GenomePlan& p) {
  p.rows_pad = round_up(s.nv, 64);
  p.wn = ceil_div(s.m, 16);
  Carve c;
  p.off_D = c.take(p.rows_pad * p.wn * 4);
  p.off_terms = c.take(5 * p.rows_pad * 8);
  p.off_used = c.take(p.rows_pad * 4);
  p.off_sums = c.take(8 * genome_sums_doubles(s.nv));
  p.bytes = c.off;
}
}  // namespace

int pg_genome_workspace_bytes(const pg_genotypes* g, int64_t n_sel, int64_t v_begin,
                              int64_t v_end, size_t* bytes) {
  g_last_error[0] = 0;
  if (!bytes) return fail(PG_EINVAL, "bytes is NULL");
  Sel s;
  const int rc = make_sel(g, n_sel > 0, nullptr, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  GenomePlan p;
  plan_genome(s, p);
  *bytes = (size_t)p.bytes;
  return PG_OK;
}

int pg_ibs_genome(const pg_genotypes* g, const int32_t* sample_idx, int64_t n_sel,
                  int64_t v_begin, int64_t v_end, const uint32_t* ibs0, const uint32_t* ibs1,
                  const uint32_t* nonmiss, int64_t count, double* z0, double* z1, double* z2,
                  double* pi_hat, void* workspace, size_t workspace_bytes, void* stream) {
  g_last_error[0] = 0;
  Sel s;
  int rc = make_sel(g, sample_idx != nullptr, sample_idx, n_sel, v_begin, v_end, s);
  if (rc != PG_OK) return rc;
  if (count < 0) return fail(PG_EINVAL, "count < 0");
  if (count > 0 && (!ibs0 || !ibs1 || !nonmiss || !z0 || !z1 || !z2 || !pi_hat))
    return fail(PG_EINVAL, "an input or output pointer is NULL");
  GenomePlan p;
  plan_genome(s, p);
  if ((int64_t)workspace_bytes < p.bytes || !workspace)
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)p.bytes);
  char* ws = (char*)workspace;
  hipStream_t st = (hipStream_t)stream;
  mark_stage(0, st);
  uint32_t* D = (uint32_t*)(ws + p.off_D);
  rc = launch_variant_major_2bit(s, D, p.rows_pad, p.wn, st);
  if (rc != PG_OK) return rc;
  rc = launch_genome(D, p.wn, s.nv, p.rows_pad, (double*)(ws + p.off_terms),
                     (uint32_t*)(ws + p.off_used), (double*)(ws + p.off_sums), ibs0, ibs1,
                     nonmiss, count, z0, z1, z2, pi_hat, st);
  if (rc == PG_OK) mark_stage(2, st);
  return rc;
}

namespace {
struct ClusterPlan {
  int64_t off_D, off_nnd, off_nnj, off_ctl, off_rows, bytes;
};
int plan_cluster(int64_t m, ClusterPlan& p) {
  if (m < 1 || m >= kMaxIndex) return fail(PG_EINVAL, "m %lld outside [1, 2^31)", (long long)m);
  Carve c;
  p.off_D = c.take(m * m * 8);
  p.off_nnd = c.take(m * 8);
  p.off_nnj = c.take(m * 4);
  p.off_ctl = c.take(16);
  p.off_rows = c.take(m * 4);
  p.bytes = c.off;
  return PG_OK;
}
}  // namespace

int pg_cluster_workspace_bytes(int64_t m, size_t* bytes) {
  g_last_error[0] = 0;
  if (!bytes) return fail(PG_EINVAL, "bytes is NULL");
  ClusterPlan p;
  const int rc = plan_cluster(m, p);
  if (rc != PG_OK) return rc;
  *bytes = (size_t)p.bytes;
  return PG_OK;
}

int pg_ibs_cluster(const uint32_t* ibs0, const uint32_t* ibs1, const uint32_t* nonmiss,
                   int64_t m, pg_merge* merges, void* workspace, size_t workspace_bytes,
                   void* stream) {
  g_last_error[0] = 0;
  ClusterPlan p;
  int rc = plan_cluster(m, p);
  if (rc != PG_OK) return rc;
  if (!ibs0 || !ibs1 || !nonmiss) return fail(PG_EINVAL, "an input pointer is NULL");
  if (m > 1 && !merges) return fail(PG_EINVAL, "merges is NULL");
  if ((int64_t)workspace_bytes < p.bytes || !workspace)
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)p.bytes);
  char* ws = (char*)workspace;
  hipStream_t st = (hipStream_t)stream;
  mark_stage(0, st);
  return launch_ibs_cluster(ibs0, ibs1, nonmiss, m, (double*)(ws + p.off_D),
                            (double*)(ws + p.off_nnd), (int*)(ws + p.off_nnj),
                            (int*)(ws + p.off_ctl), (int*)(ws + p.off_rows), merges, st);
}

}  // extern "C"
