// Batched execution: many independent IBS and LD problems in at most three
// persistent launches, one per kind of tile body.
//
// A plan validates every problem exactly as the one-problem entry points do,
// carves one workspace into per-problem operands and LD scratch, and orders
// the problems by part (IBS, LD matrix-core, LD popcount), longest tile first
// within each part, so that the tiles of all problems form one global list.
// A launch enqueues two branches that run concurrently: on the caller's
// stream the IBS problems' operand layouts, a reset of their tile counter
// and the IBS persistent kernel; on a stream of the plan's own (forked from
// the caller's with an event and joined back with another) the LD problems'
// layouts and scratch clearing, their tile counters, the LD persistent
// kernels and every LD problem's scan and emit.  A persistent kernel's
// blocks take tiles of their part with an atomic counter until the part is
// exhausted, so as one branch's tiles run out its CUs go to the other
// branch's blocks, and neither part's tail leaves the GPU idle.  The tile
// bodies are the same device functions the one-problem kernels run, so
// results are identical to calling pg_ibs_matrix / pg_ld_window per problem.
// The sequence contains kernels and event waits only (no memset or copy
// nodes), so it can be captured into a HIP graph and replayed.
#include <algorithm>
#include <new>
#include <vector>

#include "tiles.h"

namespace pg {

// Device descriptor of one problem, in schedule order.
struct BatchItem {
  int32_t kind;          // PG_KIND_IBS / PG_KIND_LD
  int32_t path;          // PG_PATH_MFMA / PG_PATH_POPC (resolved)
  int32_t variant;
  int32_t window;
  int64_t tile_begin;    // first global tile index
  int64_t ntiles;
  const uint32_t* X;     // operand layout in the workspace
  int64_t words;         // K words of the operand
  int64_t rows_pad;
  int64_t nt;            // IBS: tiles per side; LD: row tiles
  int64_t n_band;        // LD: column tiles per row tile
  int64_t nv;            // LD: selected variants
  double r2_min;
  IbsOut o;
  LdScratch sc;
};

// The global tile list in three parts, one persistent kernel each, so that
// every tile body runs at its own occupancy: IBS tiles (both paths) at one
// block per CU (the matrix-core tile's register budget), then LD matrix-core
// tiles, then LD popcount tiles.
enum { kPartIbs = 0, kPartLdMfma = 1, kPartLdPopc = 2, kParts = 3 };
constexpr int kCounters = 8 + kParts - 1;   // 8 XCD runs of the IBS part, one per LD part

__host__ __device__ inline int batch_part(int kind, int path) {
  return kind == PG_KIND_IBS ? kPartIbs : path == PG_PATH_MFMA ? kPartLdMfma : kPartLdPopc;
}

// Persistent loop over the tiles [t_begin, t_end) of the global list: every
// block takes tiles from `counter` until the range is used up.  The IBS part
// is XCD-aware, as the one-problem launch is: its range is cut into 8
// contiguous runs with a counter each (counter[0..7]), block b takes tiles
// from run b % 8 (the XCD it runs on) and, once that run is used up, from
// the other runs in turn; within a problem the tiles go in the banded order
// (valid_band_tile), so the tiles one XCD runs together share operand rows
// in its L2.
template <int kPart>
__global__ __launch_bounds__(256, kPart == kPartIbs ? 1 : 2) void k_batch_persistent(
    const BatchItem* __restrict__ items, int n_items, int64_t t_begin, int64_t t_end,
    unsigned long long* counter) {
  constexpr int kSmem = kPart == kPartIbs
                            ? (kIbsMfmaSmem > kIbsPopcSmem ? kIbsMfmaSmem : kIbsPopcSmem)
                            : kPart == kPartLdMfma ? kLdMfmaSmem : kLdPopcSmem;
  __shared__ __attribute__((aligned(16))) uint32_t smem[kSmem];
  __shared__ int64_t s_tile;
  const int xcd = (int)(blockIdx.x % 8);
  unsigned used = 0;   // IBS: runs found used up (thread 0 only)
  for (;;) {
    if (threadIdx.x == 0) {
      if constexpr (kPart == kPartIbs) {
        const int64_t n = t_end - t_begin;
        int64_t got = t_end;
        for (int k = 0; k < 8; ++k) {
          const int y = (xcd + k) & 7;
          if (used & (1u << y)) continue;
          const int64_t v = t_begin + n * y / 8 + (int64_t)atomicAdd(&counter[y], 1ull);
          if (v < t_begin + n * (y + 1) / 8) {
            got = v;
            break;
          }
          used |= 1u << y;
        }
        s_tile = got;
      } else {
        s_tile = t_begin + (int64_t)atomicAdd(counter, 1ull);
      }
    }
    __syncthreads();
    const int64_t t = s_tile;
    __syncthreads();
    if (t >= t_end) break;   // block-uniform: every block leaves once the range is used up
    int lo = 0, hi = n_items;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (items[mid].tile_begin <= t) lo = mid; else hi = mid;
    }
    const BatchItem& it = items[lo];
    const int64_t local = t - it.tile_begin;
    if constexpr (kPart == kPartIbs) {
      int64_t I, J;
      valid_band_tile(local, it.nt, I, J);
      if (it.path == PG_PATH_MFMA) {
        if (it.variant == kIbsVariantFp4Pipe)
          ibs_fp4_tile_pipe(it.X, it.words, I, J, it.o, (lds_t*)smem);
        else
          ibs_mfma_tile_pipe<true>(it.X, it.words, I, J, it.o, (lds_t*)smem);
      } else {
        ibs_popc_tile(it.X, it.rows_pad, it.words, I, J, it.o, (lds_t*)smem);
      }
    } else {
      const int64_t I = local / it.n_band;
      const int64_t J = I + local % it.n_band;
      if (J < it.nt) {
        if constexpr (kPart == kPartLdMfma) {
          if (it.variant == kLdVariantFp4)
            ld_fp4_tile_pipe(it.X, it.words, it.nv, I, J, it.window, it.r2_min, it.sc,
                             (lds_t*)smem);
          else
            ld_mfma_tile(it.X, it.words, it.nv, I, J, it.window, it.r2_min, it.sc, (lds_t*)smem);
        } else {
          ld_popc_tile(it.X, it.words, it.nv, it.rows_pad, I, J, it.window, it.r2_min, it.sc,
                       (lds_t*)smem);
        }
      }
    }
    __syncthreads();   // LDS is reused by the next tile
  }
}

}  // namespace pg

// ---- host side -------------------------------------------------------------------

using namespace pg;

namespace {

constexpr int64_t kAlign = 256;

int64_t take(int64_t& off, int64_t bytes) {
  const int64_t o = off;
  off = round_up(off + bytes, kAlign);
  return o;
}

struct ProblemPlan {
  pg_problem p;
  Sel s;
  int path, variant;
  int64_t rows_pad, words, nt, n_band, bm_words;
  int64_t off_x, off_bm, off_cnt, off_off, off_bsum;
  int64_t ntiles;
  double tile_cost;
};

}  // namespace

struct pg_plan {
  std::vector<ProblemPlan> probs;
  std::vector<int> order;          // schedule order (indices into probs), by part
  int64_t total_tiles = 0;
  int64_t part_begin[kParts + 1] = {0, 0, 0, 0};   // tile range of each part
  int64_t off_items = 0, off_counter = 0, bytes = 0;
  // the sample-major layouts of the matrix-core IBS problems without a
  // sample list run as one launch (LayoutJob table at off_jobs)
  int64_t off_jobs = 0, job_blocks = 0;
  int n_jobs = 0;
  int grid[kParts] = {256, 256, 256};
  const void* uploaded_ws = nullptr;
  // the LD branch runs on a stream of the plan's own, forked from and
  // joined back into the caller's stream with two events
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  ~pg_plan() {
    if (join) (void)hipEventDestroy(join);
    if (fork) (void)hipEventDestroy(fork);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace pg {
// Defined in abi.hip: the same validation as the one-problem entry points.
int batch_validate_ibs(const pg_problem& p, Sel& s, int& path, int& variant, int64_t& rows_pad,
                       int64_t& words);
int batch_validate_ld(const pg_problem& p, Sel& s, int& path, int& variant, int64_t& rows_pad,
                      int64_t& words, int64_t& bm_words);
}  // namespace pg

extern "C" {

int pg_batch_plan(const pg_problem* probs, int n_probs, pg_plan** out) {
  if (!out) return fail(PG_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (!probs || n_probs < 1) return fail(PG_EINVAL, "no problems");
  pg_plan* plan = new (std::nothrow) pg_plan;
  if (!plan) return fail(PG_EINVAL, "host allocation failed");
  int64_t off = 0;
  for (int i = 0; i < n_probs; ++i) {
    ProblemPlan q{};
    q.p = probs[i];
    int rc;
    if (q.p.kind == PG_KIND_IBS) {
      rc = batch_validate_ibs(q.p, q.s, q.path, q.variant, q.rows_pad, q.words);
      // the persistent kernel hosts the two pipelined matrix-core bodies
      // (fp4, the default; int8, variant 7, also the default where fp4 sums
      // could reach 2^24); every other matrix-core variant gives the same
      // counts and runs the default body, since hosting more bodies would
      // raise the kernel's register and LDS budget for every tile
      if (rc == PG_OK && q.path == PG_PATH_MFMA && q.variant != kIbsVariantPipe) {
        IbsPlan dflt;
        rc = plan_ibs_default(q.s, dflt);
        q.variant = dflt.variant;
        q.rows_pad = dflt.rows_pad;
        q.words = dflt.words;
      }
      if (rc == PG_OK) {
        const int tile = q.path == PG_PATH_MFMA ? kIbsMfmaTile : kIbsPopcTile;
        q.nt = q.rows_pad / tile;
        q.ntiles = q.nt * (q.nt + 1) / 2;
        const int64_t bytes = q.path == PG_PATH_MFMA ? q.rows_pad * q.words * 4
                                                     : 3 * q.rows_pad * q.words * 4;
        q.off_x = take(off, bytes);
        // rough cycles per tile, for longest-first ordering
        q.tile_cost = q.path != PG_PATH_MFMA ? (double)q.words * 520.0
                      : (double)q.words * (q.variant == kIbsVariantFp4Pipe ? 310.0 : 440.0);
      }
    } else if (q.p.kind == PG_KIND_LD) {
      rc = batch_validate_ld(q.p, q.s, q.path, q.variant, q.rows_pad, q.words, q.bm_words);
      if (rc == PG_OK) {
        q.nt = q.rows_pad / kLdTile;
        q.n_band = ((int64_t)q.p.window + kLdTile - 1) / kLdTile + 1;
        q.ntiles = q.nt * q.n_band;
        const int64_t bytes = q.path == PG_PATH_MFMA ? q.rows_pad * q.words * 4
                                                     : 3 * q.rows_pad * q.words * 4;
        q.off_x = take(off, bytes);
        q.off_bm = take(off, q.rows_pad * q.bm_words * 4);
        q.off_cnt = take(off, q.rows_pad * 4);
        q.off_off = take(off, (q.rows_pad + 1) * 8);
        q.off_bsum = take(off, (int64_t)ld_scan_blocks(q.rows_pad) * 8);
        q.tile_cost = q.path == PG_PATH_MFMA ? (double)q.words * 172.0 : (double)q.words * 1024.0;
      }
    } else {
      rc = fail(PG_EINVAL, "problem %d: unknown kind %d", i, q.p.kind);
    }
    if (rc != PG_OK) {
      delete plan;
      return fail(rc, "problem %d: %s", i, pg_last_error());
    }
    plan->probs.push_back(q);
  }
  plan->order.resize(n_probs);
  for (int i = 0; i < n_probs; ++i) plan->order[i] = i;
  // by part (IBS, LD matrix-core, LD popcount), longest tiles first within one
  auto part = [&](int k) { return batch_part(plan->probs[k].p.kind, plan->probs[k].path); };
  std::stable_sort(plan->order.begin(), plan->order.end(), [&](int a, int b) {
    if (part(a) != part(b)) return part(a) < part(b);
    return plan->probs[a].tile_cost > plan->probs[b].tile_cost;
  });
  int64_t tiles[kParts] = {0, 0, 0};
  for (int k : plan->order) tiles[part(k)] += plan->probs[k].ntiles;
  for (int q = 0; q < kParts; ++q) plan->part_begin[q + 1] = plan->part_begin[q] + tiles[q];
  const int64_t t = plan->part_begin[kParts];
  plan->total_tiles = t;
  plan->off_items = take(off, (int64_t)sizeof(BatchItem) * n_probs);
  for (int k : plan->order) {
    const ProblemPlan& q = plan->probs[k];
    if (q.p.kind == PG_KIND_IBS && q.path == PG_PATH_MFMA && !q.s.idx) {
      ++plan->n_jobs;
      plan->job_blocks += sample_major_job_blocks(q.rows_pad, q.words);
    }
  }
  plan->off_jobs = take(off, (int64_t)sizeof(LayoutJob) * std::max(plan->n_jobs, 1));
  plan->off_counter = take(off, 8 * kCounters);   // tile counters: 8 (IBS) + 2 (LD)
  plan->bytes = off;
  // persistent grids: resident blocks of each kernel on this device
  auto resident = [](const void* kernel, int64_t tiles) {
    int dev = 0, cus = 0, per_cu = 0;
    int64_t g = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) == hipSuccess &&
        cus > 0 && per_cu > 0) {
      g = (int64_t)cus * per_cu;
    } else {
      (void)hipGetLastError();
    }
    return (int)std::max<int64_t>(std::min<int64_t>(g, tiles), 1);
  };
  plan->grid[kPartIbs] = resident((const void*)k_batch_persistent<kPartIbs>, tiles[kPartIbs]);
  plan->grid[kPartLdMfma] =
      resident((const void*)k_batch_persistent<kPartLdMfma>, tiles[kPartLdMfma]);
  plan->grid[kPartLdPopc] =
      resident((const void*)k_batch_persistent<kPartLdPopc>, tiles[kPartLdPopc]);
  *out = plan;
  return PG_OK;
}

int pg_batch_workspace_bytes(const pg_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(PG_EINVAL, "NULL argument");
  *bytes = (size_t)plan->bytes;
  return PG_OK;
}

int pg_batch_tiles(const pg_plan* plan, int64_t* total_tiles, int* grid) {
  if (!plan) return fail(PG_EINVAL, "plan is NULL");
  if (total_tiles) *total_tiles = plan->total_tiles;
  if (grid) {
    *grid = 0;   // blocks of the largest persistent launch
    for (int q = 0; q < kParts; ++q)
      if (plan->part_begin[q + 1] > plan->part_begin[q]) *grid = std::max(*grid, plan->grid[q]);
  }
  return PG_OK;
}

int pg_batch_upload(pg_plan* plan, void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan || !workspace) return fail(PG_EINVAL, "NULL argument");
  if ((int64_t)workspace_bytes < plan->bytes)
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)plan->bytes);
  char* ws = (char*)workspace;
  std::vector<BatchItem> items;
  int64_t t = 0;
  for (int k : plan->order) {
    const ProblemPlan& q = plan->probs[k];
    BatchItem it{};
    it.kind = q.p.kind;
    it.path = q.path;
    it.variant = q.variant;
    it.tile_begin = t;
    it.ntiles = q.ntiles;
    it.X = (const uint32_t*)(ws + q.off_x);
    it.words = q.words;
    it.rows_pad = q.rows_pad;
    it.nt = q.nt;
    if (q.p.kind == PG_KIND_IBS) {
      it.o = IbsOut{q.p.ibs0, q.p.ibs1, q.p.ibs2, q.p.nonmiss, q.s.m,
                    (q.p.out_layout & ~PG_COUNTS_U16) == PG_FULL,
                    (q.p.out_layout & PG_COUNTS_U16) ? 1 : 0};
    } else {
      it.window = q.p.window;
      it.n_band = q.n_band;
      it.nv = q.s.nv;
      it.r2_min = q.p.r2_min;
      it.sc = LdScratch{(uint32_t*)(ws + q.off_bm), q.bm_words, (uint32_t*)(ws + q.off_cnt),
                        (int64_t*)(ws + q.off_off), (int64_t*)(ws + q.off_bsum)};
    }
    items.push_back(it);
    t += q.ntiles;
  }
  std::vector<LayoutJob> jobs;
  int64_t jb = 0;
  for (int k : plan->order) {
    const ProblemPlan& q = plan->probs[k];
    if (!(q.p.kind == PG_KIND_IBS && q.path == PG_PATH_MFMA && !q.s.idx)) continue;
    LayoutJob j{};
    j.s = q.s;
    j.T = (uint32_t*)(ws + q.off_x);
    j.rows_pad = q.rows_pad;
    j.wp = q.words;
    j.block_begin = jb;
    j.aligned = rows_dword_aligned(q.s) ? 1 : 0;
    jobs.push_back(j);
    jb += sample_major_job_blocks(q.rows_pad, q.words);
  }
  hipStream_t st = (hipStream_t)stream;
  if (!plan->side &&
      (hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&plan->fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&plan->join, hipEventDisableTiming) != hipSuccess))
    return fail(PG_EDEVICE, "batch stream and events: %s", hipGetErrorString(hipGetLastError()));
  if (hipMemcpyAsync(ws + plan->off_items, items.data(), sizeof(BatchItem) * items.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      (!jobs.empty() &&
       hipMemcpyAsync(ws + plan->off_jobs, jobs.data(), sizeof(LayoutJob) * jobs.size(),
                      hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(PG_EDEVICE, "tile table upload failed: %s", hipGetErrorString(hipGetLastError()));
  plan->uploaded_ws = workspace;
  return PG_OK;
}

int pg_batch_launch(const pg_plan* plan, void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan || !workspace) return fail(PG_EINVAL, "NULL argument");
  if ((int64_t)workspace_bytes < plan->bytes)
    return fail(PG_ENOMEM, "workspace of %llu bytes < %lld required",
                (unsigned long long)workspace_bytes, (long long)plan->bytes);
  if (plan->uploaded_ws != workspace)
    return fail(PG_EINVAL, "workspace differs from the one given to pg_batch_upload");
  hipStream_t st = (hipStream_t)stream;
  hipStream_t side = plan->side;
  char* ws = (char*)workspace;
  int rc = PG_OK;
  mark_stage(0, st);
  // fork: the LD branch waits for everything before this call on `st`
  if (hipEventRecord(plan->fork, st) != hipSuccess ||
      hipStreamWaitEvent(side, plan->fork, 0) != hipSuccess)
    return fail(PG_EDEVICE, "batch fork: %s", hipGetErrorString(hipGetLastError()));
  unsigned long long* counter = (unsigned long long*)(ws + plan->off_counter);
  const BatchItem* items = (const BatchItem*)(ws + plan->off_items);
  const int n_items = (int)plan->probs.size();
  const int64_t* pb = plan->part_begin;
  // IBS branch on `st`: layouts (one launch for the jobs), the tile counter,
  // the persistent kernel
  rc = launch_sample_major_jobs((const LayoutJob*)(ws + plan->off_jobs), plan->n_jobs,
                                plan->job_blocks, st);
  if (rc != PG_OK) return rc;
  for (int k : plan->order) {
    const ProblemPlan& q = plan->probs[k];
    if (q.p.kind != PG_KIND_IBS) continue;
    if (q.path == PG_PATH_MFMA && !q.s.idx) continue;   // a layout job
    uint32_t* X = (uint32_t*)(ws + q.off_x);
    rc = q.path == PG_PATH_MFMA ? launch_sample_major_2bit(q.s, X, q.rows_pad, q.words, st)
                                : launch_ibs_planes(q.s, X, q.rows_pad, q.words, st);
    if (rc != PG_OK) return rc;
  }
  if (pb[1] > pb[0]) {
    rc = fill_u32((uint32_t*)counter, 16, 0u, st);
    if (rc != PG_OK) return rc;
    hipLaunchKernelGGL(k_batch_persistent<kPartIbs>, dim3((unsigned)plan->grid[kPartIbs]),
                       dim3(256), 0, st, items, n_items, pb[0], pb[1], counter);
    rc = check_launch("batch_persistent_ibs");
    if (rc != PG_OK) return rc;
  }
  mark_stage(1, st);
  // LD branch on `side`: layouts and scratch clearing, the tile counters,
  // the persistent kernels, the scans and emits
  for (int k : plan->order) {
    const ProblemPlan& q = plan->probs[k];
    if (q.p.kind != PG_KIND_LD) continue;
    uint32_t* X = (uint32_t*)(ws + q.off_x);
    rc = q.path == PG_PATH_MFMA ? launch_variant_major_2bit(q.s, X, q.rows_pad, q.words, side)
                                : launch_ld_planes(q.s, X, q.rows_pad, q.words, side);
    const LdScratch sc{(uint32_t*)(ws + q.off_bm), q.bm_words, (uint32_t*)(ws + q.off_cnt),
                       (int64_t*)(ws + q.off_off), (int64_t*)(ws + q.off_bsum)};
    if (rc == PG_OK) rc = ld_clear(sc, q.rows_pad, side);
    if (rc != PG_OK) return rc;
  }
  if (pb[3] > pb[1]) {
    rc = fill_u32((uint32_t*)(counter + 8), 2 * (kParts - 1), 0u, side);
    if (rc != PG_OK) return rc;
  }
  if (pb[2] > pb[1])
    hipLaunchKernelGGL(k_batch_persistent<kPartLdMfma>, dim3((unsigned)plan->grid[kPartLdMfma]),
                       dim3(256), 0, side, items, n_items, pb[1], pb[2], counter + 8);
  if (pb[3] > pb[2])
    hipLaunchKernelGGL(k_batch_persistent<kPartLdPopc>, dim3((unsigned)plan->grid[kPartLdPopc]),
                       dim3(256), 0, side, items, n_items, pb[2], pb[3], counter + 9);
  rc = check_launch("batch_persistent_ld");
  if (rc != PG_OK) return rc;
  for (int k : plan->order) {
    const ProblemPlan& q = plan->probs[k];
    if (q.p.kind != PG_KIND_LD) continue;
    const LdScratch sc{(uint32_t*)(ws + q.off_bm), q.bm_words, (uint32_t*)(ws + q.off_cnt),
                       (int64_t*)(ws + q.off_off), (int64_t*)(ws + q.off_bsum)};
    rc = launch_ld_finish((uint32_t*)(ws + q.off_x), q.path == PG_PATH_POPC, q.words, q.rows_pad,
                          q.s.nv, q.s.v0, sc, q.p.out, q.p.capacity, q.p.n_out, side, false);
    if (rc != PG_OK) return rc;
  }
  // join: `st` continues once the LD branch is done
  if (hipEventRecord(plan->join, side) != hipSuccess ||
      hipStreamWaitEvent(st, plan->join, 0) != hipSuccess)
    return fail(PG_EDEVICE, "batch join: %s", hipGetErrorString(hipGetLastError()));
  mark_stage(2, st);
  return PG_OK;
}

void pg_plan_free(pg_plan* plan) { delete plan; }

int pg_batch_capture(const pg_plan* plan, void* workspace, size_t workspace_bytes, void* stream,
                     void** graph_exec) {
  if (!graph_exec) return fail(PG_EINVAL, "graph_exec is NULL");
  *graph_exec = nullptr;
  if (!stream) return fail(PG_EINVAL, "capture needs a non-default stream");
  hipStream_t st = (hipStream_t)stream;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(PG_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(hipGetLastError()));
  const int rc = pg_batch_launch(plan, workspace, workspace_bytes, stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &graph);
  if (rc != PG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess || !graph) return fail(PG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(PG_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  *graph_exec = (void*)exec;
  return PG_OK;
}

int pg_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return fail(PG_EINVAL, "graph_exec is NULL");
  const hipError_t e = hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(PG_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
  return PG_OK;
}

int pg_graph_destroy(void* graph_exec) {
  if (!graph_exec) return PG_OK;
  const hipError_t e = hipGraphExecDestroy((hipGraphExec_t)graph_exec);
  if (e != hipSuccess) return fail(PG_EDEVICE, "hipGraphExecDestroy: %s", hipGetErrorString(e));
  return PG_OK;
}

}  // extern "C"
