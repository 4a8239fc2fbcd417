// Measured throughput of the units the library's kernels are bound by, for
// roofline context next to the published peaks: int8 and fp64 matrix cores,
// the vector ALU's popcount-add, and an HBM copy.  Each probe keeps every
// SIMD busy with independent work and no memory traffic (the copy aside).
#include "tiles.h"

namespace pg {

typedef double peak_d4 __attribute__((ext_vector_type(4)));

// 8 waves per block (two per SIMD), 8 independent 32x32x32 int8 MFMA chains
// per wave.
__global__ __launch_bounds__(512, 1) void k_peak_i8(int iters, int* out) {
  v16i acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = (v16i){0};
  const v4i a = {(int)threadIdx.x, 1, 2, 3}, b = {3, 2, 1, (int)threadIdx.x};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[i], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][15];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8 waves per block, 16 independent 16x16x4 fp64 MFMA chains per wave.
__global__ __launch_bounds__(512, 1) void k_peak_f64(int iters, double* out) {
  peak_d4 acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = peak_d4{0.0, 0.0, 0.0, 0.0};
  const double a = threadIdx.x * 1e-3, b = 1.0 + threadIdx.x * 1e-4;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8 independent popcount-add chains per thread (v_bcnt_u32_b32).
__global__ __launch_bounds__(256) void k_peak_bcnt(int iters, uint32_t* out) {
  uint32_t c[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) c[i] = threadIdx.x * 0x9e3779b9u + i * 0x85ebca6bu;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = __builtin_popcount(c[i]) + c[i];   // one v_bcnt_u32_b32
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += c[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Copy with four 16-byte loads in flight per thread before their stores, a
// block moving 4 x 256 consecutive vectors per step, and nontemporal hints
// (the data is touched once).  One load in flight per thread measured
// 4.8 TB/s read + written on MI355X, this form 5.9 TB/s.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_peak_copy(const v4u* __restrict__ src,
                                                   v4u* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256 * 4;
  for (int64_t base = (int64_t)blockIdx.x * 256 * 4; base < n; base += stride) {
    v4u v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = base + u * 256 + threadIdx.x;
      if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = base + u * 256 + threadIdx.x;
      if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
}

}  // namespace pg

extern "C" {

int pg_peak_rates(void* workspace, size_t workspace_bytes, double* out) {
  using namespace pg;
  if (!out) return fail(PG_EINVAL, "out is NULL");
  const size_t scratch = (size_t)1024 * 512 * 8;
  if (!workspace || workspace_bytes < scratch + ((size_t)64 << 20))
    return fail(PG_ENOMEM, "workspace of %llu bytes < %llu required",
                (unsigned long long)workspace_bytes,
                (unsigned long long)(scratch + ((size_t)64 << 20)));
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(PG_EDEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PG_EDEVICE, "hipEventCreate failed");
  }
  char* ws = (char*)workspace;
  const int blocks = 1024;   // 4 blocks per CU on 256 CUs
  int rc = PG_OK;
  auto timed = [&](auto launch, double work, double unit, double* dst) {
    if (rc != PG_OK) return;
    launch();   // warm-up
    (void)hipEventRecord(e0, 0);
    launch();
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(PG_EDEVICE, "peak probe failed: %s", hipGetErrorString(hipGetLastError()));
      return;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *dst = work / (ms * 1e-3) / unit;
  };
  const int it_i8 = 4000, it_f64 = 1000, it_pc = 20000;
  timed([&] { hipLaunchKernelGGL(k_peak_i8, dim3(blocks), dim3(512), 0, 0, it_i8, (int*)ws); },
        (double)blocks * 8 * it_i8 * 8 * (32.0 * 32 * 32 * 2), 1e12, &out[0]);
  timed([&] { hipLaunchKernelGGL(k_peak_f64, dim3(blocks), dim3(512), 0, 0, it_f64, (double*)ws); },
        (double)blocks * 8 * it_f64 * 16 * (16.0 * 16 * 4 * 2), 1e12, &out[1]);
  timed([&] {
    hipLaunchKernelGGL(k_peak_bcnt, dim3(blocks * 4), dim3(256), 0, 0, it_pc, (uint32_t*)ws);
  }, (double)blocks * 4 * 256 * it_pc * 8, 1e12, &out[2]);
  const int64_t half = (int64_t)((workspace_bytes - scratch) / 2 / 16);
  const v4u* src = (const v4u*)(ws + scratch);
  v4u* dst = (v4u*)(ws + scratch) + half;
  timed([&] {
    hipLaunchKernelGGL(k_peak_copy, dim3(8192), dim3(256), 0, 0, src, dst, half);
  }, (double)half * 16 * 2, 1e9, &out[3]);
  if (rc == PG_OK) rc = check_launch("peak probes");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
