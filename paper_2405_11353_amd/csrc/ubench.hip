// Microbenchmarks that fix the gfx950 roofline used by the NTT kernels:
// issue rate of the 32-bit integer multiply forms the 64-bit modular
// multiply is built from, the 64-bit add/compare forms, and HBM copy
// bandwidth. Pure VALU inline asm (no memory ops in asm); each wave keeps
// 8 independent dependency chains so the measurement is issue-bound.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#define CHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { \
  fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); return -1; } } while (0)

enum { OP_ADD_U32, OP_MUL_LO_U32, OP_MUL_HI_U32, OP_MAD_U64_U32, OP_LSHL_ADD_U64,
       OP_CMP_GE_U64, OP_CNDMASK, OP_SUB_CO, OP_FMA_F64, OP_MUL_U32_U24, OP_MAD_U32_U24,
       OP_COUNT };
static const char* kOpName[OP_COUNT] = {
  "v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32", "v_lshl_add_u64",
  "v_cmp_ge_u64", "v_cndmask_b32", "v_sub_co_u32", "v_fma_f64", "v_mul_u32_u24",
  "v_mad_u32_u24"};

template <int OP>
__device__ __forceinline__ void step8(uint32_t (&a)[8], uint64_t (&w)[8], double (&d)[8], uint32_t m, uint64_t m64, double md) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if constexpr (OP == OP_ADD_U32) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(m));
    if constexpr (OP == OP_MUL_LO_U32) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[k]) : "v"(m));
    if constexpr (OP == OP_MUL_HI_U32) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[k]) : "v"(m));
    if constexpr (OP == OP_MAD_U64_U32) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w[k]) : "v"(a[k]), "v"(m) : "vcc");
    if constexpr (OP == OP_LSHL_ADD_U64) asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(w[k]) : "v"(m64));
    if constexpr (OP == OP_CMP_GE_U64) asm volatile("v_cmp_ge_u64 vcc, %0, %1" : : "v"(w[k]), "v"(m64) : "vcc");
    if constexpr (OP == OP_CNDMASK) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(a[k]) : "v"(m));
    if constexpr (OP == OP_SUB_CO) asm volatile("v_sub_co_u32 %0, vcc, %0, %1" : "+v"(a[k]) : "v"(m) : "vcc");
    if constexpr (OP == OP_FMA_F64) asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(d[k]) : "v"(md));
    if constexpr (OP == OP_MUL_U32_U24) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(a[k]) : "v"(m));
    if constexpr (OP == OP_MAD_U32_U24) asm volatile("v_mad_u32_u24 %0, %0, %1, %0" : "+v"(a[k]) : "v"(m));
  }
}

template <int OP>
__global__ void __launch_bounds__(256) k_issue(uint64_t* sink, int iters, uint32_t seed, uint64_t* clk) {
  uint32_t a[8]; uint64_t w[8]; double d[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) { a[k] = seed * (threadIdx.x + 17 * k + 1); w[k] = a[k] * 3ull; d[k] = 1.0 + a[k]; }
  uint32_t m = seed | 1u; uint64_t m64 = (uint64_t)m << 7; double md = 1.0000001;
  uint64_t t0 = clock64();
  for (int it = 0; it < iters; ++it) {
    step8<OP>(a, w, d, m, m64, md); step8<OP>(a, w, d, m, m64, md);
    step8<OP>(a, w, d, m, m64, md); step8<OP>(a, w, d, m, m64, md);
  }
  uint64_t t1 = clock64();
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += a[k] + w[k] + (uint64_t)d[k];
  if (acc == 0x123456789abcdefull) sink[threadIdx.x] = acc;  // keeps the chains live
  if (threadIdx.x == 0 && blockIdx.x == 0) clk[0] = t1 - t0;
}

__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// One 16-byte vector per thread, no loop (the grid covers the buffer), with
// or without the nontemporal hint; and the read-only / write-only halves.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
template <bool NT>
__global__ void __launch_bounds__(256) k_copy1(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    if (NT) __builtin_nontemporal_store(__builtin_nontemporal_load((const v4u*)src + i), (v4u*)dst + i);
    else dst[i] = src[i];
  }
}
__global__ void __launch_bounds__(256) k_read1(const uint4* __restrict__ src, uint32_t* sink, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const v4u v = __builtin_nontemporal_load((const v4u*)src + i);
    if ((v.x ^ v.y ^ v.z ^ v.w) == 0x9e3779b9u) sink[0] = v.x;
  }
}
__global__ void __launch_bounds__(256) k_write1(uint4* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const v4u v = {(uint32_t)i, 1u, 2u, 3u};
  if (i < n) __builtin_nontemporal_store(v, (v4u*)dst + i);
}

template <int OP>
static int run_issue(int ncu, FILE* out) {
  const int blocks = ncu * 8, threads = 256, iters = 4096;
  uint64_t *sink, *clk;
  CHK(hipMalloc(&sink, threads * sizeof(uint64_t)));
  CHK(hipMalloc(&clk, sizeof(uint64_t)));
  hipEvent_t e0, e1; CHK(hipEventCreate(&e0)); CHK(hipEventCreate(&e1));
  k_issue<OP><<<blocks, threads>>>(sink, 16, 12345u, clk);  // warm-up
  CHK(hipGetLastError());
  CHK(hipEventRecord(e0));
  k_issue<OP><<<blocks, threads>>>(sink, iters, 12345u, clk);
  CHK(hipEventRecord(e1));
  CHK(hipEventSynchronize(e1));
  float ms = 0; CHK(hipEventElapsedTime(&ms, e0, e1));
  uint64_t cyc = 0; CHK(hipMemcpy(&cyc, clk, sizeof(cyc), hipMemcpyDeviceToHost));
  double wave_instr = (double)blocks * (threads / 64) * iters * 32.0;  // wave-level instructions
  double lane_ops_per_s = wave_instr * 64.0 / (ms * 1e-3);
  double simds = ncu * 4.0;
  // GHz from one wave's clock counter over its loop vs wall time is only an
  // estimate (waves are interleaved), so report the rate per SIMD per ns too.
  fprintf(out, "{\"op\": \"%s\", \"ms\": %.4f, \"lane_ops_per_s\": %.4e, \"lanes_per_simd_per_ns\": %.3f, \"wave0_cycles\": %llu}\n",
          kOpName[OP], ms, lane_ops_per_s, lane_ops_per_s / simds / 1e9, (unsigned long long)cyc);
  CHK(hipFree(sink)); CHK(hipFree(clk));
  return 0;
}

static int run_copy(FILE* out) {
  const size_t bytes = (size_t)2 << 30;  // 2 GiB per buffer: 8x the 256 MB last-level cache
  const size_t n = bytes / sizeof(uint4);
  uint4 *a, *b;
  CHK(hipMalloc(&a, bytes)); CHK(hipMalloc(&b, bytes));
  CHK(hipMemset(a, 1, bytes)); CHK(hipMemset(b, 0, bytes));
  hipEvent_t e0, e1; CHK(hipEventCreate(&e0)); CHK(hipEventCreate(&e1));
  int dev; CHK(hipGetDevice(&dev)); hipDeviceProp_t p; CHK(hipGetDeviceProperties(&p, dev));
  const int grid = p.multiProcessorCount * 16;
  k_copy<<<grid, 256>>>(a, b, n);
  CHK(hipGetLastError());
  CHK(hipDeviceSynchronize());
  const int reps = 10;
  CHK(hipEventRecord(e0));
  for (int r = 0; r < reps; ++r) k_copy<<<grid, 256>>>((r & 1) ? b : a, (r & 1) ? a : b, n);
  CHK(hipEventRecord(e1)); CHK(hipEventSynchronize(e1));
  float ms = 0; CHK(hipEventElapsedTime(&ms, e0, e1));
  double gbps = 2.0 * bytes * reps / (ms * 1e-3) / 1e9;
  fprintf(out, "{\"op\": \"copy_kernel_2GiB\", \"ms_per_copy\": %.4f, \"GBps_read_plus_write\": %.1f}\n", ms / reps, gbps);
  CHK(hipEventRecord(e0));
  for (int r = 0; r < reps; ++r) CHK(hipMemcpyAsync((r & 1) ? a : b, (r & 1) ? b : a, bytes, hipMemcpyDeviceToDevice, 0));
  CHK(hipEventRecord(e1)); CHK(hipEventSynchronize(e1));
  CHK(hipEventElapsedTime(&ms, e0, e1));
  gbps = 2.0 * bytes * reps / (ms * 1e-3) / 1e9;
  fprintf(out, "{\"op\": \"hipMemcpy_d2d_2GiB\", \"ms_per_copy\": %.4f, \"GBps_read_plus_write\": %.1f}\n", ms / reps, gbps);
  // one vector per thread over the whole buffer
  const size_t blocks1 = (n + 255) / 256;
  uint32_t* sink;
  CHK(hipMalloc(&sink, 64));
  auto time_it = [&](auto launch) -> float {
    launch(0);
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    CHK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) launch(r);
    CHK(hipEventRecord(e1)); CHK(hipEventSynchronize(e1));
    float t = 0; CHK(hipEventElapsedTime(&t, e0, e1));
    return t / reps;
  };
  ms = time_it([&](int r) { k_copy1<false><<<blocks1, 256>>>((r & 1) ? b : a, (r & 1) ? a : b, n); });
  fprintf(out, "{\"op\": \"copy_one_vector_per_thread_2GiB\", \"ms_per_copy\": %.4f, \"GBps_read_plus_write\": %.1f}\n", ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
  ms = time_it([&](int r) { k_copy1<true><<<blocks1, 256>>>((r & 1) ? b : a, (r & 1) ? a : b, n); });
  fprintf(out, "{\"op\": \"copy_one_vector_per_thread_nontemporal_2GiB\", \"ms_per_copy\": %.4f, \"GBps_read_plus_write\": %.1f}\n", ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
  ms = time_it([&](int r) { k_read1<<<blocks1, 256>>>((r & 1) ? b : a, sink, n); });
  fprintf(out, "{\"op\": \"read_one_vector_per_thread_nontemporal_2GiB\", \"ms\": %.4f, \"GBps\": %.1f}\n", ms, 1.0 * bytes / (ms * 1e-3) / 1e9);
  ms = time_it([&](int r) { k_write1<<<blocks1, 256>>>((r & 1) ? b : a, n); });
  fprintf(out, "{\"op\": \"write_one_vector_per_thread_nontemporal_2GiB\", \"ms\": %.4f, \"GBps\": %.1f}\n", ms, 1.0 * bytes / (ms * 1e-3) / 1e9);
  CHK(hipFree(sink));
  CHK(hipFree(a)); CHK(hipFree(b));
  return 0;
}

// --copy-only: three dispatches of a plain copy of 1 GiB (read 1 GiB, write
// 1 GiB each), the reference for scaling FETCH_SIZE / WRITE_SIZE counters.
static int run_copy_only() {
  const size_t bytes = (size_t)1 << 30, n = bytes / sizeof(uint4);
  uint4 *a, *b;
  CHK(hipMalloc(&a, bytes)); CHK(hipMalloc(&b, bytes));
  CHK(hipMemset(a, 1, bytes)); CHK(hipMemset(b, 0, bytes));
  CHK(hipDeviceSynchronize());
  int dev; CHK(hipGetDevice(&dev)); hipDeviceProp_t p; CHK(hipGetDeviceProperties(&p, dev));
  for (int r = 0; r < 3; ++r) k_copy<<<p.multiProcessorCount * 16, 256>>>(a, b, n);
  CHK(hipGetLastError());
  CHK(hipDeviceSynchronize());
  printf("{\"op\": \"copy_only\", \"dispatches\": 3, \"bytes_read_per_dispatch\": %zu, \"bytes_written_per_dispatch\": %zu}\n", bytes, bytes);
  CHK(hipFree(a)); CHK(hipFree(b));
  return 0;
}

int main(int argc, char** argv) {
  int dev = 0; CHK(hipSetDevice(dev));
  if (argc > 1 && strcmp(argv[1], "--copy-only") == 0) return run_copy_only() ? 1 : 0;
  hipDeviceProp_t p; CHK(hipGetDeviceProperties(&p, dev));
  printf("{\"device\": \"%s\", \"gcnArchName\": \"%s\", \"cus\": %d, \"clock_khz\": %d, \"lds_per_block\": %zu, \"lds_per_cu\": %zu, \"l2_bytes\": %d, \"regs_per_block\": %d, \"hbm_bytes\": %zu, \"mem_clock_khz\": %d, \"mem_bus_bits\": %d}\n",
         p.name, p.gcnArchName, p.multiProcessorCount, p.clockRate, p.sharedMemPerBlock,
         p.maxSharedMemoryPerMultiProcessor, p.l2CacheSize, p.regsPerBlock, p.totalGlobalMem,
         p.memoryClockRate, p.memoryBusWidth);
  fflush(stdout);
  const int ncu = p.multiProcessorCount;
  int rc = 0;
  rc |= run_issue<OP_ADD_U32>(ncu, stdout);
  rc |= run_issue<OP_MUL_LO_U32>(ncu, stdout);
  rc |= run_issue<OP_MUL_HI_U32>(ncu, stdout);
  rc |= run_issue<OP_MAD_U64_U32>(ncu, stdout);
  rc |= run_issue<OP_LSHL_ADD_U64>(ncu, stdout);
  rc |= run_issue<OP_CMP_GE_U64>(ncu, stdout);
  rc |= run_issue<OP_CNDMASK>(ncu, stdout);
  rc |= run_issue<OP_SUB_CO>(ncu, stdout);
  rc |= run_issue<OP_FMA_F64>(ncu, stdout);
  rc |= run_issue<OP_MUL_U32_U24>(ncu, stdout);
  rc |= run_issue<OP_MAD_U32_U24>(ncu, stdout);
  fflush(stdout);
  if (argc < 2 || strcmp(argv[1], "--no-copy") != 0) rc |= run_copy(stdout);
  return rc ? 1 : 0;
}
