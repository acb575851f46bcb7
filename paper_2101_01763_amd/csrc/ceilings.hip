// Achievable ceilings of the device, measured by kernels of this library
// (the measurement helpers of include/spand.h): a streaming copy and a
// streaming read for the HBM bandwidth, and loops of independent matrix-core instructions for the FP32
// and FP64 matrix throughput, the instructions the factorization's products
// use (v_mfma_f32_32x32x2f32, v_mfma_f64_16x16x4f64).
#include "internal.h"

namespace spand {

typedef double ceil_f64x2 __attribute__((ext_vector_type(2)));

// dst = src, 16-byte loads and stores, grid-stride over n 16-byte words
__global__ __launch_bounds__(256) void k_stream_copy(const ceil_f64x2 *__restrict__ src,
                                                     ceil_f64x2 *__restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const ceil_f64x2 a = __builtin_nontemporal_load(src + i);
    const ceil_f64x2 b = __builtin_nontemporal_load(src + i + stride);
    const ceil_f64x2 c = __builtin_nontemporal_load(src + i + 2 * stride);
    const ceil_f64x2 d = __builtin_nontemporal_load(src + i + 3 * stride);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
    __builtin_nontemporal_store(c, dst + i + 2 * stride);
    __builtin_nontemporal_store(d, dst + i + 3 * stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// streaming read of n 16-byte words (the sum is stored only if it takes an
// impossible value, which keeps the loads)
__global__ __launch_bounds__(256) void k_stream_read(const ceil_f64x2 *__restrict__ src,
                                                     double *__restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  ceil_f64x2 acc = {0.0, 0.0};
  for (; i + 3 * stride < n; i += 4 * stride) {
    const ceil_f64x2 a = __builtin_nontemporal_load(src + i);
    const ceil_f64x2 b = __builtin_nontemporal_load(src + i + stride);
    const ceil_f64x2 c = __builtin_nontemporal_load(src + i + 2 * stride);
    const ceil_f64x2 d = __builtin_nontemporal_load(src + i + 3 * stride);
    acc += (a + b) + (c + d);
  }
  for (; i < n; i += stride) acc += src[i];
  if (acc[0] + acc[1] == -1.0) out[0] = acc[0];
}

typedef float ceil_f32x16 __attribute__((ext_vector_type(16)));
typedef double ceil_f64x4 __attribute__((ext_vector_type(4)));

// iters rounds of 4 independent v_mfma_f32_32x32x2f32 per wave (4096 flops each)
__global__ __launch_bounds__(256) void k_mfma_f32_loop(float *__restrict__ out, int iters) {
  ceil_f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  const float a = 1.0f + 1e-3f * float(threadIdx.x & 63), b = 0.5f;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c3, 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < 16; ++q) s += c0[q] + c1[q] + c2[q] + c3[q];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// iters rounds of 8 independent v_mfma_f64_16x16x4f64 per wave (2048 flops each)
__global__ __launch_bounds__(256) void k_mfma_f64_loop(double *__restrict__ out, int iters) {
  ceil_f64x4 c[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) c[q] = ceil_f64x4{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + 1e-3 * double(threadIdx.x & 63), b = 0.5;
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[q], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += (c[q][0] + c[q][1]) + (c[q][2] + c[q][3]);
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace spand

using namespace spand;

// median of `reps` timed launches (after one untimed)
template <typename F>
static int time_launches(hipStream_t st, int reps, F &&launch, float *ms_out) {
  hipEvent_t a, b;
  SP_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return SPAND_EHIP;
  }
  std::vector<float> t;
  int r = SPAND_OK;
  for (int i = 0; i <= reps && r == SPAND_OK; ++i) {
    if (hipEventRecord(a, st) != hipSuccess) r = SPAND_EHIP;
    launch();
    if (r == SPAND_OK && (hipGetLastError() != hipSuccess || hipEventRecord(b, st) != hipSuccess ||
                          hipEventSynchronize(b) != hipSuccess))
      r = SPAND_EHIP;
    float ms = 0.f;
    if (r == SPAND_OK && hipEventElapsedTime(&ms, a, b) == hipSuccess && i > 0) t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (r != SPAND_OK || t.empty()) {
    set_error("ceiling measurement failed");
    return SPAND_EHIP;
  }
  std::sort(t.begin(), t.end());
  *ms_out = t[t.size() / 2];
  return SPAND_OK;
}

extern "C" {

int spand_measure_bandwidth(int32_t mode, size_t bytes, int reps, void *stream, double *gbs) {
  set_error("");
  if (!gbs || bytes < 16 * 256 || reps < 1 || (mode != 0 && mode != 1)) {
    set_error("bad bandwidth measurement arguments");
    return SPAND_EINVAL;
  }
  bytes &= ~size_t(15);
  hipStream_t st = (hipStream_t)stream;
  void *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, mode == 0 ? bytes : 256) != hipSuccess) {
    if (src) (void)hipFree(src);
    set_error("hipMalloc of %zu bytes failed", bytes);
    return SPAND_ENOMEM;
  }
  int r = hipMemsetAsync(src, 0, bytes, st) == hipSuccess ? SPAND_OK : SPAND_EHIP;
  const int64_t n = int64_t(bytes / 16);
  float ms = 0.f;
  if (r == SPAND_OK)
    r = time_launches(st, reps, [&]() {
      // 128 workgroups per CU (measured best of 8-128 on MI355X)
      if (mode == 0)
        hipLaunchKernelGGL(k_stream_copy, dim3(32768), dim3(256), 0, st, (const ceil_f64x2 *)src,
                           (ceil_f64x2 *)dst, n);
      else
        hipLaunchKernelGGL(k_stream_read, dim3(32768), dim3(256), 0, st, (const ceil_f64x2 *)src,
                           (double *)dst, n);
    }, &ms);
  (void)hipStreamSynchronize(st);
  (void)hipFree(src);
  (void)hipFree(dst);
  if (r == SPAND_OK) *gbs = (mode == 0 ? 2.0 : 1.0) * double(bytes) / (double(ms) * 1e-3) / 1e9;
  return r;
}

int spand_measure_mfma(int32_t dtype, int reps, void *stream, double *tflops) {
  set_error("");
  if (!tflops || reps < 1 || (dtype != SPAND_F32 && dtype != SPAND_F64)) {
    set_error("bad matrix-core measurement arguments");
    return SPAND_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int blocks = 256 * 16, iters = 2048;     // 16 workgroups (64 waves) per CU
  void *out = nullptr;
  if (hipMalloc(&out, size_t(blocks) * 256 * 8) != hipSuccess) {
    set_error("hipMalloc failed");
    return SPAND_ENOMEM;
  }
  float ms = 0.f;
  const int r = time_launches(st, reps, [&]() {
    if (dtype == SPAND_F32)
      hipLaunchKernelGGL(k_mfma_f32_loop, dim3(blocks), dim3(256), 0, st, (float *)out, iters);
    else
      hipLaunchKernelGGL(k_mfma_f64_loop, dim3(blocks), dim3(256), 0, st, (double *)out, iters);
  }, &ms);
  (void)hipStreamSynchronize(st);
  (void)hipFree(out);
  if (r != SPAND_OK) return r;
  const double per_inst = dtype == SPAND_F32 ? 2.0 * 32 * 32 * 2 : 2.0 * 16 * 16 * 4;
  const double waves = double(blocks) * 4;
  const int chains = dtype == SPAND_F32 ? 4 : 8;
  *tflops = waves * iters * chains * per_inst / (double(ms) * 1e-3) / 1e12;
  return SPAND_OK;
}

}  // extern "C"
