// Peak probes for the roofline: the rates this GPU sustains for the
// instructions the IFGF kernels are built from, measured with HIP events.
// A separate library (libifgf_probe.so) used by the benchmark only; it is not
// part of the IFGF C ABI.
//
//   ifgf_probe_run(IFGF_PROBE_MFMA_F32, &v)  v_mfma_f32_16x16x4_f32 chains, TFLOP/s
//   ifgf_probe_run(IFGF_PROBE_FMA_F32,  &v)  v_fma_f32 (non-packed) chains, TFLOP/s
//   ifgf_probe_run(IFGF_PROBE_FMA_F64,  &v)  v_fma_f64 chains, TFLOP/s
//   ifgf_probe_run(IFGF_PROBE_COPY,     &v)  1 GiB device copy with 16-byte
//                                           vector loads/stores, GB/s (read + written)
//
// Returns 0 on success, a HIP error code otherwise (v untouched).
//
//   ifgf_probe_math64(x, out, n, stream)  for device FP64 x[n]: out[5 i ..] =
//       sin x_i, cos x_i (sincos_cw64), sqrt |x_i|, 1/sqrt |x_i|
//       (sqrt_rsqrt_nr64) and 1/x_i (rcp_nr64), as the IFGF kernels compute
//       them; for the accuracy tests (x_i != 0).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int PTPB = 256;

// Four independent accumulation chains of 16x16x4 FP32 MFMAs per wave.
__global__ __launch_bounds__(PTPB) void k_probe_mfma(const float* __restrict__ in, float* __restrict__ out,
                                                     int iters) {
  const int l = threadIdx.x;
  float a[8], b[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = in[(l + i) & 255];
    b[i] = in[(3 * l + i) & 255];
  }
  floatx4 d0 = {0, 0, 0, 0}, d1 = d0, d2 = d0, d3 = d0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; i += 4) {
      d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[i], d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i + 1], b[i + 1], d1, 0, 0, 0);
      d2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i + 2], b[i + 2], d2, 0, 0, 0);
      d3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i + 3], b[i + 3], d3, 0, 0, 0);
    }
  }
  const floatx4 s = d0 + d1 + d2 + d3;
  out[blockIdx.x * PTPB + l] = s[0] + s[1] + s[2] + s[3];
}

// Eight independent FMA chains per lane (no packed instructions: the library
// is built without them).
template <typename T>
__global__ __launch_bounds__(PTPB) void k_probe_fma(const T* __restrict__ in, T* __restrict__ out, int iters) {
  const int l = threadIdx.x;
  T x[8];
  const T m = in[l & 255], c = in[(l + 7) & 255];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = in[(l + i) & 255];
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if constexpr (sizeof(T) == 4)
          x[i] = __builtin_fmaf(x[i], m, c);
        else
          x[i] = __builtin_fma(x[i], m, c);
      }
    }
  }
  T s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += x[i];
  out[blockIdx.x * PTPB + l] = s;
}

// Grid-stride copy, four 16-byte loads in flight per thread before the stores.
__global__ __launch_bounds__(PTPB) void k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * PTPB;
  for (int64_t i = (int64_t)blockIdx.x * PTPB + threadIdx.x; i < n; i += 4 * stride) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * stride < n) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * stride < n) dst[i + u * stride] = v[u];
  }
}

template <typename F>
hipError_t timed(F launch, float* ms) {
  hipEvent_t e0, e1;
  hipError_t st = hipEventCreate(&e0);
  if (st != hipSuccess) return st;
  st = hipEventCreate(&e1);
  if (st != hipSuccess) {
    (void)hipEventDestroy(e0);
    return st;
  }
  launch();   // warm-up
  st = hipDeviceSynchronize();
  if (st == hipSuccess) st = hipEventRecord(e0, nullptr);
  if (st == hipSuccess) {
    launch();
    st = hipGetLastError();
  }
  if (st == hipSuccess) st = hipEventRecord(e1, nullptr);
  if (st == hipSuccess) st = hipEventSynchronize(e1);
  if (st == hipSuccess) st = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

__global__ __launch_bounds__(PTPB) void k_probe_math64(const double* __restrict__ x, double* __restrict__ out,
                                                       int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * PTPB + threadIdx.x;
  if (i >= n) return;
  double s, c, sq, rs;
  sincos_cw64(x[i], &s, &c);
  sqrt_rsqrt_nr64(fabs(x[i]), &sq, &rs);
  out[5 * i] = s;
  out[5 * i + 1] = c;
  out[5 * i + 2] = sq;
  out[5 * i + 3] = rs;
  out[5 * i + 4] = rcp_nr64(x[i]);
}

}  // namespace

extern "C" {

int ifgf_probe_math64(const double* x, double* out, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!x || !out))) return (int)hipErrorInvalidValue;
  if (n == 0) return 0;
  k_probe_math64<<<(unsigned)((n + PTPB - 1) / PTPB), PTPB, 0, (hipStream_t)stream>>>(x, out, n);
  return (int)hipGetLastError();
}

enum { IFGF_PROBE_MFMA_F32 = 0, IFGF_PROBE_FMA_F32 = 1, IFGF_PROBE_FMA_F64 = 2, IFGF_PROBE_COPY = 3 };

int ifgf_probe_run(int which, double* value) {
  if (!value || which < 0 || which > IFGF_PROBE_COPY) return (int)hipErrorInvalidValue;
  int dev = 0, ncu = 0;
  hipError_t st = hipGetDevice(&dev);
  if (st == hipSuccess) st = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (st != hipSuccess) return (int)st;
  const int nblk = 8 * ncu;   // 8 four-wave blocks per CU
  void* in = nullptr;
  void* out = nullptr;
  st = hipMalloc(&in, 256 * sizeof(double));
  if (st == hipSuccess) st = hipMalloc(&out, (size_t)nblk * PTPB * sizeof(double));
  if (st == hipSuccess) st = hipMemset(in, 0, 256 * sizeof(double));
  float ms = 0;
  double v = 0;
  if (st == hipSuccess) {
    if (which == IFGF_PROBE_MFMA_F32) {
      const int iters = 2000;
      st = timed([&] { k_probe_mfma<<<nblk, PTPB>>>((const float*)in, (float*)out, iters); }, &ms);
      v = (double)nblk * (PTPB / 64) * iters * 8 * (16.0 * 16 * 4 * 2) / (ms * 1e-3) / 1e12;
    } else if (which == IFGF_PROBE_FMA_F32) {
      const int iters = 4000;
      st = timed([&] { k_probe_fma<float><<<nblk, PTPB>>>((const float*)in, (float*)out, iters); }, &ms);
      v = (double)nblk * PTPB * iters * 16 * 8 * 2 / (ms * 1e-3) / 1e12;
    } else if (which == IFGF_PROBE_FMA_F64) {
      const int iters = 2000;
      st = timed([&] { k_probe_fma<double><<<nblk, PTPB>>>((const double*)in, (double*)out, iters); }, &ms);
      v = (double)nblk * PTPB * iters * 16 * 8 * 2 / (ms * 1e-3) / 1e12;
    } else {
      const int64_t bytes = (int64_t)1 << 30;
      void* a = nullptr;
      void* b = nullptr;
      st = hipMalloc(&a, bytes);
      if (st == hipSuccess) st = hipMalloc(&b, bytes);
      if (st == hipSuccess) st = hipMemset(a, 0, bytes);
      if (st == hipSuccess)
        st = timed([&] { k_probe_copy<<<4 * nblk, PTPB>>>((const float4*)a, (float4*)b, bytes / 16); }, &ms);
      v = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
      if (a) (void)hipFree(a);
      if (b) (void)hipFree(b);
    }
  }
  if (in) (void)hipFree(in);
  if (out) (void)hipFree(out);
  if (st != hipSuccess) return (int)st;
  *value = v;
  return 0;
}

}  // extern "C"
