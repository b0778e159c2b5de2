// Measured peaks of the chip for the roofline of the local TT-matvec: matrix-core throughput
// of the MFMA instructions the contractions use (FP64, FP32, BF16) and HBM bandwidth of a
// plain copy and a plain read. Each kernel keeps every SIMD busy with independent
// accumulators (or every memory channel with streaming vector accesses), so its rate is the
// attainable ceiling of that unit on this device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"

namespace iga {
namespace k {
namespace {

constexpr int PT = 256;    // threads per workgroup (four waves)
constexpr int NACC = 8;    // independent accumulators per wave
constexpr int PBLK = 2048; // workgroups: eight per CU on 256 CUs

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(PT) void mfma_f64_4x4(const double* a, double* out, int iters) {
  const int l = threadIdx.x & 63;
  const double av = a[l], bv = a[(l + 7) & 63];
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bv, acc[i], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i];
  out[blockIdx.x * PT + threadIdx.x] = s;
}

__global__ __launch_bounds__(PT) void mfma_f64_16x16(const double* a, double* out, int iters) {
  const int l = threadIdx.x & 63;
  const double av = a[l], bv = a[(l + 7) & 63];
  d4 acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[i], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * PT + threadIdx.x] = s;
}

__global__ __launch_bounds__(PT) void mfma_f32_16x16(const double* a, double* out, int iters) {
  const int l = threadIdx.x & 63;
  const float av = (float)a[l], bv = (float)a[(l + 7) & 63];
  f4 acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i], 0, 0, 0);
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * PT + threadIdx.x] = s;
}

__global__ __launch_bounds__(PT) void mfma_bf16_16x16x32(const double* a, double* out, int iters) {
  const int l = threadIdx.x & 63;
  s8 av, bv;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    // bfloat16 bits of small positive values (the upper half of their float encoding)
    const float x = (float)a[(l + e) & 63], y = (float)a[(l + 7 + e) & 63];
    av[e] = (short)(__float_as_uint(x) >> 16);
    bv[e] = (short)(__float_as_uint(y) >> 16);
  }
  f4 acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * PT + threadIdx.x] = s;
}

// y = x, 16 bytes per lane per access, grid-stride over n2 double2 elements
__global__ __launch_bounds__(PT) void stream_copy(const double2* __restrict__ x, double2* __restrict__ y, long n2) {
  for (long i = (long)blockIdx.x * PT + threadIdx.x; i < n2; i += (long)gridDim.x * PT) y[i] = x[i];
}

// per-thread partial sums of x (read only; the partials are written once)
__global__ __launch_bounds__(PT) void stream_read(const double2* __restrict__ x, long n2, double* part) {
  double s = 0.0;
  for (long i = (long)blockIdx.x * PT + threadIdx.x; i < n2; i += (long)gridDim.x * PT) {
    const double2 v = x[i];
    s += v.x + v.y;
  }
  part[(long)blockIdx.x * PT + threadIdx.x] = s;
}

__global__ void probe_init(double* a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = 1e-3 * (double)(1 + (i % 61));
}

struct HipMem {
  void* p = nullptr;
  ~HipMem() {
    if (p) (void)hipFree(p);
  }
};
struct HipEv {
  hipEvent_t e = nullptr;
  ~HipEv() {
    if (e) (void)hipEventDestroy(e);
  }
};

}  // namespace

// out[0..5]: TFLOP/s of v_mfma_f64_4x4x4_4b, v_mfma_f64_16x16x4, v_mfma_f32_16x16x4,
// v_mfma_f32_16x16x32_bf16; GB/s of a device copy (bytes read + written) and of a device read.
// Best of three timed launches each, after one untimed launch.
void measure_peaks(iga_ctx* ctx, double* out) {
  hipStream_t s = ctx->stream;
  DBuf a(ctx, 64), sink(ctx, (size_t)PBLK * PT);
  probe_init<<<1, 64, 0, s>>>(a.get(), 64);
  IGA_HIP(hipGetLastError());
  HipEv ev0, ev1;
  IGA_HIP(hipEventCreate(&ev0.e));
  IGA_HIP(hipEventCreate(&ev1.e));
  hipEvent_t e0 = ev0.e, e1 = ev1.e;
  auto best_ms = [&](auto&& launch) {
    launch();
    IGA_HIP(hipGetLastError());
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      IGA_HIP(hipEventRecord(e0, s));
      launch();
      IGA_HIP(hipEventRecord(e1, s));
      IGA_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      IGA_HIP(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, ms);
    }
    IGA_HIP(hipGetLastError());
    return (double)best;
  };
  const double waves = (double)PBLK * (PT / 64);
  struct M {
    void (*kern)(const double*, double*, int);
    int iters;
    double flops_per_inst;
  };
  const M mf[4] = {{mfma_f64_4x4, 20000, 512.0},
                   {mfma_f64_16x16, 5000, 2048.0},
                   {mfma_f32_16x16, 10000, 2048.0},
                   {mfma_bf16_16x16x32, 20000, 16384.0}};
  for (int i = 0; i < 4; ++i) {
    const double ms = best_ms([&] { mf[i].kern<<<PBLK, PT, 0, s>>>(a.get(), sink.get(), mf[i].iters); });
    out[i] = waves * mf[i].iters * NACC * mf[i].flops_per_inst / (ms * 1e-3) / 1e12;
  }
  // 512 MiB per buffer: far beyond the last-level caches
  const long bytes = 512L << 20, n2 = bytes / 16;
  HipMem xm, ym;
  if (hipMalloc(&xm.p, bytes) != hipSuccess || hipMalloc(&ym.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    fail(IGA_ENOMEM, "measure_peaks: device allocation of 2 x 512 MiB failed");
  }
  void *x = xm.p, *y = ym.p;
  probe_init<<<1024, 256, 0, s>>>(static_cast<double*>(x), bytes / 8);
  const unsigned grid = 256 * 16;
  DBuf part(ctx, (size_t)grid * PT);
  const double mc = best_ms([&] {
    stream_copy<<<grid, PT, 0, s>>>(static_cast<const double2*>(x), static_cast<double2*>(y), n2);
  });
  const double mr = best_ms([&] { stream_read<<<grid, PT, 0, s>>>(static_cast<const double2*>(x), n2, part.get()); });
  IGA_HIP(hipStreamSynchronize(s));
  out[4] = 2.0 * bytes / (mc * 1e-3) / 1e9;
  out[5] = (double)bytes / (mr * 1e-3) / 1e9;
}

}  // namespace k
}  // namespace iga
