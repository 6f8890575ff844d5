// Measured peaks of the board, beside the published ones in a roofline: the HBM bandwidth of
// a plain float64 copy and the FP64 vector FMA rate, each the best of several launches timed
// with HIP events.  A measurement aid of the benchmark, not a step of the method.
#include <hip/hip_runtime.h>

#include "dgx.h"

namespace {

constexpr size_t COPY_BYTES = size_t(2) << 30;   // per buffer: far beyond the 256 MB last-level cache
constexpr int COPY_BLOCKS = 32768;
constexpr int COPY_UNROLL = 4;                    // 16-byte loads in flight per lane
constexpr int FMA_BLOCKS = 2048;                  // 8 waves on each of the 1024 SIMDs
constexpr int FMA_ITERS = 2048;
constexpr int REPS = 10;

typedef double f64x2 __attribute__((ext_vector_type(2)));

// dst = src over n2 16-byte vectors, grid-stride: every lane issues COPY_UNROLL loads before
// its stores, and both bypass the caches' retention (non-temporal), which is the fastest of
// the copy shapes tried on gfx950 (about 6 TB/s against 4.7 TB/s for one plain load per lane).
__global__ __launch_bounds__(256) void k_peak_copy(const f64x2* __restrict__ src,
                                                   f64x2* __restrict__ dst, size_t n2) {
  const size_t step = (size_t)gridDim.x * 256 * COPY_UNROLL;
  for (size_t b = (size_t)blockIdx.x * 256 * COPY_UNROLL + threadIdx.x; b < n2; b += step) {
    f64x2 v[COPY_UNROLL];
#pragma unroll
    for (int k = 0; k < COPY_UNROLL; ++k) {
      const size_t i = b + (size_t)k * 256;
      if (i < n2) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < COPY_UNROLL; ++k) {
      const size_t i = b + (size_t)k * 256;
      if (i < n2) __builtin_nontemporal_store(v[k], dst + i);
    }
  }
}

// Eight independent FMA chains per lane, 32 FMAs per chain and iteration; the chains' sum is
// stored so that none of them is dead.  With |a| < 1 the values stay bounded.
__global__ __launch_bounds__(256) void k_peak_fma(double* __restrict__ out, int iters, double a,
                                                  double b) {
  const double s = 1e-3 * (double)(threadIdx.x & 63u);
  double x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = s + c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 32; ++r) {
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = fma(x[c], a, b);
    }
  }
  double t = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) t += x[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

struct Probe {
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* p0 = nullptr;
  void* p1 = nullptr;
  ~Probe() {
    if (st) (void)hipStreamSynchronize(st);
    if (p0) (void)hipFree(p0);
    if (p1) (void)hipFree(p1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
  }
};

template <typename Launch>
dgx_status best_ms(Probe& p, Launch launch, float& best) {
  launch();   // warm-up
  if (hipGetLastError() != hipSuccess) return DGX_EHIP;
  best = 1e30f;
  for (int r = 0; r < REPS; ++r) {
    float ms = 0.0f;
    if (hipEventRecord(p.e0, p.st) != hipSuccess) return DGX_EHIP;
    launch();
    if (hipEventRecord(p.e1, p.st) != hipSuccess || hipEventSynchronize(p.e1) != hipSuccess ||
        hipEventElapsedTime(&ms, p.e0, p.e1) != hipSuccess)
      return DGX_EHIP;
    if (ms < best) best = ms;
  }
  return hipGetLastError() == hipSuccess ? DGX_OK : DGX_EHIP;
}

dgx_status measure(int kind, double* value) {
  Probe p;
  if (hipStreamCreateWithFlags(&p.st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&p.e0) != hipSuccess || hipEventCreate(&p.e1) != hipSuccess)
    return DGX_EHIP;
  float ms = 0.0f;
  if (kind == 0) {
    if (hipMalloc(&p.p0, COPY_BYTES) != hipSuccess || hipMalloc(&p.p1, COPY_BYTES) != hipSuccess) {
      (void)hipGetLastError();
      return DGX_ENOMEM;
    }
    if (hipMemsetAsync(p.p0, 0, COPY_BYTES, p.st) != hipSuccess) return DGX_EHIP;
    const size_t n2 = COPY_BYTES / sizeof(f64x2);
    const auto* src = static_cast<const f64x2*>(p.p0);
    auto* dst = static_cast<f64x2*>(p.p1);
    const dgx_status s = best_ms(p, [&] {
      hipLaunchKernelGGL(k_peak_copy, dim3(COPY_BLOCKS), dim3(256), 0, p.st, src, dst, n2);
    }, ms);
    if (s != DGX_OK) return s;
    *value = 2.0 * (double)COPY_BYTES / (ms * 1e-3) * 1e-9;   // GB/s, read + written
  } else {
    const size_t n = (size_t)FMA_BLOCKS * 256;
    if (hipMalloc(&p.p0, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return DGX_ENOMEM;
    }
    auto* out = static_cast<double*>(p.p0);
    const dgx_status s = best_ms(p, [&] {
      hipLaunchKernelGGL(k_peak_fma, dim3(FMA_BLOCKS), dim3(256), 0, p.st, out, FMA_ITERS,
                         0.999999, 1e-7);
    }, ms);
    if (s != DGX_OK) return s;
    const double flops = 2.0 * 8 * 32 * (double)FMA_ITERS * (double)n;
    *value = flops / (ms * 1e-3) * 1e-12;   // TFLOP/s
  }
  return DGX_OK;
}

}  // namespace

extern "C" dgx_status dgx_measure_peak(int32_t device, int32_t kind, double* value) {
  if (!value || (kind != DGX_PEAK_HBM_COPY && kind != DGX_PEAK_FP64_FMA)) return DGX_EINVAL;
  int ndev = 0, prev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DGX_EINVAL;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return DGX_EHIP;
  const dgx_status s = measure(kind, value);
  (void)hipSetDevice(prev);
  return s;
}
