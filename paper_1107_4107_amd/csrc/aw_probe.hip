// Achievable FP64 vector rate and the sustained shader clock of the device,
// and the device's own sine and cosine evaluated on given arguments.
//
// Probes built into their own library (libaw_probe.so), used by the benchmark
// and the tests, never by the library.  The rate probe: every lane runs CHAINS independent chains of FP64
// fused multiply-adds, so that the issue of v_fma_f64 is limited by the SIMD's
// FP64 throughput and not by the latency of one chain.  Each wave also reads
// the shader-clock counter and the constant-rate wall clock around its loop;
// their ratio gives the clock the SIMDs actually ran at under full FP64 load.
//
// The chains iterate a <- a*m + c with |m| < 1, a contraction towards
// c/(1-m), so the values stay finite for any iteration count.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "aw_device.hpp"

namespace {

constexpr int CHAINS = 8;   // independent FMA chains per lane
constexpr int INNER = 16;   // FMAs per chain per trip of the counted loop
constexpr int BLOCK = 256;

__global__ __launch_bounds__(BLOCK) void k_fma_chains(double m, double c, int64_t trips, double* sink,
                                                      unsigned long long* clk) {
  const int gid = blockIdx.x * BLOCK + threadIdx.x;
  double a[CHAINS];
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) a[k] = 1.0 + 1e-3 * (gid & 15) + 1e-4 * k;
  const unsigned long long t0 = clock64();
  const unsigned long long w0 = wall_clock64();
  for (int64_t it = 0; it < trips; ++it) {
#pragma unroll
    for (int r = 0; r < INNER; ++r) {
#pragma unroll
      for (int k = 0; k < CHAINS; ++k) a[k] = __builtin_fma(a[k], m, c);
    }
  }
  const unsigned long long t1 = clock64();
  const unsigned long long w1 = wall_clock64();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) s += a[k];
  sink[gid] = s;
  if ((threadIdx.x & 63) == 0) {
    const int wave = gid >> 6;
    clk[2 * wave] = t1 - t0;
    clk[2 * wave + 1] = w1 - w0;
  }
}

// The table-driven sine and cosine of the propagation and adjoint kernels, the
// kicks' doubled-angle z terms and the polynomial form of the initial
// conditions, one argument per lane.
__global__ __launch_bounds__(BLOCK) void k_sincos(const double* __restrict__ x, double* __restrict__ s,
                                                  double* __restrict__ c, int64_t n, int32_t form) {
  __shared__ double2 tab[AW_TAB_N];
  aw::load_sincos_table(tab);  // before any lane returns: it ends in a barrier
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  if (form == 0) {
    const aw::SinCosT r = aw::sincos_tab(x[i], tab);
    s[i] = r.s;
    c[i] = r.c;
  } else if (form == 2) {
    const aw::ZTerms r = aw::zterms_tab(x[i], tab);
    s[i] = r.czsz;
    c[i] = r.cz2;
  } else {
    double sv, cv;
    aw::sincos_full(x[i], sv, cv);
    s[i] = sv;
    c[i] = cv;
  }
}

int fail(hipError_t e, const char* what) {
  std::fprintf(stderr, "aw_probe: %s: %s\n", what, hipGetErrorString(e));
  return 1;
}

}  // namespace

// Runs the probe once untimed (trips/8) and once timed, on the current
// device, with waves_per_simd waves resident on each of the device's SIMDs.
// out[0] = kernel time in ms (HIP events), out[1] = FP64 TFLOP/s (an FMA
// counts 2), out[2] = mean shader clock in Hz over the waves, out[3] = the
// wall-clock counter rate in Hz, out[4] = number of waves.
// Returns 0 on success, 1 on a HIP error (printed), 2 on bad arguments.
extern "C" int awp_fma_peak(int32_t waves_per_simd, int64_t trips, double* out) {
  if (waves_per_simd < 1 || waves_per_simd > 8 || trips < 8 || out == nullptr) return 2;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(e, "hipGetDevice");
  int n_cu = 0, wall_khz = 0;
  if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return fail(e, "CU count");
  if ((e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess)
    return fail(e, "wall clock rate");
  const int64_t threads = (int64_t)n_cu * 4 * waves_per_simd * 64;  // 4 SIMDs per CU, wave64
  const int blocks = (int)(threads / BLOCK);                          // threads is a multiple of 256
  const int waves = (int)(threads / 64);
  double* sink = nullptr;
  unsigned long long* clk = nullptr;
  if ((e = hipMalloc(&sink, threads * sizeof(double))) != hipSuccess) return fail(e, "hipMalloc sink");
  if ((e = hipMalloc(&clk, 2 * (size_t)waves * sizeof(unsigned long long))) != hipSuccess) {
    (void)hipFree(sink);
    return fail(e, "hipMalloc clk");
  }
  unsigned long long* host = new unsigned long long[2 * (size_t)waves];
  hipEvent_t ev0, ev1;
  (void)hipEventCreate(&ev0);
  (void)hipEventCreate(&ev1);
  const double m = 0.9999999, c = 1e-7;
  int rc = 0;
  k_fma_chains<<<blocks, BLOCK>>>(m, c, trips / 8, sink, clk);
  (void)hipEventRecord(ev0, nullptr);
  k_fma_chains<<<blocks, BLOCK>>>(m, c, trips, sink, clk);
  (void)hipEventRecord(ev1, nullptr);
  if ((e = hipEventSynchronize(ev1)) != hipSuccess) {
    rc = fail(e, "probe kernel");
  } else if ((e = hipMemcpy(host, clk, 2 * (size_t)waves * sizeof(unsigned long long), hipMemcpyDeviceToHost)) !=
             hipSuccess) {
    rc = fail(e, "clock copy");
  } else {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    const double wall_hz = 1e3 * wall_khz;
    double sum_hz = 0.0;
    for (int w = 0; w < waves; ++w) {
      const double dt = host[2 * w + 1] / wall_hz;
      sum_hz += dt > 0.0 ? host[2 * w] / dt : 0.0;
    }
    const double flop = 2.0 * CHAINS * INNER * (double)trips * (double)threads;
    out[0] = ms;
    out[1] = flop / (ms * 1e-3) / 1e12;
    out[2] = sum_hz / waves;
    out[3] = wall_hz;
    out[4] = waves;
  }
  delete[] host;
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  (void)hipFree(sink);
  (void)hipFree(clk);
  return rc;
}

// Writes s_dev[i], c_dev[i] = sin, cos of x_dev[i] (device arrays of n
// doubles) as the kernels compute them: form 0 = the table-driven routine of
// the step loops, 1 = the polynomial routine of the initial conditions and
// the energy; form 2 writes the kicks' z terms instead, s = cos x sin x and
// c = cos^2 x, from the table at the doubled angle.  Enqueued on `stream`
// (NULL = default).  Returns 0, 1 on a HIP error (printed), 2 on bad
// arguments.
extern "C" int awp_sincos(const double* x_dev, double* s_dev, double* c_dev, int64_t n, int32_t form,
                          void* stream) {
  if (n < 0 || form < 0 || form > 2) return 2;
  if (n == 0) return 0;
  if (!x_dev || !s_dev || !c_dev) return 2;
  const int64_t blocks = (n + BLOCK - 1) / BLOCK;
  if (blocks > INT32_MAX) return 2;
  hipLaunchKernelGGL(k_sincos, dim3((unsigned)blocks), dim3(BLOCK), 0, (hipStream_t)stream, x_dev, s_dev, c_dev, n,
                     form);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : fail(e, "sincos probe");
}
