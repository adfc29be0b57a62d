// Device calibration for the roofline of the stage kernels (a measurement aid, not part of the
// scheme): a sustained FP64 FMA stream whose rate and shader clock show what the vector FP64
// units deliver under a long, dense load, to set beside the published peak.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

namespace swe_calib {

constexpr int CHAINS = 8;   // independent FMA chains per lane
constexpr int UNROLL = 16;  // FMAs per chain per loop trip

// Each lane runs CHAINS independent FMA chains; lane 0 of each wavefront records its shader-clock
// and constant-rate clock spans. A block is four wavefronts, which the device places on the four
// SIMDs of a CU; dynamic LDS limits how many blocks share a CU, so W blocks per CU are W
// wavefronts per SIMD.
__global__ __launch_bounds__(256) void k_fma_stream(double* out, unsigned long long* spans, int iters, double b,
                                                   double c) {
  extern __shared__ double pad[];
  const int t = threadIdx.x;
  const unsigned long long c0 = clock64(), w0 = wall_clock64();
  pad[t] = (double)t;
  __syncthreads();
  double a[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) a[j] = pad[(t + j) & 255] * 1e-3 + j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
      for (int j = 0; j < CHAINS; ++j) a[j] = __builtin_fma(a[j], b, c);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) s += a[j];
  out[(size_t)blockIdx.x * 256 + t] = s;
  const unsigned long long c1 = clock64(), w1 = wall_clock64();
  if ((t & 63) == 0) {
    const size_t wv = (size_t)blockIdx.x * 4 + (t >> 6);
    spans[2 * wv] = c1 - c0;
    spans[2 * wv + 1] = w1 - w0;
  }
}

}  // namespace swe_calib

extern "C" {

// Sustained FP64 FMA rate with waves_per_simd (1, 2, 4 or 8) wavefronts per SIMD (that many
// four-wavefront blocks per CU), launched back to back for about `seconds` on the current device
// and default stream. Reports (host
// pointers) the median TFLOP/s of the second half of the launches (FMA = 2 flops) and the mean
// shader clock of those launches in MHz. Returns 0, -1 for bad arguments, -3 for a HIP error.
// Synchronises the device; allocates and frees its own buffers.
int swe_calib_fp64_fma(int waves_per_simd, double seconds, double* tflops, double* shader_mhz) {
  if ((waves_per_simd != 1 && waves_per_simd != 2 && waves_per_simd != 4 && waves_per_simd != 8) ||
      !(seconds > 0.0) || seconds > 60.0 || !tflops || !shader_mhz)
    return -1;
  int dev = 0, cus = 0, wclk_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -3;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return -3;
  if (hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wclk_khz <= 0)
    return -3;
  size_t lds_cu = 0;
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || v <= 0)
      return -3;
    lds_cu = (size_t)v;
  }
  // blocks per CU = waves_per_simd: LDS per block just above 1/(that+1) of the CU's
  const int per_cu = waves_per_simd;
  const size_t lds = ((lds_cu / per_cu) / 512) * 512 - 1024;
  if (lds * (per_cu + 1) <= lds_cu || lds * per_cu > lds_cu) return -1;
  {
    int blk = 0;  // the device's largest LDS allocation per block
    if (hipDeviceGetAttribute(&blk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return -3;
    if (lds > (size_t)blk) return -1;
  }
  const int nblk = cus * per_cu * 4;  // four rounds of resident blocks per launch
  const int nwave = nblk * 4;
  const int iters = 1 << 11;
  double* out = nullptr;
  unsigned long long* spans = nullptr;
  if (hipMalloc(&out, sizeof(double) * 256 * (size_t)nblk) != hipSuccess) return -3;
  if (hipMalloc(&spans, sizeof(unsigned long long) * 2 * (size_t)nwave) != hipSuccess) {
    (void)hipFree(out);
    return -3;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  std::vector<double> rate, mhz;
  std::vector<unsigned long long> h(2 * (size_t)nwave);
  const double flops = 2.0 * swe_calib::CHAINS * swe_calib::UNROLL * (double)iters * 256.0 * nblk;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -3;
  const auto t0 = std::chrono::steady_clock::now();
  while (rc == 0) {
    if (hipEventRecord(e0, nullptr) != hipSuccess) { rc = -3; break; }
    hipLaunchKernelGGL(swe_calib::k_fma_stream, dim3(nblk), dim3(256), lds, 0, out, spans, iters, 0.999999, 1e-7);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, nullptr) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess) { rc = -3; break; }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipMemcpy(h.data(), spans, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess) {
      rc = -3;
      break;
    }
    double cyc = 0.0, wt = 0.0;
    for (int i = 0; i < nwave; ++i) { cyc += (double)h[2 * i]; wt += (double)h[2 * i + 1]; }
    rate.push_back(flops / (ms * 1e-3) / 1e12);
    mhz.push_back(wt > 0 ? cyc / wt * wclk_khz * 1e-3 : 0.0);
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (el >= seconds && rate.size() >= 4) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  (void)hipFree(spans);
  if (rc != 0) return rc;
  const size_t half = rate.size() / 2;
  std::vector<double> r(rate.begin() + half, rate.end());
  std::sort(r.begin(), r.end());
  double m = 0.0;
  for (size_t i = half; i < mhz.size(); ++i) m += mhz[i];
  *tflops = r[r.size() / 2];
  *shader_mhz = m / (double)(mhz.size() - half);
  return 0;
}

}  // extern "C"
