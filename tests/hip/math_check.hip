// Test infrastructure: the exact build's reciprocal and square root (MRCP,
// MSQRT of mlswe_device.hpp) against the GPU's general IEEE division and
// square root, and against the host's, bit for bit, on caller-given operands.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "mlswe_device.hpp"

namespace {
using namespace mlswe;

__global__ void k_math(const double* __restrict__ x, double* __restrict__ o, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  o[4 * i + 0] = MRCP(v);
  o[4 * i + 1] = 1.0 / v;
  o[4 * i + 2] = MSQRT(v);
  o[4 * i + 3] = __builtin_sqrt(v);
}

bool same(double a, double b) {
  if (std::isnan(a) && std::isnan(b)) return true;
  uint64_t ua, ub;
  std::memcpy(&ua, &a, 8);
  std::memcpy(&ub, &b, 8);
  return ua == ub;
}

}  // namespace

// counts[0]: reciprocals differing from the GPU's 1/x, [1]: square roots
// differing from the GPU's sqrt, [2] / [3]: the same against the host's.
// Returns 0, or a HIP error code.
extern "C" int math_check(const double* x, long long n, long long* counts) {
  for (int k = 0; k < 4; ++k) counts[k] = 0;
  if (n <= 0) return 0;
  double *dx = nullptr, *dout = nullptr;
  hipError_t e = hipMalloc(&dx, n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&dout, 4 * n * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(dx, x, n * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_math, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, dx, dout, n);
    e = hipGetLastError();
  }
  std::vector<double> o(4 * (size_t)n);
  if (e == hipSuccess) e = hipMemcpy(o.data(), dout, 4 * n * sizeof(double), hipMemcpyDeviceToHost);
  if (dx) (void)hipFree(dx);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return (int)e;
  for (long long i = 0; i < n; ++i) {
    const double v = x[i];
    counts[0] += !same(o[4 * i + 0], o[4 * i + 1]);
    counts[1] += !same(o[4 * i + 2], o[4 * i + 3]);
    counts[2] += !same(o[4 * i + 0], 1.0 / v);
    counts[3] += !same(o[4 * i + 2], std::sqrt(v));
  }
  return 0;
}
