// Stage combination of the explicit Runge-Kutta integrators with a Butcher
// tableau (RK4, Bogacki-Shampine 3(2), Tsitouras 5(4), the integrators the
// paper's tables name): out = u + dt sum_j a_j K_j over the stage right-hand
// sides K_j, elementwise over the flat state.  dt is read on the device (the
// CFL pass writes it there).  HBM-bound: each element is read from u and from
// the n stage buffers once and written once.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace frsg {
namespace {

constexpr int kRkBlock = 256;

__global__ void __launch_bounds__(kRkBlock) k_rk_combine(const double* __restrict__ u, RkTerms T,
                                                         const double* __restrict__ dt, double* out, long n) {
  const double h = *dt;
  for (long i = blockIdx.x * (long)kRkBlock + threadIdx.x; i < n; i += (long)gridDim.x * kRkBlock) {
    double acc = 0.0;
    for (int j = 0; j < T.n; ++j) acc = acc + T.a[j] * T.K[j][i];
    out[i] = u[i] + h * acc;
  }
}

__global__ void __launch_bounds__(kRkBlock) k_or_flags(unsigned char* dst, const unsigned char* __restrict__ src,
                                                       long n) {
  const long i = blockIdx.x * (long)kRkBlock + threadIdx.x;
  if (i < n) dst[i] = (unsigned char)(dst[i] | src[i]);
}

}  // namespace

hipError_t launch_rk_combine(const double* u, const RkTerms& T, const double* dt, double* out, long n,
                             hipStream_t s) {
  if (T.n < 0 || T.n > kRkMaxTerms) return hipErrorInvalidValue;
  // a grid of a few waves per CU, each thread striding over the state
  long blocks = (n + kRkBlock - 1) / kRkBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_rk_combine, dim3((unsigned)blocks), dim3(kRkBlock), 0, s, u, T, dt, out, n);
  return hipGetLastError();
}

hipError_t launch_or_flags(unsigned char* dst, const unsigned char* src, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_or_flags, dim3((unsigned)((n + kRkBlock - 1) / kRkBlock)), dim3(kRkBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace frsg
