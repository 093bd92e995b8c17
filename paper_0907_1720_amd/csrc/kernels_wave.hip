// Boundary rows of travelling-wave exact solutions, evaluated on the device
// for the bounded boundaries of Sec. IV (the closed forms of its examples):
//   phi*(x, t) = a + b h(z)^p + d h(z)^r,  z = k (x - xc - c t),
// one value per (step, boundary node), in the row layout the bounded kernels
// read: row s (after step s + 1) holds the `layers` left nodes, then the
// `layers` right nodes.
#include "wave.hpp"

#include <cmath>

namespace lbm {
namespace {

constexpr double kHalfPi = 1.5707963267948966;

__device__ __forceinline__ double wave_shape(int shape, double z) {
  switch (shape) {
    case LBM_WAVE_SECH:
      return 1.0 / cosh(z);
    case LBM_WAVE_TANH:
      return tanh(z);
    case LBM_WAVE_LOGISTIC:
      return 1.0 / (1.0 + exp(z));
    default:   // LBM_WAVE_COS: a compacton, zero outside its support
      return fabs(z) <= kHalfPi ? cos(z) : 0.0;
  }
}

// h^e: ie >= 0 is the integer e (repeated products); ie < 0: pow(h, e), h >= 0
__device__ __forceinline__ double wave_power(double h, double e, int ie) {
  if (ie < 0) return pow(h, e);
  double v = 1.0;
  for (int i = 0; i < ie; ++i) v *= h;
  return v;
}

__global__ __launch_bounds__(256) void k_wave_rows(double* __restrict__ rows, int64_t total, int layers, int n,
                                                   double dx, double dt, lbm_wave w, int ip, int ir) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t s = idx / (2 * layers);
  const int k = (int)(idx - s * 2 * layers);
  const int node = k < layers ? k : n - 2 * layers + k;
  const double x = w.x_first + (double)node * dx;
  const double t = w.t0 + (double)(s + 1) * dt;
  const double z = w.k * (x - w.xc - w.c * t);
  const double h = wave_shape(w.shape, z);
  rows[idx] = w.a + w.b * wave_power(h, w.p, ip) + w.d * wave_power(h, w.r, ir);
}

// e itself when it is a whole number <= 64 (bounded before the conversion), else -1
int integer_exponent(double e) { return (e <= 64.0 && e == std::floor(e)) ? (int)e : -1; }

}  // namespace

hipError_t launch_wave_rows(double* rows, int64_t steps, int layers, int n, double dx, double dt,
                            const lbm_wave& w, hipStream_t s) {
  const int64_t total = steps * 2 * layers;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_wave_rows, dim3((unsigned)blocks), dim3(256), 0, s, rows, total, layers, n, dx, dt, w,
                     integer_exponent(w.p), integer_exponent(w.r));
  return hipGetLastError();
}

}  // namespace lbm
