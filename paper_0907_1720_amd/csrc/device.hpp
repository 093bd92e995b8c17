// Device-side data structures and the per-node collision shared by every
// kernel (so all kernel paths give bitwise identical results).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbm {

constexpr int kRow = 20;   // coefficient row length (max degree 19 + 1)

// Per-problem constants on the device.
struct DevCoef {
  double w0;                 // 1 - omega
  double phi_rest;           // rest state (F32 deviation storage); 0 for FP64
  double f_rest[8];
  double wG[8][kRow];        // FP64: omega * G[j][d];  F32-dev: omega * H[j][d] (d >= 1)
  double G[8][kRow];         // FP64: G[j][d];          F32-dev: H[j][d]   (for f := f_eq(phi))
  float w0f;
  float pad_[3];
  float wHf[8][kRow];        // F32-dev: omega * H[j][d] rounded to float
};

// Per-instance launch record of the batched kernels.
struct DevInst {
  int64_t off;               // element offset of row 0 in the state array of its precision
  int32_t n;                 // nodes
  int32_t stride;            // row stride in elements
  int32_t steps;             // steps to run in this launch
  int32_t degree;            // padded degree D of the kernel variant
  int32_t q;
  int32_t inst;              // index into coefficients / status
};

__host__ __device__ constexpr int velocity(int j) {
  return j == 0 ? 0 : ((j & 1) ? (j + 1) / 2 : -(j / 2));
}
// population with the opposite velocity
__host__ __device__ constexpr int opposite(int j) {
  return j == 0 ? 0 : ((j & 1) ? j + 1 : j - 1);
}

// ---- a1 + a2 + a3 + a4: phi = sum_j f_j, f_eq_j(phi) by Horner, BGK ----
//
// Storage type T, arithmetic type A.  The zeroth moment is always summed in
// FP64.  With FP64 storage the polynomials are G (f_eq_j(phi) = sum_d G phi^d);
// with FP32 deviation storage g = f - f_rest they are H, the Taylor shift of
// G about the rest state (f_eq_j(phi_rest + delta) - f_rest_j = sum_d H delta^d,
// H[j][0] = 0), so the same code serves both:
//     f*_j = w0 f_j + sum_d (omega C[j][d]) s^d,   s = sum_j f_j,  w0 = 1 - omega.
__device__ __forceinline__ double fma_a(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_a(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int Q, int D, typename T, typename A>
__device__ __forceinline__ void collide(T (&f)[Q], const A* __restrict__ wc, A w0) {
  double s = (double)f[0];
#pragma unroll
  for (int j = 1; j < Q; ++j) s += (double)f[j];
  const A p = (A)s;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    A acc = wc[j * kRow + D];
#pragma unroll
    for (int d = D - 1; d >= 0; --d) acc = fma_a(acc, p, wc[j * kRow + d]);
    f[j] = (T)fma_a(w0, (A)f[j], acc);
  }
}

template <typename A> struct CoefView;
template <> struct CoefView<double> {
  __device__ static const double* relax(const DevCoef* c) { return &c->wG[0][0]; }
  __device__ static double w0(const DevCoef* c) { return c->w0; }
};
template <> struct CoefView<float> {
  __device__ static const float* relax(const DevCoef* c) { return &c->wHf[0][0]; }
  __device__ static float w0(const DevCoef* c) { return c->w0f; }
};

}  // namespace lbm
