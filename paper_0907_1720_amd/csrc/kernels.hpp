// Launchers of the HIP kernels (kernels.hip).  All take device pointers.
#pragma once

#include "device.hpp"

// Padded degrees of the equilibrium polynomials that have a kernel variant.
// D1Q5: KdV/KS/K(2,2) 5, mKdV 9, cubic Pi 13, quartic Pi_1 up to 13;
// D1Q7: Kawahara 7, cubic Pi 13, quartic Pi_1 19.
#define LBM_DEGREE_CASES(Q) \
  LBM_CASE(5)               \
  LBM_CASE(7)               \
  LBM_CASE(9)               \
  LBM_CASE(13)              \
  LBM_CASE(19)

namespace lbm {

// smallest kernel degree >= D (0 if none)
inline int padded_degree(int D) {
  const int menu[] = {5, 7, 9, 13, 19};
  for (int v : menu)
    if (v >= D) return v;
  return 0;
}

// prec: 0 = FP64 storage and arithmetic; 1 = FP32 deviation storage, FP64
// relaxation; 2 = FP32 deviation storage, FP32 relaxation.
hipError_t launch_init(int q, int D, int prec, const double* phi, void* f, int n, int stride,
                       const DevCoef* cf, hipStream_t s);
hipError_t launch_stream(int q, int D, int prec, const void* fin, void* fout, int n, int stride,
                         const DevCoef* cf, hipStream_t s);
hipError_t launch_resident(int q, int prec, const DevInst* items, int count, int* counter, int* slots,
                           void* state, const DevCoef* coefs, int* status, int grid, int block, size_t lds,
                           hipStream_t s);
// static LDS bytes of the resident kernel (0 by construction)
size_t resident_static_lds(int q, int prec);
hipError_t launch_phi(int prec, const void* f, double* phi, int n, int stride, int q, double phi_rest,
                      int* nonfinite, hipStream_t s);
hipError_t launch_sum(const double* v, int n, double* part, int nparts, hipStream_t s);
hipError_t resident_occupancy(int q, int prec, int block, size_t lds, int* blocks_per_cu);

}  // namespace lbm
