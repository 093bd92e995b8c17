// Launch entry points of the kernels of one lattice size, one table per
// lattice (kernels_q.hip, built once for each q in 4..7).
#pragma once

#include "device.hpp"

namespace lbm {

struct QKernels {
  hipError_t (*init)(int D, int prec, const double* phi, void* f, int n, int stride, const DevCoef* cf,
                     hipStream_t s);
  hipError_t (*bound)(int D, int prec, void* f, int n, int stride, int layers, int kind, const double* phib,
                      const DevCoef* cf, hipStream_t s);
  hipError_t (*stream)(int code, int prec, const void* fin, void* fout, int n, int stride, const DevCoef* cf,
                       hipStream_t s);
  const void* (*stream_fn)(int prec, int code);
  const void* (*resident_fn)(int prec, int code);
  const void* (*tile_fn)(int prec);
  const void* (*slab_fn)(int prec, int code);
};

// host-side tables (not const: a const table would also be emitted for the
// device, where its host function pointers do not exist)
extern QKernels q_kernels_4, q_kernels_5, q_kernels_6, q_kernels_7;

}  // namespace lbm
