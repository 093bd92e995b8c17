// The kernels of one lattice size, LBM_Q = 4, 5, 6 or 7 (set by the build):
// instantiates the templates of kernels_body.hpp for that q and exports their
// launchers as the table q_kernels_<q>.  `prec` selects (storage, arithmetic):
// 0 (double, double), 1 (float, double), 2 (float, float).
#include "kernels_body.hpp"
#include "kernels_table.hpp"

#ifndef LBM_Q
#error "LBM_Q (the lattice size) must be defined"
#endif
#define LBM_CAT2(a, b) a##b
#define LBM_CAT(a, b) LBM_CAT2(a, b)

namespace lbm {
namespace {
template <int Q, typename T>
hipError_t launch_init_q(int D, const double* phi, T* f, int n, int stride, const DevCoef* cf,
                         hipStream_t s) {
  dim3 grid((n + 255) / 256);
  switch (D) {
#define LBM_CASE(DD) \
  case DD:           \
    k_init<Q, DD, T><<<grid, 256, 0, s>>>(phi, f, n, stride, cf); \
    return hipGetLastError();
    LBM_INIT_CASES
#undef LBM_CASE
  }
  return hipErrorInvalidValue;
}

template <int Q, typename T, typename A>
hipError_t launch_stream_q(int code, const T* fin, T* fout, int n, int stride, const DevCoef* cf,
                           hipStream_t s) {
  dim3 grid((n + 255) / 256);
  switch (code) {
#define LBM_CASE(DD, PP)                                                         \
  case DD | (PP << 8):                                                           \
    k_stream<Q, DD, PP, T, A><<<grid, 256, 0, s>>>(fin, fout, n, stride, cf); \
    return hipGetLastError();
    LBM_VARIANT_CASES
#undef LBM_CASE
  }
  return hipErrorInvalidValue;
}

template <int Q, typename T, typename A>
const void* stream_fn(int code) {
  switch (code) {
#define LBM_CASE(DD, PP) \
  case DD | (PP << 8):   \
    return (const void*)k_stream<Q, DD, PP, T, A>;
    LBM_VARIANT_CASES
#undef LBM_CASE
  }
  return nullptr;
}

template <int Q, typename T, typename A>
const void* resident_fn(int code) {
  switch (code) {
#define LBM_CASE(DD, PP) \
  case DD | (PP << 8):   \
    return (const void*)k_resident<Q, DD, PP, T, A, false>;
    LBM_VARIANT_CASES
#undef LBM_CASE
#define LBM_CASE(DD, PP)            \
  case DD | (PP << 8) | (1 << 16): \
    return (const void*)k_resident<Q, DD, PP, T, A, true>;
    LBM_VARIANT_CASES
#undef LBM_CASE
  }
  return nullptr;
}

template <int Q>
const void* resident_prec(int prec, int code) {
  if (prec == 0) return resident_fn<Q, double, double>(code);
  if (prec == 1) return resident_fn<Q, float, double>(code);
  return resident_fn<Q, float, float>(code);
}

template <int Q>
hipError_t launch_init_p(int D, int prec, const double* phi, void* f, int n, int stride, const DevCoef* cf,
                         hipStream_t s) {
  if (prec == 0) return launch_init_q<Q, double>(D, phi, (double*)f, n, stride, cf, s);
  return launch_init_q<Q, float>(D, phi, (float*)f, n, stride, cf, s);
}

template <int Q, typename T>
hipError_t launch_bound_q(int D, T* f, int n, int stride, int layers, int kind, const double* phib,
                          const DevCoef* cf, hipStream_t s) {
  switch (D) {
#define LBM_CASE(DD) \
  case DD:           \
    k_bound<Q, DD, T><<<1, 64, 0, s>>>(f, n, stride, layers, kind, phib, cf); \
    return hipGetLastError();
    LBM_INIT_CASES
#undef LBM_CASE
  }
  return hipErrorInvalidValue;
}

template <int Q>
hipError_t launch_bound_p(int D, int prec, void* f, int n, int stride, int layers, int kind, const double* phib,
                          const DevCoef* cf, hipStream_t s) {
  if (prec == 0) return launch_bound_q<Q, double>(D, (double*)f, n, stride, layers, kind, phib, cf, s);
  return launch_bound_q<Q, float>(D, (float*)f, n, stride, layers, kind, phib, cf, s);
}

template <int Q>
hipError_t launch_stream_p(int D, int prec, const void* fin, void* fout, int n, int stride, const DevCoef* cf,
                           hipStream_t s) {
  if (prec == 0) return launch_stream_q<Q, double, double>(D, (const double*)fin, (double*)fout, n, stride, cf, s);
  if (prec == 1) return launch_stream_q<Q, float, double>(D, (const float*)fin, (float*)fout, n, stride, cf, s);
  return launch_stream_q<Q, float, float>(D, (const float*)fin, (float*)fout, n, stride, cf, s);
}

template <int Q>
const void* stream_prec(int prec, int code) {
  if (prec == 0) return stream_fn<Q, double, double>(code);
  if (prec == 1) return stream_fn<Q, float, double>(code);
  return stream_fn<Q, float, float>(code);
}

template <int Q, typename T, typename A>
const void* tile_fn() { return (const void*)k_tile<Q, T, A>; }
template <int Q>
const void* tile_prec(int prec) {
  if (prec == 0) return tile_fn<Q, double, double>();
  if (prec == 1) return tile_fn<Q, float, double>();
  return tile_fn<Q, float, float>();
}

template <int Q, typename T, typename A>
const void* slab_fn(int code) {
  switch (code) {
#define LBM_CASE(DD, PP) \
  case DD | (PP << 8):   \
    return (const void*)k_slab<Q, DD, PP, T, A>;
    LBM_VARIANT_CASES
#undef LBM_CASE
  }
  return nullptr;
}
template <int Q>
const void* slab_prec(int prec, int code) {
  if (prec == 0) return slab_fn<Q, double, double>(code);
  if (prec == 1) return slab_fn<Q, float, double>(code);
  return slab_fn<Q, float, float>(code);
}
}  // namespace

QKernels LBM_CAT(q_kernels_, LBM_Q) = {
    &launch_init_p<LBM_Q>, &launch_bound_p<LBM_Q>, &launch_stream_p<LBM_Q>, &stream_prec<LBM_Q>,
    &resident_prec<LBM_Q>, &tile_prec<LBM_Q>,      &slab_prec<LBM_Q>,
};

}  // namespace lbm
