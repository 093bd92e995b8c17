// Read-out kernels and the host launchers of every kernel; the lattice step
// itself is in kernels_body.hpp, instantiated per lattice size by
// kernels_q.hip (tables q_kernels_4 .. q_kernels_7).
//
//  k_phi       phi = sum_j f_j  (FP64)
//  k_sum       FP64 sum of phi over a grid, deterministic two-pass
#include <mutex>
#include <unordered_map>

#include "kernels.hpp"
#include "kernels_table.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// read-outs
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_phi(const T* __restrict__ f, double* __restrict__ phi, int n,
                                             int stride, int q, double phi_rest,
                                             int* __restrict__ nonfinite) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
  double s = (double)f[x];
  for (int j = 1; j < q; ++j) s += (double)f[(int64_t)j * stride + x];
  s += phi_rest;
  phi[x] = s;
  if (!__builtin_isfinite(s)) atomicOr(nonfinite, 1);
}

__global__ __launch_bounds__(256) void k_sum_partial(const double* __restrict__ v, int n,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {
const QKernels* table(int q) {
  switch (q) {
    case 4: return &q_kernels_4;
    case 5: return &q_kernels_5;
    case 6: return &q_kernels_6;
    case 7: return &q_kernels_7;
  }
  return nullptr;
}

const void* resident_kernel(int q, int prec, int code) {
  const QKernels* t = table(q);
  return t ? t->resident_fn(prec, code) : nullptr;
}

const void* tile_kernel(int q, int prec) {
  const QKernels* t = table(q);
  return t ? t->tile_fn(prec) : nullptr;
}

const void* slab_kernel(int q, int prec, int code) {
  const QKernels* t = table(q);
  return t ? t->slab_fn(prec, code) : nullptr;
}
}  // namespace

hipError_t launch_init(int q, int D, int prec, const double* phi, void* f, int n, int stride,
                       const DevCoef* cf, hipStream_t s) {
  const QKernels* t = table(q);
  return t ? t->init(D, prec, phi, f, n, stride, cf, s) : hipErrorInvalidValue;
}

hipError_t launch_bound(int q, int D, int prec, void* f, int n, int stride, int layers, int kind,
                        const double* phib, const DevCoef* cf, hipStream_t s) {
  if (layers < 1 || 2 * layers > 64) return hipErrorInvalidValue;
  const QKernels* t = table(q);
  return t ? t->bound(D, prec, f, n, stride, layers, kind, phib, cf, s) : hipErrorInvalidValue;
}

hipError_t launch_stream(int q, int D, int prec, const void* fin, void* fout, int n, int stride,
                         const DevCoef* cf, hipStream_t s) {
  // D carries the variant code (degree | parity << 8)
  const QKernels* t = table(q);
  return t ? t->stream(D, prec, fin, fout, n, stride, cf, s) : hipErrorInvalidValue;
}

const void* stream_kernel(int q, int code, int prec) {
  const QKernels* t = table(q);
  return t ? t->stream_fn(prec, code) : nullptr;
}

hipError_t launch_resident(int q, int prec, int code, const DevJob* jobs, const DevJobInst* jinst, int njobs,
                           int nchunks, int* counter, int* slots, int* done, const DevCoef* coefs, int* status,
                           long long wait_ticks, int stall_item, int grid, int block, size_t lds, hipStream_t s) {
  const void* fn = resident_kernel(q, prec, code);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&jobs,  (void*)&jinst, (void*)&njobs, (void*)&nchunks,    (void*)&counter,  (void*)&slots,
                  (void*)&done,  (void*)&coefs, (void*)&status, (void*)&wait_ticks, (void*)&stall_item};
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, s);
}

namespace {
// kernel attributes, queried once per kernel (the planner asks per instance)
bool kernel_attributes(const void* fn, hipFuncAttributes* out) {
  static std::mutex mu;
  static std::unordered_map<const void*, hipFuncAttributes> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(fn);
  if (it == cache.end()) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, fn) != hipSuccess) return false;
    it = cache.emplace(fn, a).first;
  }
  *out = it->second;
  return true;
}
}  // namespace

int resident_vgprs(int q, int prec, int code) {
  hipFuncAttributes a;
  const void* fn = resident_kernel(q, prec, code);
  if (!fn || !kernel_attributes(fn, &a) || a.numRegs <= 0) return 128;
  return a.numRegs;
}

size_t resident_static_lds(int q, int prec, int code) {
  hipFuncAttributes a;
  const void* fn = resident_kernel(q, prec, code);
  if (!fn || !kernel_attributes(fn, &a)) return 1024;
  return a.sharedSizeBytes;
}

hipError_t launch_tile(int q, int prec, const DevTile* tiles, int ntiles, const DevTileInst* tinsts, void* buf0,
                       void* buf1, int launch, int s_per, int halo, const DevCoef* coefs, int* status, int block,
                       size_t lds, hipStream_t s) {
  const void* fn = tile_kernel(q, prec);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&tiles, (void*)&tinsts, (void*)&buf0, (void*)&buf1, (void*)&launch, (void*)&s_per,
                  (void*)&halo,  (void*)&coefs,  (void*)&status};
  return hipLaunchKernel(fn, dim3(ntiles), dim3(block), args, lds, s);
}

hipError_t launch_slab(int q, int prec, int code, const DevSlab* slabs, int nslabs, const DevTileInst* tinsts, void* buf0,
                       void* buf1, int s_per, int halo, void* xbuf, int* flags, const DevCoef* coefs, int* status,
                       long long wait_ticks, int mute_slab, int block, size_t lds, hipStream_t s) {
  const void* fn = slab_kernel(q, prec, code);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&slabs, (void*)&tinsts, (void*)&buf0,  (void*)&buf1,   (void*)&s_per,
                  (void*)&halo,  (void*)&xbuf,   (void*)&flags, (void*)&coefs,  (void*)&status,
                  (void*)&wait_ticks, (void*)&mute_slab};
  return hipLaunchKernel(fn, dim3(nslabs), dim3(block), args, lds, s);
}

hipError_t slab_occupancy(int q, int prec, int code, int block, size_t lds, int* blocks_per_cu) {
  const void* fn = slab_kernel(q, prec, code);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, lds);
}

hipError_t resident_occupancy(int q, int prec, int code, int block, size_t lds, int* blocks_per_cu) {
  const void* fn = resident_kernel(q, prec, code);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, lds);
}

hipError_t launch_phi(int prec, const void* f, double* phi, int n, int stride, int q, double phi_rest,
                      int* nonfinite, hipStream_t s) {
  if (prec == 0)
    k_phi<double><<<(n + 255) / 256, 256, 0, s>>>((const double*)f, phi, n, stride, q, phi_rest, nonfinite);
  else
    k_phi<float><<<(n + 255) / 256, 256, 0, s>>>((const float*)f, phi, n, stride, q, phi_rest, nonfinite);
  return hipGetLastError();
}

hipError_t launch_sum(const double* v, int n, double* part, int nparts, hipStream_t s) {
  k_sum_partial<<<nparts, 256, 0, s>>>(v, n, part);
  return hipGetLastError();
}

}  // namespace lbm
