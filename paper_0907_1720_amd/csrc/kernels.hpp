// Launchers of the HIP kernels (defined in kernels.hip; the kernels are in
// kernels_body.hpp, one instantiation per lattice size in kernels_q.hip).  All
// take device pointers.
#pragma once

#include "device.hpp"

// Kernel variants of the relaxation polynomial: (padded degree D, parity P).
// Dense (P = 0): D1Q5 KdV/KS/K(2,2) 5, cubic Pi 13, quartic Pi_1 up to 13;
// D1Q7 Kawahara 7, cubic Pi 13, quartic Pi_1 19.  Odd (P = 1): mKdV 9.  Power
// sums with real exponents (P = 2): degree 2, 5, 7 or 11 of each class's
// polynomial in phi^step (its strided layout); P = 3: the same for exactly the
// classes phi^0 and phi^(1/2), degree 2 or 5.
#define LBM_VARIANT_CASES \
  LBM_CASE(5, 0)          \
  LBM_CASE(7, 0)          \
  LBM_CASE(9, 0)          \
  LBM_CASE(13, 0)         \
  LBM_CASE(19, 0)         \
  LBM_CASE(5, 1)          \
  LBM_CASE(9, 1)          \
  LBM_CASE(13, 1)         \
  LBM_CASE(19, 1)         \
  LBM_CASE(2, 2)          \
  LBM_CASE(5, 2)          \
  LBM_CASE(7, 2)          \
  LBM_CASE(11, 2)         \
  LBM_CASE(2, 3)          \
  LBM_CASE(5, 3)

// dense degrees available to the initialisation kernel
#define LBM_INIT_CASES \
  LBM_CASE(5)          \
  LBM_CASE(7)          \
  LBM_CASE(9)          \
  LBM_CASE(13)         \
  LBM_CASE(19)

namespace lbm {

// smallest kernel degree >= D of the given parity (0 if none); parity 2 =
// power sums with real exponents
inline int padded_degree(int D, int parity) {
  const int dense[] = {5, 7, 9, 13, 19};
  const int odd[] = {5, 9, 13, 19};
  const int power_sum[] = {2, 5, 7, 11};
  const int half_powers[] = {2, 5};
  if (parity == 0) {
    for (int v : dense)
      if (v >= D) return v;
  } else if (parity == 2) {
    for (int v : power_sum)
      if (v >= D) return v;
  } else if (parity == 3) {
    for (int v : half_powers)
      if (v >= D) return v;
  } else {
    for (int v : odd)
      if (v >= D) return v;
  }
  return 0;
}
inline int variant_code(int D, int parity) { return D | (parity << 8); }

// prec: 0 = FP64 storage and arithmetic; 1 = FP32 deviation storage, FP64
// relaxation; 2 = FP32 deviation storage, FP32 relaxation.
hipError_t launch_init(int q, int D, int prec, const double* phi, void* f, int n, int stride,
                       const DevCoef* cf, hipStream_t s);
// slabs: one launch no larger than the GPU holds at once, one workgroup per
// slab; flags[0 .. nslabs) start at 0; xbuf holds 4 Q halo values per slab;
// a halo wait gives up after wait_ticks ticks of the wall clock (status bit
// 2); slab mute_slab (-1: none) never raises its flag (test hook)
hipError_t launch_slab(int q, int prec, int code, const DevSlab* slabs, int nslabs, const DevTileInst* tinsts,
                       void* buf0, void* buf1, int s_per, int halo, void* xbuf, int* flags, const DevCoef* coefs,
                       int* status, long long wait_ticks, int mute_slab, int block, size_t lds, hipStream_t s);
hipError_t slab_occupancy(int q, int prec, int code, int block, size_t lds, int* blocks_per_cu);
// bounded domains: reset `layers` (1..32) nodes at each end from phib[0 .. 2 layers)
// (kind 1 equilibrium, 2 non-equilibrium extrapolation); D = init degree
hipError_t launch_bound(int q, int D, int prec, void* f, int n, int stride, int layers, int kind,
                        const double* phib, const DevCoef* cf, hipStream_t s);
// `code` = variant_code(D, parity) of the relaxation polynomial
hipError_t launch_stream(int q, int code, int prec, const void* fin, void* fout, int n, int stride,
                         const DevCoef* cf, hipStream_t s);
// the fused collide+stream kernel of variant `code` (arguments: const T* fin,
// T* fout, int n, int stride, const DevCoef* cf; 256 threads per block), for
// graph nodes; nullptr for an unknown variant
const void* stream_kernel(int q, int code, int prec);
// persistent launch over `njobs` jobs (bin-packed instances of one variant
// `code`), each split into `nchunks` step chunks; done[0..njobs) starts at 0.
// code | (1 << 16) selects the kernel of bounded jobs (boundary layers reset
// in LDS after every step).  A chunk's wait for its predecessor gives up after
// wait_ticks ticks of the wall clock (status bit 4); queue item stall_item
// (-1: none) is taken but never run (test hook)
hipError_t launch_resident(int q, int prec, int code, const DevJob* jobs, const DevJobInst* jinst, int njobs,
                           int nchunks, int* counter, int* slots, int* done, const DevCoef* coefs, int* status,
                           long long wait_ticks, int stall_item, int grid, int block, size_t lds, hipStream_t s);
// VGPRs per thread of the resident kernel of variant `code`
int resident_vgprs(int q, int prec, int code);
// static LDS bytes of the resident kernel (0 by construction)
size_t resident_static_lds(int q, int prec, int code);
hipError_t launch_phi(int prec, const void* f, double* phi, int n, int stride, int q, double phi_rest,
                      int* nonfinite, hipStream_t s);
hipError_t launch_sum(const double* v, int n, double* part, int nparts, hipStream_t s);
hipError_t resident_occupancy(int q, int prec, int code, int block, size_t lds, int* blocks_per_cu);
// lbm_advance_noalloc: the fixed per-device scratch (tables at offset 0, the
// state from kNoAllocTableBytes on) and its device address on the current
// device (looked up once per device); a fill kernel that zeroes n ints
constexpr size_t kNoAllocTableBytes = size_t(16) << 10;
constexpr size_t kNoAllocStateBytes = size_t(256) << 10;
constexpr size_t kNoAllocScratchBytes = kNoAllocTableBytes + kNoAllocStateBytes;
hipError_t noalloc_scratch(void** out);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
// temporal blocking: launch `launch` of an advance, s_per steps per launch
hipError_t launch_tile(int q, int prec, const DevTile* tiles, int ntiles, const DevTileInst* tinsts, void* buf0,
                       void* buf1, int launch, int s_per, int halo, const DevCoef* coefs, int* status, int block,
                       size_t lds, hipStream_t s);

}  // namespace lbm
