// Device-side data structures and the per-node collision shared by every
// kernel (so all kernel paths give bitwise identical results).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbm {

constexpr int kRow = 20;   // coefficient row length (max degree 19 + 1)
constexpr int kGRow = 12;  // power-sum tables: integer degree <= 11 per class
constexpr int kGCls = 4;   // power-sum tables: fractional-power classes

// Slots per node in LDS: the lattice size, padded to an odd number (D1Q4 and
// D1Q6 rows take 5 and 7 slots) so that consecutive nodes on consecutive lanes
// fall on distinct LDS banks.
constexpr int lds_stride(int q) { return q | 1; }

// Per-problem constants on the device.
struct DevCoef {
  double w0;                 // 1 - omega
  double s0;                 // added to sum_j g_j before odd tables: phi_rest (FP32 storage, FP64 relaxation)
  double phi_rest;           // rest state of the FP32 deviation storage (0 for FP64 storage)
  double cst[8];             // added after relaxation: 0, or -omega f_rest_j (FP32 storage, FP64 relaxation)
  double wc[8][kRow];        // FP64 relaxation: omega * G[j][d] over the kept degrees (all, or odd only);
                             // omega * H[j][d] for dense tables with FP32 deviation storage
  double init[8][kRow];      // f := f_eq(phi): G[j][d] (FP64 storage) or H[j][d] (FP32 deviations)
  float w0f;
  float pad_[3];
  float wHf[8][kRow];        // FP32 relaxation: omega * H[j][d], H = G shifted to the rest state
  // Equilibria with real (non-integer) powers of phi (variant parity 2, or 3
  // for the two classes phi^0 and phi^(1/2)):
  //   f_eq_j(phi) = sum_{c < gF} phi^gnu[c] sum_d G[c][j][d] phi^d
  int32_t gF;                // classes; 0 for polynomial equilibria
  int32_t groots;            // 1: every gnu is 1/2, 1/4 or 3/4 (square roots suffice, no log2)
  int32_t gd0[kGCls];        // class c's nonzero degrees are gd0[c] + gstep[c] i
  int32_t gstep[kGCls];
  double gnu[kGCls];         // gnu[0] = 0, the rest the fractional parts of the exponents
  double grest[8];           // f_rest_j subtracted at initialisation (FP32 deviations), else 0
  double gwc[kGCls][7][kGRow];    // omega * G[c][j][gd0[c] + gstep[c] i] at [c][j][i] (relaxation)
  double ginit[kGCls][7][kGRow];  // G[c][j][d] (initialisation and boundary layers)
};

// Resident path: a job is the set of instances one workgroup advances side by
// side (same step count); each instance owns a wave-aligned range of the
// workgroup's threads and a region of its LDS.
struct DevJob {
  int32_t first;             // first DevJobInst of the job
  int32_t count;             // instances in the job (<= 16)
  int32_t steps;             // steps of this launch
  int32_t degree;            // kernel variant shared by all instances of the job
  int32_t bounded;           // 1: the instances reset their boundary layers after every step
  int32_t pad_;
};
struct DevJobInst {
  uint64_t addr;             // device address of row 0 of the instance's current state
  uint64_t phib;             // bounded: device address of phi* at the outer layers for the
                             // launch's first step, [steps][2 layers] (left, then right); else 0
  int32_t n;                 // nodes
  int32_t stride;            // row stride in elements
  int32_t degree;            // kernel variant: padded degree D | (parity << 8)
  int32_t inst;              // index into coefficients / status
  int32_t lds_off;           // element offset of the instance's LDS region
  int32_t t0;                // first thread (multiple of 64)
  int32_t nt;                // threads (multiple of 64)
  int32_t bkind;             // 0 periodic, 1 equilibrium layers, 2 non-equilibrium extrapolation
  int32_t layers;            // boundary layers at each end (bounded)
  int32_t pad_;
};

// Slab path: an instance split over several co-resident workgroups (one slab
// each) that exchange halo strips every s steps; ring neighbours by index.
struct DevSlab {
  int32_t ti;                // index into the DevTileInst table
  int32_t x0;                // first core node
  int32_t core;              // core nodes (>= halo)
  int32_t left;              // slab (workgroup) holding the nodes left of x0, periodic
  int32_t right;             // slab holding the nodes from x0 + core on
  int32_t pad_;
};

// Tiled path: one record per tile (workgroup) and one per instance.
struct DevTile {
  int32_t ti;                // index into the DevTileInst table
  int32_t x0;                // first core node
  int32_t core;              // core nodes written back by this tile
  int32_t pad_;
};
struct DevTileInst {
  int64_t off;               // element offset of row 0 in both state buffers
  int32_t n;
  int32_t stride;
  int32_t steps;             // steps of this advance (all launches)
  int32_t cur0;              // state buffer holding the input of the first launch
  int32_t degree;            // kernel variant code
  int32_t inst;              // index into coefficients / status
};

// Lattice velocities e_j in units of c.  Odd q (D1Q5, D1Q7) has the rest
// velocity first: e = (0, 1, -1, 2, -2, 3, -3); even q (D1Q4, D1Q6) has none:
// e = (1, -1, 2, -2, 3, -3).  Either way max |e_j| = q / 2.
template <int Q>
__host__ __device__ constexpr int velocity(int j) {
  if constexpr (Q % 2 == 1) return j == 0 ? 0 : ((j & 1) ? (j + 1) / 2 : -(j / 2));
  else return (j & 1) ? -(j / 2 + 1) : (j / 2 + 1);
}
// population with the opposite velocity
template <int Q>
__host__ __device__ constexpr int opposite(int j) {
  if constexpr (Q % 2 == 1) return j == 0 ? 0 : ((j & 1) ? j + 1 : j - 1);
  else return j ^ 1;
}

// ---- a1 + a2 + a3 + a4: phi = sum_j f_j, f_eq_j(phi) by Horner, BGK ----
//
// Storage type T, arithmetic type A; the zeroth moment is always summed in
// FP64.  Three precisions share this code:
//  * FP64 storage:  f*_j = w0 f_j + sum_d (omega G[j][d]) phi^d
//  * FP32 deviations g = f - f_rest, FP64 relaxation (kRest): dense tables
//        delta = sum_j g_j,  g*_j = w0 g_j + sum_{d>=1} (omega H[j][d]) delta^d
//    with H the Taylor shift of G to the rest state; odd tables keep their
//    parity in phi = phi_rest + delta:
//        g*_j = w0 g_j + sum_d (omega G[j][d]) phi^d - omega f_rest_j
//  * FP32 deviations, FP32 relaxation: delta = sum_j g_j,
//        g*_j = w0 g_j + sum_d (omega H[j][d]) delta^d  with H the Taylor shift
//        of G to the rest state (H[j][0] = 0)
// Parity P = 1 marks equilibria that are odd in phi (every kept degree odd,
// e.g. mKdV): coefficient k belongs to degree 2k+1 and Horner runs in phi^2.
// P = 2 marks equilibria with real powers of phi (power sums, in FP64 with
// phi^nu from square roots when every nu is 1/2, 1/4 or 3/4, else
// exp2(nu log2 phi); phi >= 0; FP32 storage relaxes in phi itself and adds
// -omega f_rest like the odd tables).
__device__ __forceinline__ double fma_a(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_a(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// a * b + c with c a wave-uniform value in scalar registers, as one VOP3 FMA
// with a scalar operand (the compiler otherwise copies c to vector registers
// to use the two-address form)
__device__ __forceinline__ double fma_s(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
#else
  return __builtin_fma(a, b, c);
#endif
}
__device__ __forceinline__ float fma_s(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int D, int P, typename A>
__device__ __forceinline__ A poly_eval(const A* __restrict__ c, A p) {
  if constexpr (P == 0) {
    A acc = c[D];
#pragma unroll
    for (int d = D - 1; d >= 0; --d) acc = fma_a(acc, p, c[d]);
    return acc;
  } else {
    constexpr int K = (D + 1) / 2;   // degrees 1, 3, ..., D
    const A u = p * p;
    A acc = c[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) acc = fma_a(acc, u, c[k]);
    return acc * p;
  }
}

// Per-thread relaxation constants.  The leading coefficient of each
// polynomial is pinned to a VGPR so that every Horner step is a single FMA
// with at most one scalar operand.
// phi^nu for a fractional class: the square roots for nu = 1/2, 1/4, 3/4
// (correctly rounded, a few instructions), else exp2(nu log2 phi); phi >= 0
__device__ __forceinline__ double frac_pow(double nu, double phi, double lg, bool roots) {
  if (roots) {
    const double r = __builtin_sqrt(phi);
    if (nu == 0.5) return r;
    const double r4 = __builtin_sqrt(r);
    return nu == 0.25 ? r4 : r * r4;
  }
  return exp2(nu * lg);
}

// x^k for a small wave-uniform k >= 0 (k - 1 products; x^0 = 1)
__device__ __forceinline__ double int_pow(double x, int k) {
  if (k == 0) return 1.0;
  double r = x;
  for (int i = 1; i < k; ++i) r *= x;
  return r;
}

// V: the kernel's registers are spent on the node loop (the periodic resident
// and slab kernels): coefficients are then pinned to registers as below.
// Kernels that keep other state live across the loop (the bounded resident
// kernels, the tiles that serve every variant) read them from the table.
template <int Q, int D, int P, typename T, typename A, bool V = false>
struct Relaxer {
  static constexpr int K = P == 0 ? D + 1 : (D + 1) / 2;   // coefficients per population
  static constexpr bool kRest = (sizeof(T) == 4 && sizeof(A) == 8);
  // the lower coefficients are held in scalar registers when they fit, so that
  // every code path of a kernel (the node loop, a masked or wrapped node) reads
  // the same registers instead of reloading the table
  static constexpr bool kPin = V && P < 2 && Q * (K - 1) * (int)sizeof(A) / 4 <= 52;
  // Larger tables keep their highest kNV coefficients per population in vector
  // registers, enough that the rest (read as scalar operands) leave the kernel
  // scalar registers for its own state: otherwise the node loop's operands
  // push that state out to vector-register lanes and every step reloads it.
  // (at most three per population: tables that would need more keep one)
  static constexpr int nv_for_table() {
    if (!V || P >= 2 || kPin) return 1;
    for (int nv = 2; nv <= 3 && nv < K; ++nv)
      if (Q * (K - nv) * (int)sizeof(A) / 4 <= 70) return nv;
    return 1;
  }
  static constexpr int kNV = nv_for_table();
  // Tables too large for either scheme (a dense degree-13 D1Q7 table in FP64:
  // 7 x 13 x 2 words below the top coefficients) are read from the constant
  // cache at every update, a population at a time (dense tables only): held
  // across the node loop they spilled to vector-register lanes, two lane reads
  // per FMA (213 VALU instructions per node in the D1Q7 degree-13 loop, 107
  // now).
  static constexpr bool kReload =
      V && P < 2 && !kPin && kNV == 1 && Q * (K - 1) * (int)sizeof(A) / 4 > 70;
  using CT = const __attribute__((address_space(4))) A*;
  // coefficients loaded together: a population's, at most 13
  static constexpr int kGroup = K - 1 < 13 ? (K - 1 > 0 ? K - 1 : 1) : 13;
  const A* __restrict__ c;   // [Q][kRow]: dense, or the odd degrees compacted
  const DevCoef* __restrict__ cfp;   // power-sum tables (P = 2)
  A top[Q];
  A topv[kNV > 1 ? kNV - 1 : 1][Q];   // coefficients K - 2, ..., K - kNV
  A low[kPin ? Q : 1][kPin ? K - 1 : 1];
  A add[kPin && kRest && P == 1 ? Q : 1];   // -omega f_rest_j of the odd tables (FP32 storage)
  A w0;
  double s0;                 // phi_rest (odd tables with FP32 storage)
  const double* __restrict__ cst;

  __device__ __forceinline__ void init(const A* __restrict__ coef, A w0_, const DevCoef* __restrict__ cf) {
    c = coef;
    cfp = cf;
    w0 = w0_;
    s0 = cf->s0;
    cst = cf->cst;
    if constexpr (P < 2) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        top[j] = c[j * kRow + K - 1];
        asm volatile("" : "+v"(top[j]));
#pragma unroll
        for (int v = 0; v + 1 < kNV; ++v) {
          topv[v][j] = c[j * kRow + K - 2 - v];
          asm volatile("" : "+v"(topv[v][j]));
        }
      }
    }
    if constexpr (kPin) {
#pragma unroll
      for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int d = 0; d < K - 1; ++d) {
          low[j][d] = c[j * kRow + d];
#if defined(__HIP_DEVICE_COMPILE__)
          asm volatile("" : "+s"(low[j][d]));   // device pass only: a register class of the GPU
#endif
        }
      if constexpr (kRest && P == 1) {
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          add[j] = (A)cst[j];
#if defined(__HIP_DEVICE_COMPILE__)
          asm volatile("" : "+s"(add[j]));   // device pass only: a register class of the GPU
#endif
        }
      }
    }
  }
  __device__ __forceinline__ A odd_add(int j) const {
    if constexpr (!kRest)
      return (A)0;
    else if constexpr (kPin)
      return add[j];
    else
      return (A)cst[j];
  }
  __device__ __forceinline__ A coef(int j, int d) const {
    if constexpr (kPin)
      return low[j][d];
    else if (d > K - 1 - kNV)
      return topv[K - 2 - d][j];
    else
      return c[j * kRow + d];
  }

  __device__ __forceinline__ void operator()(T (&f)[Q]) const {
    double s = (double)f[0];
    if constexpr ((kRest && P == 1) || (sizeof(T) == 4 && P >= 2)) s = s0 + s;
#pragma unroll
    for (int j = 1; j < Q; ++j) s += (double)f[j];
    const A p = (A)s;
    if constexpr (P == 2) {
      // class c contributes phi^(gnu[c] + gd0[c]) times a polynomial of
      // degree <= D in phi^gstep[c] (Horner), so that only the degrees the
      // class can hold are evaluated
      const DevCoef* __restrict__ g = cfp;
      const bool roots = g->groots != 0;
      const double lg = roots ? 0.0 : log2(s);
      double acc[Q];
      {
        const double w = int_pow(s, g->gstep[0]);
        const double base = int_pow(s, g->gd0[0]);
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          double a = g->gwc[0][j][D];
#pragma unroll
          for (int d = D - 1; d >= 0; --d) a = __builtin_fma(a, w, g->gwc[0][j][d]);
          acc[j] = base * a;
        }
      }
      const int F = g->gF;
#pragma unroll
      for (int cl = 1; cl < kGCls; ++cl) {
        if (cl < F) {
          const double w = int_pow(s, g->gstep[cl]);
          const double base = frac_pow(g->gnu[cl], s, lg, roots) * int_pow(s, g->gd0[cl]);
#pragma unroll
          for (int j = 0; j < Q; ++j) {
            double a = g->gwc[cl][j][D];
#pragma unroll
            for (int d = D - 1; d >= 0; --d) a = __builtin_fma(a, w, g->gwc[cl][j][d]);
            acc[j] = __builtin_fma(base, a, acc[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const double add = sizeof(T) == 4 ? cst[j] : 0.0;
        f[j] = (T)__builtin_fma((double)w0, (double)f[j], acc[j] + add);
      }
    } else if constexpr (P == 3) {
      // the common two-class case, phi^0 and phi^(1/2) (half-integer exponents):
      // the parity-2 arithmetic in the same order, without the class loop and
      // the general powers, so that it fits eight waves per SIMD
      const DevCoef* __restrict__ g = cfp;
      const double r = __builtin_sqrt(s);
      const double w0c = int_pow(s, g->gstep[0]), b0 = int_pow(s, g->gd0[0]);
      const double w1c = int_pow(s, g->gstep[1]), b1 = r * int_pow(s, g->gd0[1]);
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        double a0 = g->gwc[0][j][D], a1 = g->gwc[1][j][D];
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
          a0 = __builtin_fma(a0, w0c, g->gwc[0][j][d]);
          a1 = __builtin_fma(a1, w1c, g->gwc[1][j][d]);
        }
        const double acc = __builtin_fma(b1, a1, b0 * a0);
        const double add = sizeof(T) == 4 ? cst[j] : 0.0;
        f[j] = (T)__builtin_fma((double)w0, (double)f[j], acc + add);
      }
    } else if constexpr (P == 0 && kReload) {
      // the coefficients in groups of kGroup, in the order of use, as scalar
      // operands of the FMAs; the loads of group g + 1 may not start before
      // group g - 1 has ended (two pointers that the compiler must treat as
      // new after every other group), so at most two groups are live
      CT pt[2] = {(CT)c, (CT)c};
      int u = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        A acc = top[j];
#pragma unroll
        for (int d = K - 2; d >= 0; --d, ++u) {
          acc = fma_s(acc, p, pt[(u / kGroup) & 1][j * kRow + d]);
#if defined(__HIP_DEVICE_COMPILE__)
          // device pass only: a register class of the GPU
          if (u % kGroup == kGroup - 1) asm volatile("" : "+s"(pt[(u / kGroup) & 1]) : "v"(acc));
#endif
        }
        f[j] = (T)fma_a(w0, (A)f[j], acc);
      }
    } else if constexpr (P == 0) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        A acc = top[j];
#pragma unroll
        for (int d = K - 2; d >= 0; --d) acc = fma_a(acc, p, coef(j, d));
        f[j] = (T)fma_a(w0, (A)f[j], acc);
      }
    } else {
      const A u = p * p;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        A acc = top[j];
#pragma unroll
        for (int k = K - 2; k >= 0; --k) acc = fma_a(acc, u, coef(j, k));
        acc = fma_a(acc, p, odd_add(j));
        f[j] = (T)fma_a(w0, (A)f[j], acc);
      }
    }
  }
};

// Coefficient views by (storage, arithmetic)
template <typename T, typename A> struct Relax;
template <> struct Relax<double, double> {
  __device__ static const double* coef(const DevCoef* c) { return &c->wc[0][0]; }
  __device__ static double w0(const DevCoef* c) { return c->w0; }
};
template <> struct Relax<float, double> {
  __device__ static const double* coef(const DevCoef* c) { return &c->wc[0][0]; }
  __device__ static double w0(const DevCoef* c) { return c->w0; }
};
template <> struct Relax<float, float> {
  __device__ static const float* coef(const DevCoef* c) { return &c->wHf[0][0]; }
  __device__ static float w0(const DevCoef* c) { return c->w0f; }
};

template <int Q, int D, int P, typename T, typename A, bool V = false>
__device__ __forceinline__ Relaxer<Q, D, P, T, A, V> make_relaxer(const DevCoef* __restrict__ cf) {
  Relaxer<Q, D, P, T, A, V> r;
  r.init(Relax<T, A>::coef(cf), Relax<T, A>::w0(cf), cf);
  return r;
}

}  // namespace lbm
