// Device code of the lattice step for gfx950 (MI355X): the per-node LBGK
// time step of Shi, He and Guo (Sec. II.A eq. LBE with the equilibria of
// Sec. III), as templates over the lattice size.  kernels_q.hip instantiates
// them once per lattice (one translation unit each, compiled in parallel);
// kernels.hip holds the read-outs and the host launchers.
//
//  k_init      f := f_eq(phi)                        (initial distribution)
//  k_bound     exact-solution boundary layers of a bounded domain
//  k_stream    one fused collide+stream step, state in HBM, SoA rows,
//              coalesced loads, shifted stores with periodic wrap
//  k_resident  persistent work-queue kernel over jobs (instances bin-packed
//              into a workgroup's LDS, threads split in proportion to their
//              nodes); f stays in LDS for all steps of the launch; streaming in
//              place with the alternating (AA) access pattern, one barrier per
//              step
//  k_tile      temporal blocking for grids larger than one workgroup's LDS
//  k_slab      grids larger than one workgroup's LDS split over co-resident
//              workgroups that exchange halo strips
#pragma once

#include "kernels.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// f := f_eq(phi)
// ---------------------------------------------------------------------------
// stored equilibrium of a power-sum model: f_eq_j(phi) - f_rest_j (f_rest = 0
// for FP64 storage); phi >= 0
__device__ __forceinline__ double general_stored_eq(const DevCoef* __restrict__ cf, int j, double phi) {
  const bool roots = cf->groots != 0;
  const double lg = roots ? 0.0 : log2(phi);
  double acc = 0.0;
  for (int c = 0; c < cf->gF; ++c) {
    double a = cf->ginit[c][j][kGRow - 1];
    for (int d = kGRow - 2; d >= 0; --d) a = __builtin_fma(a, phi, cf->ginit[c][j][d]);
    acc = __builtin_fma(c == 0 ? 1.0 : frac_pow(cf->gnu[c], phi, lg, roots), a, acc);
  }
  return acc - cf->grest[j];
}

template <int Q, int D, typename T>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ phi, T* __restrict__ f,
                                              int n, int stride, const DevCoef* __restrict__ cf) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
  if (cf->gF > 0) {
#pragma unroll
    for (int j = 0; j < Q; ++j) f[(int64_t)j * stride + x] = (T)general_stored_eq(cf, j, phi[x]);
    return;
  }
  const double p = phi[x] - cf->phi_rest;   // phi_rest = 0 for FP64 storage
#pragma unroll
  for (int j = 0; j < Q; ++j) f[(int64_t)j * stride + x] = (T)poly_eval<D, 0, double>(cf->init[j], p);
}

// ---------------------------------------------------------------------------
// Bounded domains (exact-solution boundaries of Sec. IV): after a step the
// `layers` outer nodes at each end are reset from the exact solution phi* at
// the new time -- kind 1: f = f_eq(phi*); kind 2 (non-equilibrium
// extrapolation): f = f_eq(phi*) + (f - f_eq(phi)) taken at the first interior
// node.  One thread per boundary node; phib = {left layers, right layers}.
// The stored value is the one k_init stores: f (FP64) or f - f_rest (FP32).
// ---------------------------------------------------------------------------
template <int Q, int D, typename T>
__global__ __launch_bounds__(64) void k_bound(T* __restrict__ f, int n, int stride, int layers, int kind,
                                              const double* __restrict__ phib, const DevCoef* __restrict__ cf) {
  const int t = threadIdx.x;
  if (t >= 2 * layers) return;
  const bool left = t < layers;
  const int x = left ? t : n - 2 * layers + t;
  const int inner = left ? layers : n - 1 - layers;
  double neq[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) neq[j] = 0.0;
  if (kind == 2) {
    double g[Q];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      g[j] = (double)f[(int64_t)j * stride + inner];
      s += g[j];
    }
    // s = phi - phi_rest (phi itself for FP64 storage)
#pragma unroll
    for (int j = 0; j < Q; ++j)
      neq[j] = g[j] - (cf->gF > 0 ? general_stored_eq(cf, j, s + cf->phi_rest) : poly_eval<D, 0, double>(cf->init[j], s));
  }
  const double p = phib[t] - cf->phi_rest;
#pragma unroll
  for (int j = 0; j < Q; ++j)
    f[(int64_t)j * stride + x] =
        (T)((cf->gF > 0 ? general_stored_eq(cf, j, phib[t]) : poly_eval<D, 0, double>(cf->init[j], p)) + neq[j]);
}

// ---------------------------------------------------------------------------
// one fused collide + stream step in HBM (push: coalesced loads, stores shifted
// by e_j with periodic wrap)
// ---------------------------------------------------------------------------
template <int Q, int D, int P, typename T, typename A>
__global__ __launch_bounds__(256) void k_stream(const T* __restrict__ fin, T* __restrict__ fout, int n,
                                                int stride, const DevCoef* __restrict__ cf) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
  T f[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) f[j] = fin[(int64_t)j * stride + x];
  const Relaxer<Q, D, P, T, A> relax = make_relaxer<Q, D, P, T, A>(cf);
  relax(f);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    int y = x + velocity<Q>(j);
    y += (y < 0) ? n : 0;
    y -= (y >= n) ? n : 0;
    fout[(int64_t)j * stride + y] = f[j];
  }
}

// ---------------------------------------------------------------------------
// In-LDS time steps with the alternating (AA) access pattern.  LDS holds node
// x's populations together (S[x QS + j], QS = lds_stride(Q): every population
// of a node is an immediate offset from one address, and an odd node stride
// keeps consecutive lanes on distinct banks -- D1Q4 and D1Q6 rows are padded
// to 5 and 7 slots, since an even stride gives 4- and 2-way bank conflicts).
//   even step: node x reads S[x][j], writes f*_j to S[x][opp(j)]
//   odd step:  node x reads S[x - e_j][opp(j)], writes f*_j to S[x + e_j][j]
// Each node reads exactly the slots it writes, so one barrier per step
// suffices.  After an even number of steps S is in natural layout
// (S[x][j] = f_j(x)); after an odd number f_j(x) = S[x - e_j][opp(j)].
// Nodes are updated two at a time (all loads, both relaxations, all stores)
// so that LDS latency overlaps arithmetic.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrapn(int y, int n) {
  y += (y < 0) ? n : 0;
  y -= (y >= n) ? n : 0;
  return y;
}

template <int Q, typename T, typename R>
__device__ __forceinline__ void aa_even(T* __restrict__ S, int x, const R& r) {
  T* p = S + x * lds_stride(Q);
  T f[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) f[j] = p[j];
  r(f);
#pragma unroll
  for (int j = 0; j < Q; ++j) p[opposite<Q>(j)] = f[j];
}

template <int Q, typename T, typename R>
__device__ __forceinline__ void aa_even2(T* __restrict__ S, int x, int y, const R& r) {
  T* p = S + x * lds_stride(Q);
  T* q = S + y * lds_stride(Q);
  T f[Q], h[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    f[j] = p[j];
    h[j] = q[j];
  }
  r(f);
  r(h);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    p[opposite<Q>(j)] = f[j];
    q[opposite<Q>(j)] = h[j];
  }
}

template <int Q, typename T, typename R>
__device__ __forceinline__ void aa_odd(T* __restrict__ S, int x, const R& r) {
  constexpr int H = Q / 2;
  T* p = S + (x - H) * lds_stride(Q);
  T f[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) f[j] = p[(H - velocity<Q>(j)) * lds_stride(Q) + opposite<Q>(j)];
  r(f);
#pragma unroll
  for (int j = 0; j < Q; ++j) p[(H + velocity<Q>(j)) * lds_stride(Q) + j] = f[j];
}

template <int Q, typename T, typename R>
__device__ __forceinline__ void aa_odd2(T* __restrict__ S, int x, int y, const R& r) {
  constexpr int H = Q / 2;
  T* p = S + (x - H) * lds_stride(Q);
  T* q = S + (y - H) * lds_stride(Q);
  T f[Q], h[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    f[j] = p[(H - velocity<Q>(j)) * lds_stride(Q) + opposite<Q>(j)];
    h[j] = q[(H - velocity<Q>(j)) * lds_stride(Q) + opposite<Q>(j)];
  }
  r(f);
  r(h);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    p[(H + velocity<Q>(j)) * lds_stride(Q) + j] = f[j];
    q[(H + velocity<Q>(j)) * lds_stride(Q) + j] = h[j];
  }
}

// odd step of a node next to the periodic seam
template <int Q, typename T, typename R>
__device__ __forceinline__ void aa_odd_wrap(T* __restrict__ S, int x, int n, const R& r) {
  T f[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) f[j] = S[wrapn(x - velocity<Q>(j), n) * lds_stride(Q) + opposite<Q>(j)];
  r(f);
#pragma unroll
  for (int j = 0; j < Q; ++j) S[wrapn(x + velocity<Q>(j), n) * lds_stride(Q) + j] = f[j];
}

// every node x = lo + t + k B below hi, U (1 or 2) per iteration: two give
// each thread two independent updates to interleave, one keeps the register
// count low enough for eight waves per SIMD
template <int Q, bool ODD, int U, typename T, typename R>
__device__ __forceinline__ void aa_sweep(T* __restrict__ S, int lo, int hi, int t, int B, const R& r) {
  int x = lo + t;
  if constexpr (U == 2) {
    for (; x + B < hi; x += 2 * B) {
      if constexpr (ODD)
        aa_odd2<Q>(S, x, x + B, r);
      else
        aa_even2<Q>(S, x, x + B, r);
    }
  }
  for (; x < hi; x += B) {
    if constexpr (ODD)
      aa_odd<Q>(S, x, r);
    else
      aa_even<Q>(S, x, r);
  }
}

// Nodes x, x + B, ..., x + (iters - 1) B, and x + iters B where `extra` holds
// (the node set of aa_sweep over [lo, hi) when x = lo + t, iters = (hi - lo) / B
// and extra = t < (hi - lo) mod B); `iters` is wave-uniform.  The loop runs on a
// scalar counter and advances a pointer, so that a node costs one vector add
// besides its update; the last pass masks the lanes without an extra node.
template <int Q, bool ODD, typename T, typename R>
__device__ __forceinline__ void aa_sweep_uniform(T* __restrict__ S, int x, int iters, bool extra, int B, const R& r) {
  const int passes = iters + (__builtin_amdgcn_ballot_w64(extra) != 0 ? 1 : 0);
  T* Sx = S + x * lds_stride(Q);
  const int step = B * lds_stride(Q);
  for (int k = 0; k < passes; ++k, Sx += step) {
    if (k < iters || extra) {
      if constexpr (ODD)
        aa_odd<Q>(Sx, 0, r);
      else
        aa_even<Q>(Sx, 0, r);
    }
  }
}

// Sweep of [lo, hi) (lo + t, lo + t + B, ...) with the loop that suits the
// variant: the uniform loop when the equilibrium's coefficients sit in scalar
// registers, or for the two-class power sums with FP32 storage and FP64
// relaxation (measured faster there; with FP64 storage the same loop spills
// vector registers and is slower), else the per-lane loop -- a masked node
// body that must reload a large table spends more than the loop control it
// saves.
// `iters` and `extra` describe [lo, hi) as in aa_sweep_uniform.
template <int Q, int D, int P, typename T, typename A, bool V>
constexpr bool uniform_sweep() {
  return V && (Relaxer<Q, D, P, T, A, V>::kPin || (P == 3 && sizeof(T) == 4 && sizeof(A) == 8));
}

template <int Q, int D, int P, typename A, bool V, bool ODD, typename T, typename R>
__device__ __forceinline__ void aa_sweep_range(T* __restrict__ S, int lo, int hi, int t, int B, int iters, bool extra,
                                               const R& r) {
  if constexpr (uniform_sweep<Q, D, P, T, A, V>())
    aa_sweep_uniform<Q, ODD>(S, lo + t, iters, extra, B, r);
  else
    aa_sweep<Q, ODD, 1>(S, lo, hi, t, B, r);
}

// Initialisation polynomial of degree <= D (the kernel variant's degree bounds
// the dense initialisation table; zeros above the table's own degree leave the
// result bitwise equal to a Horner from its leading coefficient)
template <int D>
__device__ __forceinline__ double poly_init(const double* __restrict__ c, double p) {
  double acc = c[D];
#pragma unroll
  for (int d = D - 1; d >= 0; --d) acc = __builtin_fma(acc, p, c[d]);
  return acc;
}

// exact solution at boundary node b (< 2 layers, left layers first) after step `step`
__device__ __forceinline__ double bound_row(const DevJobInst& ji, int b, int step) {
  return reinterpret_cast<const double*>(ji.phib)[(size_t)step * 2 * ji.layers + b];
}

// One population of one boundary node of a bounded instance in LDS after a
// step, with the arithmetic of k_bound (boundary node b < 2 layers, left layers
// first).  `odd`: an odd number of steps of this chunk is done, so f_j(x) =
// S[x - e_j][opp(j)]; else S holds the natural layout.  Reads touch only the
// first interior node, writes only boundary slots, so all (b, j) run at once.
// `pb`: the exact solution at the node; `row`: the population's initialisation
// polynomial (cf->init[j], or a copy of it in registers).
template <int Q, int D, typename T>
__device__ __forceinline__ void aa_bound_reset(T* __restrict__ S, const DevJobInst& ji, int b, int j, double pb,
                                            bool odd, const DevCoef* __restrict__ cf, const double* __restrict__ row) {
  const int nl = ji.layers, n = ji.n;
  const bool left = b < nl;
  const int x = left ? b : n - 2 * nl + b;
  const int inner = left ? nl : n - 1 - nl;
  auto at = [&](int y, int k) -> int { return odd ? wrapn(y - velocity<Q>(k), n) * lds_stride(Q) + opposite<Q>(k) : y * lds_stride(Q) + k; };
  double neq = 0.0;
  if (ji.bkind == 2) {
    double s = 0.0, gj = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const double g = (double)S[at(inner, k)];
      s += g;
      if (k == j) gj = g;
    }
    neq = gj - (cf->gF > 0 ? general_stored_eq(cf, j, s + cf->phi_rest) : poly_init<D>(row, s));
  }
  const double eq = cf->gF > 0 ? general_stored_eq(cf, j, pb) : poly_init<D>(row, pb - cf->phi_rest);
  S[at(x, j)] = (T)(eq + neq);
}

// One job of the resident kernel: every instance of the job (same variant,
// same step count) is loaded into its LDS region, advanced by its own threads
// between workgroup barriers, and written back.  Threads beyond the job's
// instances (mine < 0) only take part in the barriers.  The bounded kernels
// (B) reset their instances' boundary layers after every step, between two
// barriers; `s0` is the chunk's first step within the launch.  (Periodic jobs
// run kernels without that code: it would cost the hot loop its registers.)
template <int Q, int D, int P, typename T, typename A, bool B>
__device__ void resident_job(T* __restrict__ L, int steps, int s0, const DevJobInst& ji, int mine, int tid,
                             const DevCoef* __restrict__ coefs, int* __restrict__ status) {
  constexpr int H = Q / 2;   // largest |e_j|
  const bool act = mine >= 0;
  T* S = L + ji.lds_off;
  T* g = reinterpret_cast<T*>(ji.addr);
  // threads beyond the job's instances hold a zeroed record (nt = 0): they get
  // a nonzero stride so that nothing below divides by zero (undefined
  // behaviour, which the compiler may use to assume every thread is active)
  const int t = tid - ji.t0, nt = act ? ji.nt : 64, n = act ? ji.n : 0;
  const DevCoef* cf = coefs + (act ? ji.inst : 0);
  // (the bounded kernels spend their vector registers on the boundary rows)
  const Relaxer<Q, D, P, T, A, !B> relax = make_relaxer<Q, D, P, T, A, !B>(cf);
  // interior odd sweeps give threads r..nt-1 one node less, r = (n - 2H) mod nt
  const int r = act ? (n - 2 * H) % nt : 0;
  const int seam0 = (r > 0 && r + 2 * H <= nt) ? r : 0;
  // nodes per thread of the even sweep [0, n) and the odd interior sweep [H, n - H)
  const int ne = act ? n / nt : 0, re = act ? n - ne * nt : 0;
  const int no = act ? (n - 2 * H) / nt : 0;
  if (act)
    for (int j = 0; j < Q; ++j)
      for (int x = t; x < n; x += nt) S[x * lds_stride(Q) + j] = g[(int64_t)j * ji.stride + x];
  __syncthreads();
  // bounded jobs: the (node, population) a thread resets first keeps its
  // equilibrium row in registers for the chunk, and each step's boundary value
  // is loaded before the sweep, so that the reset after the barrier waits on
  // no memory but LDS
  const bool resets = B && act && ji.bkind != 0 && t < 2 * ji.layers * Q;
  double row[B ? D + 1 : 1];
  if constexpr (B) {
#pragma unroll
    for (int d = 0; d <= D; ++d) row[d] = resets ? cf->init[t % Q][d] : 0.0;
  }
  for (int s = 0; s < steps; ++s) {
    double pb_first = 0.0;
    if constexpr (B) {
      if (resets) pb_first = bound_row(ji, t / Q, s0 + s);
    }
    if (act) {
      if ((s & 1) == 0) {
        aa_sweep_range<Q, D, P, A, !B, false>(S, 0, n, t, nt, ne, t < re, relax);
      } else {
        aa_sweep_range<Q, D, P, A, !B, true>(S, H, n - H, t, nt, no, t < r, relax);   // interior: no wrap
        // the 2H seam nodes go to threads with one interior node less
        const int u = t - seam0;
        if (u >= 0 && u < 2 * H) aa_odd_wrap<Q>(S, u < H ? u : n - 2 * H + u, n, relax);
      }
    }
    __syncthreads();
    if constexpr (B) {
      if (resets) {
        aa_bound_reset<Q, D, T>(S, ji, t / Q, t % Q, pb_first, (s & 1) == 0, cf, row);
        // (more than one (node, population) per thread: rows from the table)
        for (int u = t + nt; u < 2 * ji.layers * Q; u += nt)
          aa_bound_reset<Q, D, T>(S, ji, u / Q, u % Q, bound_row(ji, u / Q, s0 + s), (s & 1) == 0, cf,
                                  cf->init[u % Q]);
      }
      __syncthreads();
    }
  }
  // back to HBM in natural layout; flag non-finite values
  if (act) {
    bool bad = false;
    const bool odd = (steps & 1) != 0;
    for (int j = 0; j < Q; ++j) {
      for (int x = t; x < n; x += nt) {
        const T v = odd ? S[wrapn(x - velocity<Q>(j), n) * lds_stride(Q) + opposite<Q>(j)] : S[x * lds_stride(Q) + j];
        bad |= !__builtin_isfinite(v);
        g[(int64_t)j * ji.stride + x] = v;
      }
    }
    if (bad) atomicOr(status + ji.inst, 1);
  }
  __syncthreads();
}

// Persistent kernel over jobs: a workgroup takes the next item from the queue
// until the queue is empty.  Each job's steps are split into `nchunks` chunks
// (a chunk loads the job's state from HBM, advances it and writes it back), and
// the queue holds every job's chunk 0 (longest job first), then every chunk 1,
// and so on, so that the last items of the launch are short and the CUs finish
// together.  Chunk c of job j starts once chunk c-1 of job j has published its
// state (done[j] == c); that chunk was taken from the queue earlier by a
// running workgroup, so every wait ends.  The wait is still bounded: after
// `wait_ticks` ticks of the constant-rate wall clock the chunk gives up, marks
// its instances (status bit 4), skips its steps and publishes anyway, so that
// a scheduling fault ends the kernel instead of hanging the GPU and costs the
// job's later chunks no further wait.  `stall_item` (-1 normally) names a
// queue item that is taken but never run nor published -- a test hook that
// makes the next chunk's wait give up.  The kernel uses no static LDS (an
// instance may fill all 160 KiB): the queue slot reaches the workgroup through
// a per-workgroup word in global memory.  One instantiation per equilibrium
// variant, so that each runs at its own register count and occupancy: the
// light variants (one node per iteration fits 64 VGPRs without spilling) are
// compiled for eight waves per SIMD, the others without a bound.
template <int Q, int D, int P, typename A, typename T = A>
constexpr int resident_waves_per_simd() {
  if constexpr (P == 2) return 1;
  // (the two-class power sums with FP32 storage: four waves, whose registers
  // hold the conversions without spilling, ran faster than eight)
  if constexpr (P == 3) return sizeof(T) == 4 && sizeof(A) == 8 ? 4 : 8;
  if constexpr (sizeof(A) == 4) return 8;
  if constexpr (Q <= 5) return (P ? D <= 9 : D <= 5) ? 8 : 1;
  return 1;
}

// (bounded kernels carry the boundary arithmetic: workgroups of at most 512
// threads, so that their registers hold it without spilling)
template <int Q, int D, int P, typename T, typename A, bool B>
__global__ __launch_bounds__(B ? 512 : 1024) __attribute__((amdgpu_waves_per_eu(B ? 1 : resident_waves_per_simd<Q, D, P, A, T>())))
void k_resident(const DevJob* __restrict__ jobs, const DevJobInst* __restrict__ jinst,
                                                   int njobs, int nchunks, int* __restrict__ counter,
                                                   int* __restrict__ slots, int* __restrict__ done,
                                                   const DevCoef* __restrict__ coefs, int* __restrict__ status,
                                                   long long wait_ticks, int stall_item) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* L = reinterpret_cast<T*>(smem_raw);
  int* slot = slots + blockIdx.x;
  const int tid = threadIdx.x;
  // The only thread-0 branch that ends next to the loop's back edge is the one
  // at the top: it publishes the previous item's chunk and takes the next item.
  // (A second thread-0 branch at the end of the body can be merged with it
  // across the back edge, which gives thread 0 a loop exit of its own while the
  // other threads of its wave go round again.)
  int pub_job = -1, pub_val = 0;
  for (;;) {
    if (tid == 0) {
      if (pub_job >= 0) __hip_atomic_store(done + pub_job, pub_val, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(slot, atomicAdd(counter, 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    __syncthreads();
    if (item >= njobs * nchunks) break;
    pub_job = -1;
    if (item == stall_item) continue;
    const int c = item / njobs;
    const int jid = item - c * njobs;
    const DevJob jb = jobs[jid];
    // an empty chunk is followed by empty chunks only: nobody waits for it
    const int base = jb.steps / nchunks, rem = jb.steps % nchunks;
    const int steps = base + (c < rem ? 1 : 0);
    const int s0 = c * base + (c < rem ? c : rem);
    if (steps > 0) {
      if (c > 0) {
        if (tid == 0) {
          const long long t0 = wall_clock64();
          int seen;
          while ((seen = __hip_atomic_load(done + jid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < c &&
                 wall_clock64() - t0 < wait_ticks)
            __builtin_amdgcn_s_sleep(8);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          __hip_atomic_store(slot, seen < c ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every wave drops stale cached lines
        const int gave_up = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (gave_up) {
          if (tid < jb.count) atomicOr(status + jinst[jb.first + tid].inst, 4);
          __syncthreads();   // every wave has read the slot before thread 0 reuses it
          if (c + 1 < nchunks) {
            pub_job = jid;
            pub_val = c + 1;
          }
          continue;
        }
      }
      // the instance of this wave (thread ranges are wave aligned)
      int mine = -1;
      for (int k = 0; k < jb.count; ++k) {
        const DevJobInst& ck = jinst[jb.first + k];
        if (tid >= ck.t0 && tid < ck.t0 + ck.nt) mine = k;
      }
      mine = __builtin_amdgcn_readfirstlane(mine);
      DevJobInst ji{};
      if (mine >= 0) ji = jinst[jb.first + mine];
      resident_job<Q, D, P, T, A, B>(L, steps, s0, ji, mine, tid, coefs, status);
      if (c + 1 < nchunks) {
        __threadfence();   // this thread's write-back is visible to every CU
        __syncthreads();
        pub_job = jid;
        pub_val = c + 1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Temporal blocking for instances larger than one workgroup's LDS: a tile of
// `core` nodes plus `halo` >= s * max|e_j| nodes on each side is loaded (with
// periodic wrap) into LDS, advanced s steps in place with the AA pattern --
// step k updates nodes [k H, W - k H), the region whose inputs are still
// exact -- and its core is written to the other state buffer.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_any(int y, int n) {
  y %= n;
  return y < 0 ? y + n : y;
}

template <int Q, int D, int P, typename T, typename A>
__device__ __forceinline__ void tile_instance(T* __restrict__ S, const T* __restrict__ gin, T* __restrict__ gout, int n,
                              int stride, int x0, int core, int halo, int steps,
                              const DevCoef* __restrict__ cf, int* __restrict__ status) {
  const int B = blockDim.x;
  const int t = threadIdx.x;
  const Relaxer<Q, D, P, T, A> relax = make_relaxer<Q, D, P, T, A>(cf);
  constexpr int H = Q / 2;
  const int W = core + 2 * halo;
  for (int j = 0; j < Q; ++j)
    for (int i = t; i < W; i += B) S[i * lds_stride(Q) + j] = gin[(int64_t)j * stride + wrap_any(x0 - halo + i, n)];
  __syncthreads();
  // two nodes per iteration, except for the power sums (whose per-node
  // arithmetic already fills the registers)
  constexpr int U = P >= 2 ? 1 : 2;
  for (int s = 0; s < steps; ++s) {
    const int lo = s * H, hi = W - s * H;
    if ((s & 1) == 0)
      aa_sweep<Q, false, U>(S, lo, hi, t, B, relax);
    else
      aa_sweep<Q, true, U>(S, lo, hi, t, B, relax);
    __syncthreads();
  }
  bool bad = false;
  const bool odd = (steps & 1) != 0;
  for (int j = 0; j < Q; ++j) {
    for (int i = halo + t; i < halo + core; i += B) {
      const T v = odd ? S[(i - velocity<Q>(j)) * lds_stride(Q) + opposite<Q>(j)] : S[i * lds_stride(Q) + j];
      bad |= !__builtin_isfinite(v);
      gout[(int64_t)j * stride + x0 + (i - halo)] = v;
    }
  }
  if (bad) atomicOr(status, 1);
}

// One launch = `launch`-th block of up to s steps for every tile.  Instance
// inputs alternate between the two state buffers from launch to launch.
template <int Q, typename T, typename A>
__global__ __launch_bounds__(1024) void k_tile(const DevTile* __restrict__ tiles, const DevTileInst* __restrict__ tinsts,
                                              T* __restrict__ buf0, T* __restrict__ buf1, int launch, int s_per,
                                              int halo, const DevCoef* __restrict__ coefs,
                                              int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* S = reinterpret_cast<T*>(smem_raw);
  const DevTile tl = tiles[blockIdx.x];
  const DevTileInst ti = tinsts[tl.ti];
  const int left = ti.steps - launch * s_per;
  if (left <= 0) return;
  const int st = left < s_per ? left : s_per;
  const int par = ti.cur0 ^ (launch & 1);
  const T* gin = (par ? buf1 : buf0) + ti.off;
  T* gout = (par ? buf0 : buf1) + ti.off;
  const DevCoef* cf = coefs + ti.inst;
  switch (ti.degree) {
#define LBM_CASE(DD, PP)                                                                                   \
  case DD | (PP << 8):                                                                                     \
    tile_instance<Q, DD, PP, T, A>(S, gin, gout, ti.n, ti.stride, tl.x0, tl.core, halo, st, cf, status + ti.inst); \
    break;
    LBM_VARIANT_CASES
#undef LBM_CASE
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// Slabs: an instance too large for one workgroup's LDS is split into slabs,
// one per workgroup of a launch small enough for all its workgroups to be
// resident at once.  A slab holds its core and a halo of s H nodes on each
// side in LDS for all steps of the call: every block of s steps shrinks the
// exact region by H per step down to the core (as in the tiled path), then the
// slab publishes the first and last `halo` nodes of its core, raises its flag,
// waits for both ring neighbours' flags and refills its halos from their
// strips.  State crosses HBM only at the start and the end of the call
// (input buffer -> LDS -> other buffer).  Strips alternate between two buffers
// by block parity: a slab overwrites a parity only after its neighbours have
// raised the flag of the following block, i.e. after they read it.  A wait
// that outlasts `wait_ticks` ticks of the constant-rate wall clock marks the
// instance (status bit 2) and the workgroup stops, so a scheduling fault
// cannot hang the GPU.  `mute_slab` (-1 normally) names a slab that never
// raises its flag -- a test hook that makes its neighbours' waits give up.
//
// Strips and flags move with device-scope (agent) relaxed atomic stores and
// loads, which are coherent across the XCDs' L2 caches without whole-cache
// write-back or invalidation; each wave waits for its strip stores to complete
// (vmcnt 0) before the workgroup barrier that precedes the flag store, and the
// strips are loaded only after the flag load has returned.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until this wave's vector memory operations have completed
__device__ __forceinline__ void wait_vm() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0) expcnt(7) lgkmcnt(15)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <int Q, int D, int P, typename T, typename A>
__device__ void slab_instance(T* __restrict__ S, int* __restrict__ bail, const DevSlab& sl, const DevTileInst& ti,
                              const T* __restrict__ gin, T* __restrict__ gout, int s_per, int halo,
                              T* __restrict__ xbuf, int* __restrict__ flags, int me,
                              const DevCoef* __restrict__ cf, int* __restrict__ status, long long wait_ticks,
                              bool mute) {
  constexpr int H = Q / 2;
  const int B = blockDim.x;
  const int t = threadIdx.x;
  const int n = ti.n, stride = ti.stride;
  const int W = sl.core + 2 * halo;
  const int strip = Q * halo;   // values per strip
  const Relaxer<Q, D, P, T, A, true> relax = make_relaxer<Q, D, P, T, A, true>(cf);
  for (int j = 0; j < Q; ++j)
    for (int i = t; i < W; i += B) S[i * lds_stride(Q) + j] = gin[(int64_t)j * stride + wrap_any(sl.x0 - halo + i, n)];
  if (t == 0) *bail = 0;
  __syncthreads();
  // step k of a block sweeps [k H, W - k H): nodes per thread W / B at k = 0,
  // then 2H nodes fewer per step (kept as a count and a remainder, no division)
  const int iters0 = W / B, rem0 = W - iters0 * B;
  int done = 0, sb = 0;
  for (int blk = 0; done < ti.steps; ++blk) {
    sb = ti.steps - done < s_per ? ti.steps - done : s_per;
    int iters = iters0, rem = rem0;
    for (int k = 0; k < sb; ++k) {
      if (k > 0) {
        rem -= 2 * H;
        while (rem < 0) {
          rem += B;
          --iters;
        }
      }
      if ((k & 1) == 0)
        aa_sweep_range<Q, D, P, A, true, false>(S, k * H, W - k * H, t, B, iters, t < rem, relax);
      else
        aa_sweep_range<Q, D, P, A, true, true>(S, k * H, W - k * H, t, B, iters, t < rem, relax);
      __syncthreads();
    }
    done += sb;
    if (done >= ti.steps) break;
    // publish [left strip | right strip] of the core (natural layout: sb = s_per is even)
    T* mine = xbuf + ((size_t)me * 2 + (blk & 1)) * 2 * strip;
    for (int idx = t; idx < 2 * strip; idx += B) {
      const int side = idx / strip, r = idx - side * strip, j = r / halo, h = r - j * halo;
      const int x = side == 0 ? halo + h : W - 2 * halo + h;
      store_agent(mine + idx, S[x * lds_stride(Q) + j]);
    }
    wait_vm();
    __syncthreads();
    if (t == 0) {
      if (!mute) store_agent(flags + me, blk + 1);
      const long long t0 = wall_clock64();
      bool ready;
      while (!(ready = __hip_atomic_load(flags + sl.left, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > blk &&
                       __hip_atomic_load(flags + sl.right, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > blk) &&
             wall_clock64() - t0 < wait_ticks)
        __builtin_amdgcn_s_sleep(4);
      if (!ready) {
        atomicOr(status + ti.inst, 2);
        *bail = 1;
      }
    }
    __syncthreads();
    if (*bail) break;
    // my left halo <- the left neighbour's right strip; my right halo <- the right neighbour's left strip
    const T* lft = xbuf + ((size_t)sl.left * 2 + (blk & 1)) * 2 * strip + strip;
    const T* rgt = xbuf + ((size_t)sl.right * 2 + (blk & 1)) * 2 * strip;
    for (int idx = t; idx < 2 * strip; idx += B) {
      const int side = idx / strip, r = idx - side * strip, j = r / halo, h = r - j * halo;
      if (side == 0)
        S[h * lds_stride(Q) + j] = load_agent(lft + r);
      else
        S[(W - halo + h) * lds_stride(Q) + j] = load_agent(rgt + r);
    }
    __syncthreads();
  }
  bool bad = false;
  const bool odd = (sb & 1) != 0;
  for (int j = 0; j < Q; ++j) {
    for (int i = halo + t; i < halo + sl.core; i += B) {
      const T v = odd ? S[(i - velocity<Q>(j)) * lds_stride(Q) + opposite<Q>(j)] : S[i * lds_stride(Q) + j];
      bad |= !__builtin_isfinite(v);
      gout[(int64_t)j * stride + sl.x0 + (i - halo)] = v;
    }
  }
  if (bad) atomicOr(status + ti.inst, 1);
}

// one instantiation per equilibrium variant (own register count, as k_resident)
template <int Q, int D, int P, typename T, typename A>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(resident_waves_per_simd<Q, D, P, A>())))
void k_slab(const DevSlab* __restrict__ slabs, const DevTileInst* __restrict__ tinsts, T* __restrict__ buf0,
            T* __restrict__ buf1, int s_per, int halo, T* __restrict__ xbuf, int* __restrict__ flags,
            const DevCoef* __restrict__ coefs, int* __restrict__ status, long long wait_ticks, int mute_slab) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* S = reinterpret_cast<T*>(smem_raw);
  const int me = blockIdx.x;
  const DevSlab sl = slabs[me];
  const DevTileInst ti = tinsts[sl.ti];
  int* bail = reinterpret_cast<int*>(smem_raw + (size_t)(sl.core + 2 * halo) * lds_stride(Q) * sizeof(T));
  const T* gin = (ti.cur0 ? buf1 : buf0) + ti.off;
  T* gout = (ti.cur0 ? buf0 : buf1) + ti.off;
  slab_instance<Q, D, P, T, A>(S, bail, sl, ti, gin, gout, s_per, halo, xbuf, flags, me, coefs + ti.inst, status,
                               wait_ticks, me == mute_slab);
}

}  // namespace lbm
