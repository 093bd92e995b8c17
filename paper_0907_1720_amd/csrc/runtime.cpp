// C-ABI runtime: problem and batch handles, device memory, the planner that
// chooses between the LDS-resident, slab, temporal-blocking and HBM streaming
// kernels, bounded advances, the server, the autotuner and the read-outs.
// Host code only; the kernels live in kernels_body.hpp (instantiated per
// lattice by kernels_q.hip) and their launchers in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <new>
#include <vector>

#include "coeffs.hpp"
#include "kernels.hpp"
#include "wave.hpp"
#include "lbmhpde.h"

using namespace lbm;

#define LBM_HIP(call)                                \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return LBM_ERR_DEVICE;     \
  } while (0)

namespace {

constexpr int kBlock = 256;
constexpr int kMaxSlabs = 2048;       // workgroups of one slab launch
constexpr int kSplitNodes = 1024;     // smallest grid split into slabs when the GPU is mostly idle
constexpr int kMaxResidentGrid = 256 * 8;
constexpr int kMaxLaunches = 64;      // resident launches per advance pass (one per lattice, precision, variant)
constexpr int kAuxStreams = 16;       // concurrent lanes (resident launches, tiled groups, slab launches)
constexpr uint64_t kMagic = 0x4c424d4850444531ull;   // "LBMHPDE1"

struct HostInst {
  lbm_desc desc;
  Model mdl;
  int q = 5;
  int D = 5;        // variant code of the relaxation polynomial (padded degree | parity << 8)
  int Dinit = 5;    // padded dense degree of the initialisation polynomial
  int n = 0;
  int stride = 0;
  bool f32 = false;  // FP32 deviation storage
  int prec = 0;      // lbm_precision
  int64_t off = 0;  // element offset in its precision's state arrays
  int cur = 0;      // which of the two state buffers is current
  int64_t steps_done = 0;
};

// A block of kStepBlock fused collide+stream launches of one instance as a
// HIP graph (the streaming path is launch bound for small grids): replayed
// whole, it advances the instance kStepBlock steps and, kStepBlock being even,
// leaves its state in the buffer it started from.
constexpr int kStepBlock = 64;
struct StepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* fin = nullptr;    // what the graph was built for
  const void* fout = nullptr;
  const void* cf = nullptr;
  int n = 0, stride = 0, code = -1, q = 0, prec = -1;
};

void release_graph(StepGraph* g) {
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  *g = StepGraph{};
}

struct DeviceLimits {
  int cus = 0;
  size_t lds_max = 0;
  double wall_ticks_per_us = 100.0;   // constant-rate device clock (wall_clock64)
  bool ok = false;
};

DeviceLimits query_limits() {
  DeviceLimits L;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return L;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return L;
  L.cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return L;
  L.lds_max = (size_t)v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) == hipSuccess && v > 0)
    L.wall_ticks_per_us = v / 1000.0;   // kHz
  L.ok = true;
  return L;
}

}  // namespace

struct lbm_batch_s {
  hipStream_t stream = nullptr;
  std::vector<HostInst> inst;
  DeviceLimits lim;
  int path = 0;
  // state: two buffers per precision (current / other for the streaming path)
  double* f64[2] = {nullptr, nullptr};
  float* f32[2] = {nullptr, nullptr};
  size_t n64 = 0, n32 = 0;            // elements per buffer
  bool own_state = true;
  void* arena[2] = {nullptr, nullptr};  // serving: both state buffers carved from two arenas
  DevCoef* coefs = nullptr;
  int* status = nullptr;              // per instance: 1 = non-finite seen
  int* counter = nullptr;             // work queue counters (one per group launch)
  int* slots = nullptr;               // per-workgroup queue slot of the resident kernel
  int counters_cap = 0;
  DevJobInst* items = nullptr;        // two slots of items_cap records (alternating calls)
  DevJobInst* items_host = nullptr;   // pinned mirror of both slots
  DevJob* jobs = nullptr;             // two slots of items_cap jobs
  int* done = nullptr;                // per job: chunks published (two slots of items_cap)
  DevJob* jobs_host = nullptr;
  hipEvent_t items_done[2] = {nullptr, nullptr};
  int items_cap = 0;
  int slot = 0;
  double* scratch = nullptr;          // phi read-out (max n) + partial sums
  size_t scratch_elems = 0;
  int* flag = nullptr;                // non-finite flag for read-outs
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // temporal blocking tables (two slots like the items)
  DevTile* tiles = nullptr;
  DevTile* tiles_host = nullptr;
  int tiles_cap = 0;
  DevTileInst* tinsts = nullptr;       // two slots of tinsts_cap records
  int tinsts_cap = 0;
  DevSlab* slabs = nullptr;           // two slots of slabs_cap records
  DevSlab* slabs_host = nullptr;
  int slabs_cap = 0;
  void* xbuf = nullptr;               // halo strips of the slab path
  size_t xbuf_bytes = 0;
  int* sflags = nullptr;              // per-slab block flags
  int sflags_cap = 0;
  DevTileInst* tinsts_host = nullptr;
  int tile_steps = 0;                 // steps per tiled launch (0 = automatic)
  int tile_wgs = 0;                   // tiled workgroups per CU the LDS budget is split for (0 = automatic)
  int res_grid = 0;                   // cap on the resident grid (0 = automatic)
  int res_chunks = 0;                 // step chunks per resident job (0 = automatic)
  int lanes = 0;                      // streams a pass spreads its launches over (0 = automatic)
  hipStream_t aux[kAuxStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kAuxStreams] = {};
  float last_ms = 0.0f;
  std::vector<DevCoef> hcoef;
  std::vector<StepGraph> step_graphs;   // per instance and current-buffer parity
  double* bound = nullptr;              // boundary values of bounded problems (device)
  size_t bound_cap = 0;                 // doubles
  // a bounded advance in progress: phi* rows per instance (device address, 0
  // for periodic instances) and the layers reset at each end
  bool bnd_active = false;
  int bnd_layers = 0;
  std::vector<uint64_t> bnd_ptr;
  // bounded device waits (test hook lbm_batch_test_stall): limit in us (0 =
  // automatic) and the wait to force to give up (0 none, 1 resident, 2 slab)
  int64_t test_wait_us = 0;
  int test_stall = 0;
};

struct lbm_problem_s {
  lbm_batch_s* b = nullptr;
};

namespace {

void fill_devcoef(const HostInst& h, DevCoef* c) {
  std::memset(c, 0, sizeof(*c));
  const Model& m = h.mdl;
  const int parity = h.D >> 8;
  c->w0 = m.w0;
  c->w0f = (float)m.w0;
  if (m.gF > 0) {
    // power sums: omega * G and G per class; FP32 deviations relax in phi
    // = phi_rest + sum_j g_j and add -omega f_rest
    c->gF = m.gF;
    c->groots = 1;
    for (int cl = 1; cl < m.gF; ++cl)
      if (m.gnu[cl] != 0.5 && m.gnu[cl] != 0.25 && m.gnu[cl] != 0.75) c->groots = 0;
    for (int cl = 0; cl < m.gF; ++cl) {
      c->gnu[cl] = m.gnu[cl];
      c->gd0[cl] = m.gd0[cl];
      c->gstep[cl] = m.gstep[cl];
      for (int j = 0; j < m.q; ++j) {
        for (int d = 0; d <= kGDeg && d < kGRow; ++d) c->ginit[cl][j][d] = m.gG[cl][j][d];
        for (int i = 0; i < m.gK[cl] && i < kGRow; ++i) c->gwc[cl][j][i] = m.gwG[cl][j][m.gd0[cl] + m.gstep[cl] * i];
      }
    }
    if (h.f32) {
      c->phi_rest = m.phi_rest;
      c->s0 = m.phi_rest;
      for (int j = 0; j < m.q; ++j) {
        c->cst[j] = -m.wfrest[j];
        c->grest[j] = m.f_rest[j];
      }
    }
    return;
  }
  // FP64 relaxation table: omega * G over the kept degrees
  for (int j = 0; j < m.q; ++j) {
    if (parity == 0) {
      for (int d = 0; d <= m.D; ++d) c->wc[j][d] = m.wG[j][d];
    } else {
      for (int d = 1, k = 0; d <= m.D; d += 2, ++k) c->wc[j][k] = m.wG[j][d];
    }
  }
  if (h.f32) {
    c->phi_rest = m.phi_rest;
    for (int j = 0; j < m.q; ++j) {
      for (int d = 0; d <= m.D; ++d) {
        c->init[j][d] = m.H[j][d];
        c->wHf[j][d] = (float)m.wH[j][d];
      }
    }
    if (h.prec == LBM_F32_DEV) {
      // odd tables: Horner in phi = phi_rest + delta, then -omega f_rest;
      // dense tables: omega * H, the Taylor shift to the rest state, in delta
      // itself (no cancellation against f_rest, one add less per node)
      c->s0 = m.phi_rest;
      for (int j = 0; j < m.q; ++j) {
        c->cst[j] = -m.wfrest[j];
        if (parity == 0)
          for (int d = 0; d <= m.D; ++d) c->wc[j][d] = m.wH[j][d];
      }
    }
  } else {
    for (int j = 0; j < m.q; ++j)
      for (int d = 0; d <= m.D; ++d) c->init[j][d] = m.G[j][d];
  }
}

lbm_status upload_coef(lbm_batch_s* b, int i) {
  fill_devcoef(b->inst[i], &b->hcoef[i]);
  LBM_HIP(hipMemcpyAsync(b->coefs + i, &b->hcoef[i], sizeof(DevCoef), hipMemcpyHostToDevice, b->stream));
  return LBM_OK;
}

size_t elem_size(const HostInst& h) { return h.f32 ? sizeof(float) : sizeof(double); }

void destroy_batch(lbm_batch_s* b) {
  if (!b) return;
  hipStreamSynchronize(b->stream);
  if (b->arena[0]) {
    hipFree(b->arena[0]);
    hipFree(b->arena[1]);
  } else {
    if (b->own_state) {
      hipFree(b->f64[0]);
      hipFree(b->f32[0]);
    }
    hipFree(b->f64[1]);
    hipFree(b->f32[1]);
  }
  hipFree(b->coefs);
  hipFree(b->status);
  hipFree(b->counter);
  hipFree(b->slots);
  hipFree(b->items);
  if (b->items_host) hipHostFree(b->items_host);
  hipFree(b->jobs);
  hipFree(b->done);
  for (StepGraph& g : b->step_graphs) release_graph(&g);
  hipFree(b->bound);
  if (b->jobs_host) hipHostFree(b->jobs_host);
  for (int k = 0; k < 2; ++k)
    if (b->items_done[k]) hipEventDestroy(b->items_done[k]);
  hipFree(b->scratch);
  hipFree(b->flag);
  hipFree(b->tiles);
  hipFree(b->tinsts);
  if (b->tiles_host) hipHostFree(b->tiles_host);
  if (b->tinsts_host) hipHostFree(b->tinsts_host);
  hipFree(b->slabs);
  if (b->slabs_host) hipHostFree(b->slabs_host);
  hipFree(b->xbuf);
  hipFree(b->sflags);
  if (b->ev0) hipEventDestroy(b->ev0);
  if (b->ev1) hipEventDestroy(b->ev1);
  for (int k = 0; k < kAuxStreams; ++k) {
    if (b->aux[k]) hipStreamDestroy(b->aux[k]);
    if (b->join[k]) hipEventDestroy(b->join[k]);
  }
  if (b->fork) hipEventDestroy(b->fork);
  delete b;
}

lbm_status prepare_one(const lbm_desc& d, HostInst* hp) {
  HostInst& h = *hp;
  h = HostInst();
  h.desc = d;
  lbm_status s = build_model(d, &h.mdl);
  if (s != LBM_OK) return s;
  h.q = h.mdl.q;
  h.prec = d.prec;
  h.f32 = h.prec != LBM_F64;
  // odd equilibria (every degree with a nonzero coefficient is odd) evaluate in phi^2;
  // the FP32 relaxation uses the shifted (dense) table
  bool odd = h.prec != LBM_F32_DEV_ARITH32 && h.mdl.gF == 0;
  for (int j = 0; j < h.mdl.q && odd; ++j)
    for (int p = 0; p <= h.mdl.D; p += 2)
      if (h.mdl.G[j][p] != 0.0) odd = false;
  int parity = h.mdl.gF > 0 ? 2 : (odd ? 1 : 0);
  int kmax = 1;   // power sums: the longest strided class
  for (int c = 0; c < h.mdl.gF; ++c) kmax = std::max(kmax, h.mdl.gK[c]);
  int kd = padded_degree(h.mdl.gF > 0 ? kmax - 1 : h.mdl.D, parity);
  // exactly the classes phi^0 and phi^(1/2): the specialised variant, if its degree fits
  if (parity == 2 && h.mdl.gF == 2 && h.mdl.gnu[1] == 0.5 && padded_degree(kmax - 1, 3) > 0) {
    parity = 3;
    kd = padded_degree(kmax - 1, 3);
  }
  // power sums initialise through their own tables; any init variant serves
  h.Dinit = h.mdl.gF > 0 ? padded_degree(1, 0) : padded_degree(h.mdl.D, 0);
  if (kd == 0 || h.Dinit == 0) return LBM_ERR_UNSUPPORTED;
  h.D = variant_code(kd, parity);
  h.n = (int)d.n;
  h.stride = (int)lbm_row_stride(d.n);
  return LBM_OK;
}

lbm_status prepare_instances(const lbm_desc* descs, int count, std::vector<HostInst>* out) {
  out->resize(count);
  for (int i = 0; i < count; ++i) {
    lbm_status s = prepare_one(descs[i], &(*out)[i]);
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

lbm_status alloc_tables(lbm_batch_s* b, size_t maxn);

lbm_status alloc_batch(lbm_batch_s* b, void* dev_buf, size_t buf_bytes) {
  size_t n64 = 0, n32 = 0, maxn = 0;
  for (HostInst& h : b->inst) {
    size_t e = (size_t)h.q * h.stride;
    if (h.f32) {
      h.off = (int64_t)n32;
      n32 += e;
    } else {
      h.off = (int64_t)n64;
      n64 += e;
    }
    maxn = std::max(maxn, (size_t)h.n);
  }
  b->n64 = n64;
  b->n32 = n32;
  if (dev_buf) {
    // caller-owned memory holds the current state buffer of the single problem
    size_t need = n64 * sizeof(double) + n32 * sizeof(float);
    if (buf_bytes < need) return LBM_ERR_OUT_OF_MEMORY;
    b->own_state = false;
    if (n64) b->f64[0] = (double*)dev_buf;
    if (n32) b->f32[0] = (float*)dev_buf;
  } else {
    if (n64 && hipMalloc(&b->f64[0], n64 * sizeof(double)) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
    if (n32 && hipMalloc(&b->f32[0], n32 * sizeof(float)) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  }
  return alloc_tables(b, maxn);
}

// Per-instance tables, queues, streams and events for `b->inst.size()` slots;
// read-out scratch for grids of up to maxn nodes.
lbm_status alloc_tables(lbm_batch_s* b, size_t maxn) {
  const int count = (int)b->inst.size();
  if (hipMalloc(&b->coefs, sizeof(DevCoef) * count) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  if (hipMalloc(&b->status, sizeof(int) * count) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  b->counters_cap = 2 * kMaxLaunches;   // 2 item slots x up to kMaxLaunches launches
  if (hipMalloc(&b->counter, sizeof(int) * b->counters_cap) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  // one queue slot per workgroup of each resident launch
  if (hipMalloc(&b->slots, sizeof(int) * kMaxResidentGrid * 2 * kMaxLaunches) != hipSuccess)
    return LBM_ERR_OUT_OF_MEMORY;
  for (int k = 0; k < kAuxStreams; ++k) {
    LBM_HIP(hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking));
    LBM_HIP(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
  }
  LBM_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  b->tinsts_cap = count;
  if (hipMalloc(&b->tinsts, sizeof(DevTileInst) * 2 * count) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  if (hipHostMalloc((void**)&b->tinsts_host, sizeof(DevTileInst) * 2 * count, hipHostMallocDefault) != hipSuccess)
    return LBM_ERR_OUT_OF_MEMORY;
  b->items_cap = count;
  if (hipMalloc(&b->items, sizeof(DevJobInst) * 2 * count) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  if (hipHostMalloc((void**)&b->items_host, sizeof(DevJobInst) * 2 * count, hipHostMallocDefault) != hipSuccess)
    return LBM_ERR_OUT_OF_MEMORY;
  if (hipMalloc(&b->jobs, sizeof(DevJob) * 2 * count) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  if (hipMalloc(&b->done, sizeof(int) * 2 * count) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  if (hipHostMalloc((void**)&b->jobs_host, sizeof(DevJob) * 2 * count, hipHostMallocDefault) != hipSuccess)
    return LBM_ERR_OUT_OF_MEMORY;
  for (int k = 0; k < 2; ++k) LBM_HIP(hipEventCreateWithFlags(&b->items_done[k], hipEventDisableTiming));
  b->scratch_elems = maxn + 64;
  if (hipMalloc(&b->scratch, sizeof(double) * b->scratch_elems) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  if (hipMalloc(&b->flag, sizeof(int)) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
  LBM_HIP(hipMemsetAsync(b->status, 0, sizeof(int) * count, b->stream));
  LBM_HIP(hipEventCreate(&b->ev0));
  LBM_HIP(hipEventCreate(&b->ev1));
  b->hcoef.resize(count);
  return LBM_OK;
}

lbm_status create_batch(const lbm_desc* descs, int count, void* stream, void* dev_buf, size_t buf_bytes,
                        lbm_batch_s** out) {
  if (!descs || count <= 0 || !out) return LBM_ERR_INVALID_ARG;
  std::vector<HostInst> inst;
  lbm_status s = prepare_instances(descs, count, &inst);
  if (s != LBM_OK) return s;
  lbm_batch_s* b = new (std::nothrow) lbm_batch_s();
  if (!b) return LBM_ERR_OUT_OF_MEMORY;
  b->stream = (hipStream_t)stream;
  b->inst = std::move(inst);
  b->lim = query_limits();
  if (!b->lim.ok) {
    delete b;
    return LBM_ERR_DEVICE;
  }
  s = alloc_batch(b, dev_buf, buf_bytes);
  for (int i = 0; i < count && s == LBM_OK; ++i) s = upload_coef(b, i);
  if (s != LBM_OK) {
    destroy_batch(b);
    return s;
  }
  *out = b;
  return LBM_OK;
}

double* f64_cur(lbm_batch_s* b, const HostInst& h) { return b->f64[h.cur] + h.off; }
float* f32_cur(lbm_batch_s* b, const HostInst& h) { return b->f32[h.cur] + h.off; }
void* state_cur(lbm_batch_s* b, const HostInst& h) {
  return h.f32 ? (void*)f32_cur(b, h) : (void*)f64_cur(b, h);
}
void* state_other(lbm_batch_s* b, const HostInst& h) {
  return h.f32 ? (void*)(b->f32[1 - h.cur] + h.off) : (void*)(b->f64[1 - h.cur] + h.off);
}

lbm_status ensure_second_buffer(lbm_batch_s* b, bool f32) {
  if (f32) {
    if (!b->f32[1] && b->n32 && hipMalloc(&b->f32[1], b->n32 * sizeof(float)) != hipSuccess)
      return LBM_ERR_OUT_OF_MEMORY;
  } else {
    if (!b->f64[1] && b->n64 && hipMalloc(&b->f64[1], b->n64 * sizeof(double)) != hipSuccess)
      return LBM_ERR_OUT_OF_MEMORY;
  }
  return LBM_OK;
}

lbm_status load_phi_one(lbm_batch_s* b, int i, const double* phi, int on_device) {
  HostInst& h = b->inst[i];
  std::vector<double> host;
  if (on_device) {
    host.resize(h.n);
    LBM_HIP(hipMemcpyAsync(host.data(), phi, sizeof(double) * h.n, hipMemcpyDeviceToHost, b->stream));
    LBM_HIP(hipStreamSynchronize(b->stream));
  } else {
    host.assign(phi, phi + h.n);
  }
  for (double v : host)
    if (!std::isfinite(v)) return LBM_ERR_INVALID_ARG;
  if (h.mdl.gF > 1)   // real (non-integer) powers of phi need phi >= 0
    for (double v : host)
      if (v < 0) return LBM_ERR_INVALID_ARG;
  if (h.f32) {
    // rest state: the mean of phi0 (conserved on a periodic grid)
    long double s = 0;
    for (double v : host) s += v;
    set_rest_state(&h.mdl, (double)(s / h.n));
  }
  lbm_status st = upload_coef(b, i);
  if (st != LBM_OK) return st;
  LBM_HIP(hipMemcpyAsync(b->scratch, host.data(), sizeof(double) * h.n, hipMemcpyHostToDevice, b->stream));
  h.cur = 0;
  h.steps_done = 0;
  LBM_HIP(hipMemsetAsync(b->status + i, 0, sizeof(int), b->stream));
  LBM_HIP(launch_init(h.q, h.Dinit, h.prec, b->scratch, state_cur(b, h), h.n, h.stride, b->coefs + i, b->stream));
  // the scratch buffer is reused by the next call on this stream; keep order
  LBM_HIP(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

bool fits_resident(const lbm_batch_s* b, const HostInst& h) {
  return (size_t)lds_stride(h.q) * h.n * elem_size(h) + resident_static_lds(h.q, h.prec, h.D) <= b->lim.lds_max;
}



// The step-block graph of instance i for its current buffer, built on first use
// and rebuilt when the instance's buffers, coefficients or shape changed.
lbm_status step_graph(lbm_batch_s* b, int i, StepGraph** out) {
  const HostInst& h = b->inst[i];
  if (b->step_graphs.size() < 2 * b->inst.size()) b->step_graphs.resize(2 * b->inst.size());
  StepGraph* g = &b->step_graphs[2 * i + h.cur];
  const void* fin = state_cur(b, h);
  const void* fout = state_other(b, h);
  const void* cf = b->coefs + i;
  if (g->exec && g->fin == fin && g->fout == fout && g->cf == cf && g->n == h.n && g->stride == h.stride &&
      g->code == h.D && g->q == h.q && g->prec == h.prec) {
    *out = g;
    return LBM_OK;
  }
  if (g->exec) LBM_HIP(hipStreamSynchronize(b->stream));   // a replay of the stale graph may be in flight
  release_graph(g);
  const void* fn = stream_kernel(h.q, h.D, h.prec);
  if (!fn) return LBM_ERR_UNSUPPORTED;
  struct Args { const void* in; void* out; int n; int stride; const void* cf; };
  std::vector<Args> args(kStepBlock);
  std::vector<void*> ptrs(5 * kStepBlock);
  LBM_HIP(hipGraphCreate(&g->graph, 0));
  hipGraphNode_t prev = nullptr;
  for (int k = 0; k < kStepBlock; ++k) {
    Args& a = args[k];
    a.in = (k & 1) ? fout : fin;
    a.out = const_cast<void*>((k & 1) ? fin : fout);
    a.n = h.n;
    a.stride = h.stride;
    a.cf = cf;
    void** p = &ptrs[5 * k];
    p[0] = &a.in;
    p[1] = &a.out;
    p[2] = &a.n;
    p[3] = &a.stride;
    p[4] = &a.cf;
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3((h.n + 255) / 256);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = p;
    kp.extra = nullptr;
    hipGraphNode_t node;
    LBM_HIP(hipGraphAddKernelNode(&node, g->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
    prev = node;
  }
  LBM_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  g->fin = fin;
  g->fout = fout;
  g->cf = cf;
  g->n = h.n;
  g->stride = h.stride;
  g->code = h.D;
  g->q = h.q;
  g->prec = h.prec;
  *out = g;
  return LBM_OK;
}

constexpr int64_t kMaxStepsPerLaunch = int64_t(1) << 30;
constexpr int kNoAllocMaxNodes = 8192;   // lbm_advance_noalloc: the largest grid one LDS holds

// Limit of a device wait for a cooperating workgroup that has `steps` steps of
// work to finish first: 10 s plus 20 us per step (a node sweep takes well
// under 10 us on every path), in ticks of the device wall clock.
long long wait_ticks(const lbm_batch_s* b, int64_t steps) {
  const double us = b->test_wait_us > 0 ? (double)b->test_wait_us : 1e7 + 20.0 * (double)steps;
  return (long long)(us * b->lim.wall_ticks_per_us);
}

constexpr int kChunkItems = 16;        // queue items per workgroup when jobs outnumber workgroups
constexpr int64_t kMinChunkSteps = 256;
constexpr int kMaxChunks = 64;
constexpr int64_t kMinSlabChunk = 256;   // steps of one chunk of a slab launch

// Lanes a pass spreads its launches over.  HIP runs a process's streams on
// GPU_MAX_HW_QUEUES hardware queues (4 unless that variable is set) and new
// streams go to the least used queue; kernels on streams that share a queue
// run one after another, so more lanes than queues only chain launches
// behind each other in creation order.
int hw_lanes() {
  static const int lanes = [] {
    const char* v = std::getenv("GPU_MAX_HW_QUEUES");
    const int n = v ? std::atoi(v) : 0;
    return n > 0 ? std::min(n, kAuxStreams) : std::min(4, kAuxStreams);
  }();
  return lanes;
}

// One pass: every instance advances by steps[i] <= kMaxStepsPerLaunch.
lbm_status advance_pass(lbm_batch_s* b, const int64_t* steps) {
  const int count = (int)b->inst.size();
  // resident groups by (q, precision, variant); the rest streams through HBM
  // (q, prec, variant code, bounded)
  std::map<std::tuple<int, int, int, int>, std::vector<int>> res;
  std::vector<int> str;          // one launch per step (the plain path)
  std::vector<int> til[8][3];    // temporal blocking, by (q, prec)
  // slabs, by (q, prec, variant, workgroups per CU)
  std::map<std::tuple<int, int, int, int>, std::vector<int>> slb;
  // A pass whose resident instances fill less than a quarter of the GPU's LDS
  // leaves most CUs idle; its step time is that of its largest instances, one
  // CU each.  There, instances of kSplitNodes nodes or more are split into
  // narrow slabs (an eighth of an LDS) spread over otherwise idle CUs.
  // The same holds for instances beyond one LDS when all the pass's state is
  // that small (a serving round): their slabs are narrow too.
  size_t res_bytes = 0, all_bytes = 0;
  for (int i = 0; i < count; ++i) {
    if (!steps[i] || b->path != 0) continue;
    const size_t by = (size_t)lds_stride(b->inst[i].q) * b->inst[i].n * elem_size(b->inst[i]);
    all_bytes += by;
    if (fits_resident(b, b->inst[i])) res_bytes += by;
  }
  const size_t lds_all = (size_t)b->lim.cus * b->lim.lds_max;
  const bool latency = b->path == 0 && b->res_grid == 0 && 4 * res_bytes < lds_all;
  const int slab_wgs = b->tile_wgs > 0 ? b->tile_wgs : latency && 4 * all_bytes < lds_all ? 8 : 2;
  for (int i = 0; i < count; ++i) {
    if (steps[i] == 0) continue;
    const HostInst& h = b->inst[i];
    const bool fits = fits_resident(b, h);
    if (h.desc.bc != LBM_BC_PERIODIC) {
      // bounded instances advance only in a bounded call, on the resident path
      if (!b->bnd_active) return LBM_ERR_INVALID_ARG;
      if (!fits || (b->path != 0 && b->path != 2)) return LBM_ERR_UNSUPPORTED;
      res[std::make_tuple(h.q, h.prec, h.D, 1)].push_back(i);
      continue;
    }
    if (b->path == 2 && !fits) return LBM_ERR_UNSUPPORTED;
    if (b->path == 1)
      str.push_back(i);
    else if (b->path == 3)
      til[h.q][h.prec].push_back(i);
    else if (b->path == 4 || !fits)
      slb[std::make_tuple(h.q, h.prec, h.D, slab_wgs)].push_back(i);
    else if (latency && h.n >= kSplitNodes)
      slb[std::make_tuple(h.q, h.prec, h.D, 8)].push_back(i);
    else
      res[std::make_tuple(h.q, h.prec, h.D, 0)].push_back(i);
  }
  // item records of this call go to slot `k`; wait until the copy issued from
  // the same slot two calls ago has been consumed
  const int k = b->slot;
  b->slot ^= 1;
  LBM_HIP(hipEventSynchronize(b->items_done[k]));
  DevJobInst* hitems = b->items_host + (size_t)k * b->items_cap;
  DevJob* hjobs = b->jobs_host + (size_t)k * b->items_cap;
  // est_max / est_sum: the longest job's and all jobs' duration estimates
  struct Launch { int q; int prec; int code; int first, count; size_t lds; int block; int64_t maxsteps; double est_max, est_sum; };
  std::vector<Launch> launches;
  int used = 0, njobs = 0;
  constexpr int kMaxJobInstances = 16;   // instances per job (one wave each at least)
  for (const auto& group : res) {
    {
      const int pr = std::get<1>(group.first);
      const int bnd = std::get<3>(group.first);
      // the kernel: the variant, and whether its jobs reset boundary layers
      const int code = std::get<2>(group.first) | (bnd << 16);
      std::vector<int> g = group.second;
      const size_t es = pr ? sizeof(float) : sizeof(double);
      const int q = std::get<0>(group.first);
      auto bytes_of = [&](int i) { return ((size_t)lds_stride(q) * b->inst[i].n * es + 15) / 16 * 16; };
      // a workgroup's LDS share: half the LDS, or the largest instance
      size_t cap = b->lim.lds_max / 2;
      for (int i : g) cap = std::max(cap, bytes_of(i));
      // jobs: first-fit decreasing bin packing of equal-step instances into the
      // LDS share; jobs hold instances of one variant and one step count
      std::stable_sort(g.begin(), g.end(), [&](int a, int c) {
        if (steps[a] != steps[c]) return steps[a] > steps[c];
        if (b->inst[a].D != b->inst[c].D) return b->inst[a].D < b->inst[c].D;
        return bytes_of(a) > bytes_of(c);
      });
      // waves per job: the waves a CU can hold at this kernel's register use,
      // shared by the jobs whose LDS fits on one CU
      const int vgprs = std::max(1, resident_vgprs(q, pr, code));
      const int cu_waves = 4 * std::max(1, std::min(8, 512 / vgprs));
      const int jobs_per_cu = std::max<int>(1, (int)(b->lim.lds_max / cap));
      // waves per job: the CU's waves shared by the jobs it holds at once -- in
      // the latency regime (one job per instance) with no more instances than
      // CUs, one job per CU (a 256-tau sweep of bounded instances gets twice the
      // waves).  (bounded kernels are compiled for workgroups of at most 512
      // threads)
      const int cu_jobs = latency && (int)g.size() <= b->lim.cus ? 1 : jobs_per_cu;
      const int kJobWaves = std::max(1, std::min(bnd ? 8 : 16, cu_waves / cu_jobs));
      // a pass that leaves most CUs idle (latency regime) gives every instance a
      // job of its own and up to a wave per 64 nodes: its steps end sooner
      const int kNodesPerWave = latency ? 64 : 128;
      // Passes per step of a full job: a job's waves sweep its nodes 64 per
      // pass, and a member of n nodes needs ceil(n / (64 passes)) waves to end
      // its sweep within that many passes.  Packed by bytes alone, a job's
      // members can need more waves than the job has, so some waves take a
      // pass more than the rest and every step waits for them.  Where two jobs
      // share each CU (eight waves per SIMD: the step is bound by VALU issue) a
      // job therefore admits a member only while the members' waves at that
      // pass count fit (the 4096-instance FP32 batch: 46.5 -> 45.3 ms).  One
      // job per CU is bound by the step's latency instead, and fuller jobs pay
      // there (the FP64 batch ran 1.5% slower with the rule).
      const bool wave_budget = !latency && jobs_per_cu >= 2;
      const int full_passes = std::max<int>(
          std::max(1, kNodesPerWave / 64),
          (int)((cap / ((size_t)lds_stride(q) * es) + 64 * (size_t)kJobWaves - 1) / (64 * (size_t)kJobWaves)));
      auto waves_at = [&](int i) {
        return wave_budget ? (b->inst[i].n + 64 * full_passes - 1) / (64 * full_passes) : 0;
      };
      struct Bin { int64_t steps; int variant; size_t bytes; int waves; std::vector<int> members; };
      std::vector<Bin> bins;
      auto pack = [&](int max_inst) {
        bins.clear();
        size_t open_from = 0;   // bins before this index have another step count or variant
        for (int i : g) {
          if (!bins.empty() && (bins.back().steps != steps[i] || bins.back().variant != b->inst[i].D))
            open_from = bins.size();
          bool placed = false;
          for (size_t u = open_from; u < bins.size() && !placed; ++u) {
            Bin& bn = bins[u];
            if (bn.bytes + bytes_of(i) <= cap && (int)bn.members.size() < max_inst &&
                bn.waves + waves_at(i) <= kJobWaves) {
              bn.bytes += bytes_of(i);
              bn.waves += waves_at(i);
              bn.members.push_back(i);
              placed = true;
            }
          }
          if (!placed) bins.push_back(Bin{steps[i], b->inst[i].D, bytes_of(i), waves_at(i), {i}});
        }
      };
      pack(latency ? 1 : std::min(kMaxJobInstances, kJobWaves));
      // fewer jobs than the GPU holds at once (jobs_per_cu per CU) leave CUs
      // idle for the whole pass: cap the instances per job so that there are
      // enough (1024 instances of 1024 FP32 D1Q5 nodes would otherwise make
      // 256 half-LDS jobs for 512 slots)
      const int slots = jobs_per_cu * b->lim.cus;
      if (!latency && (int)bins.size() < slots && (int)g.size() > (int)bins.size())
        pack(std::max(1, ((int)g.size() + slots - 1) / slots));
      Launch L{q, pr, code, njobs, 0, 0, 64, 0, 0.0, 0.0};
      struct Planned { const Bin* bin; std::vector<int> waves; double est; };
      std::vector<Planned> plan;
      for (const Bin& bn : bins) {
        // waves: one each, then one more at a time to the member with the most
        // nodes per wave (at most one wave per kNodesPerWave nodes)
        const int m = (int)bn.members.size();
        std::vector<int> wv(m, 1);
        int total = m;
        while (total < kJobWaves) {
          int best = -1;
          double load = 0.0;
          for (int u = 0; u < m; ++u) {
            const int n = b->inst[bn.members[u]].n;
            if (wv[u] >= (n + kNodesPerWave - 1) / kNodesPerWave) continue;
            const double l = (double)n / wv[u];
            if (l > load) {
              load = l;
              best = u;
            }
          }
          if (best < 0) break;
          ++wv[best];
          ++total;
        }
        // duration estimate: steps x nodes of the busiest thread x arithmetic per node
        int npt = 1;
        for (int u = 0; u < m; ++u) npt = std::max(npt, (b->inst[bn.members[u]].n + 64 * wv[u] - 1) / (64 * wv[u]));
        const int dd = b->inst[bn.members[0]].D & 0xff;
        plan.push_back(Planned{&bn, wv, (double)bn.steps * npt * (q * (dd + 3))});
      }
      // longest job first (longest-processing-time order for the queue)
      std::stable_sort(plan.begin(), plan.end(), [](const Planned& a, const Planned& c) { return a.est > c.est; });
      for (const Planned& pl : plan) {
        const Bin& bn = *pl.bin;
        const std::vector<int>& wv = pl.waves;
        const int m = (int)bn.members.size();
        L.maxsteps = std::max<int64_t>(L.maxsteps, bn.steps);
        L.est_max = std::max(L.est_max, pl.est);
        L.est_sum += pl.est;
        DevJob& jb = hjobs[njobs++];
        jb.first = used;
        jb.count = m;
        jb.steps = (int)bn.steps;
        jb.degree = bn.variant;
        jb.bounded = bnd;
        jb.pad_ = 0;
        int t0 = 0, off = 0;
        for (int u = 0; u < m; ++u) {
          const int i = bn.members[u];
          const HostInst& h = b->inst[i];
          DevJobInst& it = hitems[used++];
          it.addr = (uint64_t)(uintptr_t)state_cur(b, h);
          it.n = h.n;
          it.stride = h.stride;
          it.degree = h.D;
          it.inst = i;
          it.lds_off = off;
          it.t0 = t0;
          it.nt = 64 * wv[u];
          it.phib = bnd ? b->bnd_ptr[i] : 0;
          it.bkind = bnd ? (h.desc.bc == LBM_BC_DIRICHLET_EQ ? 1 : 2) : 0;
          it.layers = bnd ? b->bnd_layers : 0;
          it.pad_ = 0;
          t0 += it.nt;
          off += (int)(bytes_of(i) / es);
        }
        L.lds = std::max(L.lds, (size_t)off * es);
        L.block = std::max(L.block, t0);
      }
      L.count = njobs - L.first;
      if ((int)launches.size() >= kMaxLaunches) return LBM_ERR_UNSUPPORTED;
      launches.push_back(L);
    }
  }
  // temporal blocking plan per (q, prec) group
  struct TileGroup { int q; int prec; int first, ntiles, tfirst, tcount, s, halo, launches, block; size_t lds; double est; };
  std::vector<TileGroup> tgroups;
  std::vector<DevTile> tvec;
  // tile-instance records of this pass (the tiled path: one per instance; the
  // slab path: one per instance and step chunk), copied to slot k below
  std::vector<DevTileInst> htin;
  int tin_used = 0;
  // slab plan per (q, prec): cooperative launches of at most `capacity` slabs
  // (every workgroup of a launch resident at once), run one after another on
  // one lane; an instance whose slabs exceed one launch, or whose slabs would
  // be narrower than a halo, goes to temporal blocking instead.  When a
  // group's instances need several launches, their steps are split into
  // chunks and the (instance, chunk) items fill the launches in chunk-major
  // order, an even share each (without chunks, a last launch with a few
  // instances costs a whole launch's time).  An instance's chunk c + 1 always
  // lies in a later launch than its chunk c (a launch holds less than one
  // chunk's items plus one instance), which the lane's order serialises.
  struct SlabLaunch { int q; int prec; int code; int first, count, cap, s, halo, block; size_t lds; size_t xoff; int foff; double est; };
  std::vector<SlabLaunch> slaunch;
  std::vector<DevSlab> svec;
  size_t xbuf_need = 0;
  int flags_need = 0;
  int min_per_cu = 1 << 30;
  const int tin_slab0 = tin_used;
  std::vector<int> slab_insts;
  for (const auto& group : slb) {
    {
      const int qq = std::get<0>(group.first), pr = std::get<1>(group.first), code = std::get<2>(group.first);
      const int wgs = std::get<3>(group.first);
      const std::vector<int>& g = group.second;
      const int q = qq, H = q / 2;
      const size_t es = pr ? sizeof(float) : sizeof(double);
      const int W = (int)((b->lim.lds_max / (size_t)wgs - 16) / (lds_stride(q) * es));
      int sp = b->tile_steps > 0 ? (b->tile_steps + 1) / 2 * 2 : 16;   // even: strips in natural layout
      while (sp > 2 && W - 2 * sp * H < 2 * sp * H) sp -= 2;
      const int halo = sp * H;
      const int cmax = W - 2 * halo;
      // two or more nodes per thread; if the kernel's registers do not let
      // `wgs` workgroups of that size share a CU (its LDS is cut for wgs), take
      // the largest smaller workgroup (a multiple of one wave, not below 256
      // threads) that lets them, so no part of the LDS stays unused
      int block = std::min(1024, std::max(64, (W / 2 + 63) / 64 * 64));
      const size_t lds = (size_t)W * lds_stride(q) * es + 16;
      int per_cu = 0;
      if (cmax < halo || slab_occupancy(q, pr, code, block, lds, &per_cu) != hipSuccess) per_cu = 0;
      for (int nb = block - 64; per_cu > 0 && per_cu < wgs && nb >= 256; nb -= 64) {
        int pc = 0;
        if (slab_occupancy(q, pr, code, nb, lds, &pc) != hipSuccess) break;
        if (pc > per_cu) {
          block = nb;
          per_cu = pc;
        }
      }
      const int capacity = std::min(per_cu * b->lim.cus, kMaxSlabs);
      if (per_cu > 0) min_per_cu = std::min(min_per_cu, per_cu);
      SlabLaunch L{q, pr, code, (int)svec.size(), 0, capacity, sp, halo, block, lds, 0, 0, 0.0};
      // the instances that take slabs, their slab counts and core widths
      std::vector<std::pair<int, int>> mem;   // (instance, slabs)
      int64_t total = 0, maxsteps = 0;
      for (int i : g) {
        const HostInst& h = b->inst[i];
        const int ks = cmax > 0 ? (h.n + cmax - 1) / cmax : 0;
        const int core = ks > 0 ? (h.n + ks - 1) / ks : 0;
        if (ks < 1 || ks > capacity || core < halo || h.n - (ks - 1) * core < halo) {
          til[qq][pr].push_back(i);
          continue;
        }
        mem.push_back({i, ks});
        total += ks;
        maxsteps = std::max<int64_t>(maxsteps, steps[i]);
      }
      // step chunks: a launch lasts about its chunk's steps whatever its fill,
      // so c chunks cost (launches needed for c chunks) / c; take the fewest
      // chunks (at most 8, each >= kMinSlabChunk steps) within 3% of the
      // cheapest, counting launches by packing whole instances as below
      auto launches_for = [&](int c) {
        int nl = 1, fill = 0;
        for (int r = 0; r < c; ++r)
          for (const auto& m : mem) {
            if (fill + m.second > capacity) {
              ++nl;
              fill = 0;
            }
            fill += m.second;
          }
        return nl;
      };
      int nch = 1;
      if (total > capacity && maxsteps >= 2 * kMinSlabChunk) {
        double best = 1e30;
        std::vector<double> cost(9, 1e30);
        for (int c = 1; c <= 8 && maxsteps / c >= kMinSlabChunk; ++c) {
          cost[c] = (double)launches_for(c) / c;
          best = std::min(best, cost[c]);
        }
        for (int c = 1; c <= 8; ++c)
          if (cost[c] <= 1.03 * best) {
            nch = c;
            break;
          }
      }
      // the items spread evenly over that many launches (a launch is closed
      // once it holds its share), so that no launch is a short tail: the
      // packing above would fill all but the last, which, lightly loaded, runs
      // its steps faster but still about as long as a full one
      const int64_t share = total * nch > capacity ? (total * nch + launches_for(nch) - 1) / launches_for(nch)
                                                   : capacity;
      for (int c = 0; c < nch; ++c) {
        for (const auto& [i, ks] : mem) {
          const HostInst& h = b->inst[i];
          const int64_t base = steps[i] / nch, rem = steps[i] % nch;
          const int64_t st = base + (c < rem ? 1 : 0);
          if (st == 0) continue;
          const int core = (h.n + ks - 1) / ks;
          if (L.count + ks > capacity || L.count >= share) {
            slaunch.push_back(L);
            L.first = (int)svec.size();
            L.count = 0;
            L.est = 0.0;
          }
          // duration estimate, in the unit of the resident jobs' (steps x nodes
          // of the busiest thread x arithmetic per node)
          L.est = std::max(L.est, (double)st * ((core + 2 * halo + block - 1) / block) * (q * ((h.D & 0xff) + 3)));
          DevTileInst ti{};
          ti.off = h.off;
          ti.n = h.n;
          ti.stride = h.stride;
          ti.steps = (int)st;
          ti.cur0 = h.cur ^ (c & 1);   // each earlier chunk flipped the buffer once
          ti.degree = h.D;
          ti.inst = i;
          htin.push_back(ti);
          for (int m = 0; m < ks; ++m) {
            DevSlab sl;
            sl.ti = tin_used;
            sl.x0 = m * core;
            sl.core = std::min(core, h.n - m * core);
            sl.left = L.count + (m + ks - 1) % ks;
            sl.right = L.count + (m + 1) % ks;
            sl.pad_ = 0;
            svec.push_back(sl);
          }
          L.count += ks;
          ++tin_used;
          if (c == 0) slab_insts.push_back(i);
        }
      }
      if (L.count) slaunch.push_back(L);
    }
  }
  // every launch its own strip and flag region (launches may run side by side)
  for (SlabLaunch& S : slaunch) {
    S.xoff = xbuf_need;
    S.foff = flags_need;
    xbuf_need += ((size_t)S.count * 4 * S.q * S.halo * (S.prec ? sizeof(float) : sizeof(double)) + 255) / 256 * 256;
    flags_need += S.count;
  }
  // side by side only while all their workgroups fit the GPU twice over;
  // otherwise one after another (each launch alone fits by construction)
  int64_t total_slabs = 0, total_cap = 0;
  for (const SlabLaunch& S : slaunch) {
    total_slabs += S.count;
    total_cap += S.cap;
  }
  bool slab_side_by_side = slaunch.size() > 1 && 2 * total_slabs <= (int64_t)min_per_cu * b->lim.cus;
  // A small pass (a serving round) whose slab launches would run one after
  // another, each less than half full on average, is bound by that sequence of
  // mostly idle launches; temporal blocking has no co-residency condition, so
  // its groups run side by side: those instances take it instead (results are
  // the same bit for bit).  Launches that fill the GPU keep their slabs.
  if (latency && slaunch.size() > 1 && !slab_side_by_side && 2 * total_slabs < total_cap) {
    for (int i : slab_insts) til[b->inst[i].q][b->inst[i].prec].push_back(i);
    tin_used = tin_slab0;
    htin.resize(tin_slab0);
    svec.clear();
    slaunch.clear();
    xbuf_need = 0;
    flags_need = 0;
    slab_side_by_side = false;
  }
  if (!svec.empty()) {
    if ((int)svec.size() > b->slabs_cap || xbuf_need > b->xbuf_bytes || flags_need > b->sflags_cap) {
      // grow the slab tables and exchange buffers; earlier passes must be done with them
      LBM_HIP(hipStreamSynchronize(b->stream));
      if ((int)svec.size() > b->slabs_cap) {
        hipFree(b->slabs);
        if (b->slabs_host) hipHostFree(b->slabs_host);
        b->slabs = nullptr;
        b->slabs_host = nullptr;
        b->slabs_cap = 0;
        const int cap = (int)svec.size() * 2;
        if (hipMalloc(&b->slabs, sizeof(DevSlab) * 2 * cap) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
        if (hipHostMalloc((void**)&b->slabs_host, sizeof(DevSlab) * 2 * cap, hipHostMallocDefault) != hipSuccess)
          return LBM_ERR_OUT_OF_MEMORY;
        b->slabs_cap = cap;
      }
      if (xbuf_need > b->xbuf_bytes) {
        hipFree(b->xbuf);
        b->xbuf = nullptr;
        b->xbuf_bytes = 0;
        if (hipMalloc(&b->xbuf, xbuf_need) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
        b->xbuf_bytes = xbuf_need;
      }
      if (flags_need > b->sflags_cap) {
        hipFree(b->sflags);
        b->sflags = nullptr;
        b->sflags_cap = 0;
        if (hipMalloc(&b->sflags, sizeof(int) * flags_need) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
        b->sflags_cap = flags_need;
      }
    }
    std::memcpy(b->slabs_host + (size_t)k * b->slabs_cap, svec.data(), sizeof(DevSlab) * svec.size());
    for (const auto& group : slb) {
      lbm_status st = ensure_second_buffer(b, std::get<1>(group.first) != 0);
      if (st != LBM_OK) return st;
    }
  }
  for (int qq = 4; qq < 8; ++qq) {
    for (int pr = 0; pr < 3; ++pr) {
      const std::vector<int>& g = til[qq][pr];
      if (g.empty()) continue;
      const int q = qq, H = q / 2;
      const size_t es = pr ? sizeof(float) : sizeof(double);
      const int wgs = b->tile_wgs > 0 ? b->tile_wgs : 2;
      const int W = (int)(b->lim.lds_max / (size_t)wgs / (lds_stride(q) * es));
      // tile core: as wide as the LDS share allows, but narrow enough that the
      // group yields about 4 tiles per CU (a few large instances would otherwise
      // leave most CUs idle); halo / core kept below 1/4
      int64_t nodes = 0;
      for (int i : g) nodes += b->inst[i].n;
      const int want = (int)std::max<int64_t>(256, nodes / (4 * (int64_t)b->lim.cus));
      int sp = b->tile_steps > 0 ? b->tile_steps : 32;
      while (sp > 1 && (W - 2 * sp * H < 2 * sp * H || (b->tile_steps == 0 && 8 * sp * H > want))) sp /= 2;
      const int halo = sp * H;
      const int core = std::max(1, std::min(W - 2 * halo, want));
      TileGroup G{q, pr, (int)tvec.size(), 0, tin_used, 0, sp, halo, 0, kBlock, 0, 0.0};
      int64_t maxsteps = 0;
      int maxcore = 1, maxd = 0;
      for (int i : g) {
        const HostInst& h = b->inst[i];
        htin.emplace_back();
        DevTileInst& ti = htin.back();
        ti.off = h.off;
        ti.n = h.n;
        ti.stride = h.stride;
        ti.steps = (int)steps[i];
        ti.cur0 = h.cur;
        ti.degree = h.D;
        ti.inst = i;
        const int c = std::min(core, h.n);
        for (int x0 = 0; x0 < h.n; x0 += c) {
          DevTile t{tin_used, x0, std::min(c, h.n - x0), 0};
          tvec.push_back(t);
        }
        maxcore = std::max(maxcore, c);
        maxd = std::max(maxd, h.D & 0xff);
        maxsteps = std::max<int64_t>(maxsteps, steps[i]);
        ++tin_used;
      }
      G.ntiles = (int)tvec.size() - G.first;
      G.tcount = tin_used - G.tfirst;
      G.launches = (int)((maxsteps + sp - 1) / sp);
      G.lds = (size_t)lds_stride(q) * (maxcore + 2 * halo) * es;
      // two or more nodes per thread
      G.block = std::min(kBlock, std::max(64, ((maxcore + 2 * halo) / 2 + 63) / 64 * 64));
      // duration estimate (as the resident jobs'): the launches' steps x nodes of
      // the busiest thread x arithmetic per node x rounds of tiles over the CUs
      G.est = (double)G.launches * sp * ((maxcore + 2 * halo + G.block - 1) / G.block) * (q * (maxd + 3)) *
              ((G.ntiles + 2 * b->lim.cus - 1) / (2 * b->lim.cus));
      tgroups.push_back(G);
    }
  }
  if (!tvec.empty()) {
    if ((int)tvec.size() > b->tiles_cap) {
      // grow the tile tables (both slots); previous users of the buffers must be done
      LBM_HIP(hipStreamSynchronize(b->stream));
      hipFree(b->tiles);
      if (b->tiles_host) hipHostFree(b->tiles_host);
      b->tiles = nullptr;
      b->tiles_host = nullptr;
      b->tiles_cap = 0;
      const int cap = (int)tvec.size() * 2;
      if (hipMalloc(&b->tiles, sizeof(DevTile) * 2 * cap) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
      if (hipHostMalloc((void**)&b->tiles_host, sizeof(DevTile) * 2 * cap, hipHostMallocDefault) != hipSuccess)
        return LBM_ERR_OUT_OF_MEMORY;
      b->tiles_cap = cap;
    }
    std::memcpy(b->tiles_host + (size_t)k * b->tiles_cap, tvec.data(), sizeof(DevTile) * tvec.size());
    for (int i : str) (void)i;
    for (int qq = 4; qq < 8; ++qq)
      for (int pr = 0; pr < 3; ++pr) {
        lbm_status st = til[qq][pr].empty() ? LBM_OK : ensure_second_buffer(b, pr != 0);
        if (st != LBM_OK) return st;
      }
  }

  LBM_HIP(hipEventRecord(b->ev0, b->stream));
  if (!tvec.empty()) {
    DevTile* dt = b->tiles + (size_t)k * b->tiles_cap;
    LBM_HIP(hipMemcpyAsync(dt, b->tiles_host + (size_t)k * b->tiles_cap, sizeof(DevTile) * tvec.size(),
                           hipMemcpyHostToDevice, b->stream));
  }
  if (!svec.empty()) {
    DevSlab* ds = b->slabs + (size_t)k * b->slabs_cap;
    LBM_HIP(hipMemcpyAsync(ds, b->slabs_host + (size_t)k * b->slabs_cap, sizeof(DevSlab) * svec.size(),
                           hipMemcpyHostToDevice, b->stream));
  }
  if (tin_used) {
    if (tin_used > b->tinsts_cap) {
      // grow both slots; earlier passes must be done with them
      LBM_HIP(hipStreamSynchronize(b->stream));
      hipFree(b->tinsts);
      hipHostFree(b->tinsts_host);
      b->tinsts = nullptr;
      b->tinsts_host = nullptr;
      b->tinsts_cap = 0;
      const int cap = 2 * tin_used;
      if (hipMalloc(&b->tinsts, sizeof(DevTileInst) * 2 * cap) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
      if (hipHostMalloc((void**)&b->tinsts_host, sizeof(DevTileInst) * 2 * cap, hipHostMallocDefault) != hipSuccess)
        return LBM_ERR_OUT_OF_MEMORY;
      b->tinsts_cap = cap;
    }
    DevTileInst* hti = b->tinsts_host + (size_t)k * b->tinsts_cap;
    std::memcpy(hti, htin.data(), sizeof(DevTileInst) * tin_used);
    DevTileInst* dti = b->tinsts + (size_t)k * b->tinsts_cap;
    LBM_HIP(hipMemcpyAsync(dti, hti, sizeof(DevTileInst) * tin_used, hipMemcpyHostToDevice, b->stream));
  }
  DevJobInst* ditems = b->items + (size_t)k * b->items_cap;
  DevJob* djobs = b->jobs + (size_t)k * b->items_cap;
  int* counters = b->counter + k * kMaxLaunches;
  if (used) {
    LBM_HIP(hipMemcpyAsync(ditems, hitems, sizeof(DevJobInst) * used, hipMemcpyHostToDevice, b->stream));
    LBM_HIP(hipMemcpyAsync(djobs, hjobs, sizeof(DevJob) * njobs, hipMemcpyHostToDevice, b->stream));
    LBM_HIP(hipMemsetAsync(counters, 0, sizeof(int) * kMaxLaunches, b->stream));
    LBM_HIP(hipMemsetAsync(b->done + (size_t)k * b->items_cap, 0, sizeof(int) * njobs, b->stream));
  }
  // Lanes: every resident launch, every tiled group and every slab launch (or
  // the chain of slab launches, when they cannot run side by side) is one
  // item; with more items than lanes, each item in order of its duration
  // estimate, longest first, goes to the lane with the least estimated work
  // so far (longest-processing-time scheduling).  With no more items than
  // lanes each has a lane of its own, issued in plan order (launches that each
  // fill the GPU take its CUs in that order: the 4096-instance KdV/mKdV pass
  // ran 1% longer with the longer mKdV launch first).  The fork is recorded
  // after all table uploads above.
  // slab launches: each needs all its workgroups resident at once.  Each fits
  // the GPU alone, and the other lanes' kernels never wait on it, so its
  // workgroups all get CUs once those kernels retire; two slab launches side
  // by side could each hold CUs the other waits for, so they share a lane, in
  // order, unless all of them fit the GPU twice over
  struct LaneItem { int kind; int idx; double est; };   // kind 0 resident, 1 tiled, 2 slab (-1: the chain)
  std::vector<LaneItem> items;
  for (size_t l = 0; l < launches.size(); ++l) {
    const Launch& L = launches[l];
    items.push_back({0, (int)l, std::max(L.est_max, L.est_sum / b->lim.cus)});
  }
  for (size_t g = 0; g < tgroups.size(); ++g) items.push_back({1, (int)g, tgroups[g].est});
  if (slab_side_by_side) {
    for (size_t l = 0; l < slaunch.size(); ++l) items.push_back({2, (int)l, slaunch[l].est});
  } else if (!slaunch.empty()) {
    double est = 0.0;
    for (const SlabLaunch& S : slaunch) est += S.est;
    items.push_back({2, -1, est});
  }
  const bool fork = items.size() > 1;
  const int nlanes = std::min<int>((int)items.size(), b->lanes > 0 ? b->lanes : hw_lanes());
  if ((int)items.size() > nlanes)
    std::stable_sort(items.begin(), items.end(), [](const LaneItem& x, const LaneItem& y) { return x.est > y.est; });
  std::vector<double> lane_load(nlanes, 0.0);
  std::vector<char> lane_forked(nlanes, 0);
  if (fork) LBM_HIP(hipEventRecord(b->fork, b->stream));
  const DevSlab* ds = b->slabs + (size_t)k * b->slabs_cap;
  const DevTileInst* dti_all = b->tinsts + (size_t)k * b->tinsts_cap;
  auto issue_slab = [&](size_t l, hipStream_t st) -> lbm_status {
    const SlabLaunch& L = slaunch[l];
    void* b0 = L.prec ? (void*)b->f32[0] : (void*)b->f64[0];
    void* b1 = L.prec ? (void*)b->f32[1] : (void*)b->f64[1];
    int* flags = b->sflags + L.foff;
    LBM_HIP(hipMemsetAsync(flags, 0, sizeof(int) * L.count, st));
    const int mute = (b->test_stall == 2 && l == 0) ? 0 : -1;
    LBM_HIP(launch_slab(L.q, L.prec, L.code, ds + L.first, L.count, dti_all, b0, b1, L.s, L.halo,
                        (unsigned char*)b->xbuf + L.xoff, flags, b->coefs, b->status, wait_ticks(b, L.s), mute,
                        L.block, L.lds, st));
    return LBM_OK;
  };
  for (size_t ii = 0; ii < items.size(); ++ii) {
    const LaneItem& it = items[ii];
    hipStream_t st = b->stream;
    if (fork) {
      const int ln = (int)items.size() <= nlanes
                         ? (int)ii
                         : (int)(std::min_element(lane_load.begin(), lane_load.end()) - lane_load.begin());
      lane_load[ln] += it.est;
      st = b->aux[ln];
      if (!lane_forked[ln]) {
        LBM_HIP(hipStreamWaitEvent(st, b->fork, 0));
        lane_forked[ln] = 1;
      }
    }
    if (it.kind == 0) {
      const int l = it.idx;
      const Launch& L = launches[l];
      int per_cu = 0;
      LBM_HIP(resident_occupancy(L.q, L.prec, L.code, L.block, L.lds, &per_cu));
      if (per_cu < 1) return LBM_ERR_UNSUPPORTED;
      int grid = std::min<int>(std::min<int>(L.count, per_cu * b->lim.cus), kMaxResidentGrid);
      if (b->res_grid > 0) grid = std::min(grid, b->res_grid);
      // more jobs than workgroups: split the steps into chunks so that each
      // workgroup takes about kChunkItems items and the launch ends evenly;
      // chunks keep at least kMinChunkSteps steps (a chunk reloads its state)
      int nchunks = 1;
      if (L.count > grid) {
        nchunks = (int)std::min<int64_t>((kChunkItems * (int64_t)grid + L.count - 1) / L.count,
                                         std::max<int64_t>(1, L.maxsteps / kMinChunkSteps));
        nchunks = std::max(1, std::min(nchunks, kMaxChunks));
      }
      if (b->res_chunks > 0) nchunks = b->res_chunks;
      int* slots = b->slots + (size_t)(k * kMaxLaunches + l) * kMaxResidentGrid;
      int* done = b->done + (size_t)k * b->items_cap + L.first;
      const long long ticks = wait_ticks(b, L.maxsteps / nchunks + 1);
      const int stall = (b->test_stall == 1 && l == 0 && nchunks > 1) ? 0 : -1;
      LBM_HIP(launch_resident(L.q, L.prec, L.code, djobs + L.first, ditems, L.count, nchunks, counters + l, slots,
                              done, b->coefs, b->status, ticks, stall, grid, L.block, L.lds, st));
    } else if (it.kind == 1) {
      const TileGroup& G = tgroups[it.idx];
      DevTile* dt = b->tiles + (size_t)k * b->tiles_cap + G.first;
      DevTileInst* dti = b->tinsts + (size_t)k * b->tinsts_cap;
      void* b0 = G.prec ? (void*)b->f32[0] : (void*)b->f64[0];
      void* b1 = G.prec ? (void*)b->f32[1] : (void*)b->f64[1];
      for (int l = 0; l < G.launches; ++l)
        LBM_HIP(launch_tile(G.q, G.prec, dt, G.ntiles, dti, b0, b1, l, G.s, G.halo, b->coefs, b->status, G.block,
                            G.lds, st));
      for (int t = G.tfirst; t < G.tfirst + G.tcount; ++t) {
        HostInst& h = b->inst[htin[t].inst];
        const int L = (int)((htin[t].steps + G.s - 1) / G.s);
        h.cur = htin[t].cur0 ^ (L & 1);
      }
    } else if (it.idx >= 0) {
      lbm_status s = issue_slab((size_t)it.idx, st);
      if (s != LBM_OK) return s;
    } else {
      for (size_t l = 0; l < slaunch.size(); ++l) {
        lbm_status s = issue_slab(l, st);
        if (s != LBM_OK) return s;
      }
    }
  }
  if (!slaunch.empty())
    for (const DevSlab& sl : svec)
      if (sl.x0 == 0) b->inst[htin[sl.ti].inst].cur ^= 1;   // one flip per instance: output in the other buffer
  if (fork) {
    for (int a = 0; a < nlanes; ++a) {
      if (!lane_forked[a]) continue;
      LBM_HIP(hipEventRecord(b->join[a], b->aux[a]));
      LBM_HIP(hipStreamWaitEvent(b->stream, b->join[a], 0));
    }
  }
  LBM_HIP(hipEventRecord(b->items_done[k], b->stream));
  // streaming instances: one fused collide+stream launch per step, whole
  // blocks of kStepBlock steps replayed from a graph
  for (int i : str) {
    HostInst& h = b->inst[i];
    lbm_status s = ensure_second_buffer(b, h.f32);
    if (s != LBM_OK) return s;
    int64_t t = 0;
    if (steps[i] >= 2 * kStepBlock) {
      StepGraph* g = nullptr;
      s = step_graph(b, i, &g);
      if (s != LBM_OK) return s;
      for (; t + kStepBlock <= steps[i]; t += kStepBlock) LBM_HIP(hipGraphLaunch(g->exec, b->stream));
    }
    for (; t < steps[i]; ++t) {
      LBM_HIP(launch_stream(h.q, h.D, h.prec, state_cur(b, h), state_other(b, h), h.n, h.stride, b->coefs + i,
                            b->stream));
      h.cur = 1 - h.cur;
    }
  }
  LBM_HIP(hipEventRecord(b->ev1, b->stream));
  for (int i = 0; i < count; ++i) b->inst[i].steps_done += steps[i];
  return LBM_OK;
}

lbm_status advance(lbm_batch_s* b, const int64_t* steps) {
  const int count = (int)b->inst.size();
  std::vector<int64_t> left(steps, steps + count);
  for (int64_t v : left)
    if (v < 0) return LBM_ERR_INVALID_ARG;
  for (;;) {
    std::vector<int64_t> now(count);
    bool any = false;
    for (int i = 0; i < count; ++i) {
      now[i] = std::min(left[i], kMaxStepsPerLaunch);
      left[i] -= now[i];
      any |= now[i] > 0;
    }
    if (!any) return LBM_OK;
    lbm_status s = advance_pass(b, now.data());
    if (s != LBM_OK) return s;
  }
}

// phi of instance i into the device scratch buffer; raises b->flag on NaN/Inf
lbm_status phi_to_scratch(lbm_batch_s* b, int i) {
  HostInst& h = b->inst[i];
  LBM_HIP(hipMemsetAsync(b->flag, 0, sizeof(int), b->stream));
  LBM_HIP(launch_phi(h.prec, state_cur(b, h), b->scratch, h.n, h.stride, h.q, h.f32 ? h.mdl.phi_rest : 0.0,
                     b->flag, b->stream));
  return LBM_OK;
}

lbm_status read_phi(lbm_batch_s* b, int i, double* out, int on_device, lbm_status* inst_status) {
  HostInst& h = b->inst[i];
  lbm_status s0 = phi_to_scratch(b, i);
  if (s0 != LBM_OK) return s0;
  LBM_HIP(hipMemcpyAsync(out, b->scratch, sizeof(double) * h.n,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
  int flags[2] = {0, 0};
  LBM_HIP(hipMemcpyAsync(&flags[0], b->flag, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  LBM_HIP(hipMemcpyAsync(&flags[1], b->status + i, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  LBM_HIP(hipStreamSynchronize(b->stream));
  // status bit 1: a non-finite value; bits 2 and 4: a device wait for a
  // cooperating workgroup gave up, so the state was not advanced as asked
  lbm_status s = (flags[1] & 6) ? LBM_ERR_TIMEOUT : (flags[0] || flags[1]) ? LBM_ERR_NONFINITE : LBM_OK;
  if (inst_status) *inst_status = s;
  return s;
}

// ---------------------------------------------------------------------------
// Autotuning: time candidate planner settings on a copy of the batch (same
// descriptors, coefficients and state) and keep the fastest.  The planner's
// choices it covers: the tile shape and steps per launch of the temporal-
// blocking path (instances that do not fit one workgroup's LDS), the step
// chunking of the resident path, and -- for small batches -- the LDS-resident
// vs HBM-streaming choice itself.
// ---------------------------------------------------------------------------
struct Knobs {
  int path, tile_steps, tile_wgs, res_grid, res_chunks;
};
constexpr double kTuneMargin = 0.97;

Knobs knobs_of(const lbm_batch_s* b) { return Knobs{b->path, b->tile_steps, b->tile_wgs, b->res_grid, b->res_chunks}; }

void set_knobs(lbm_batch_s* b, const Knobs& k) {
  b->path = k.path;
  b->tile_steps = k.tile_steps;
  b->tile_wgs = k.tile_wgs;
  b->res_grid = k.res_grid;
  b->res_chunks = k.res_chunks;
}

lbm_status clone_for_tuning(lbm_batch_s* b, lbm_batch_s** out) {
  const int count = (int)b->inst.size();
  std::vector<lbm_desc> d(count);
  for (int i = 0; i < count; ++i) d[i] = b->inst[i].desc;
  lbm_batch_s* c = nullptr;
  lbm_status s = create_batch(d.data(), count, b->stream, nullptr, 0, &c);
  if (s != LBM_OK) return s;
  // same descriptors in the same order: same layout; copy coefficients and state
  for (int i = 0; i < count && s == LBM_OK; ++i) {
    c->inst[i].mdl = b->inst[i].mdl;
    c->inst[i].cur = b->inst[i].cur;
    c->hcoef[i] = b->hcoef[i];
  }
  auto copy = [&](void* dst, const void* src, size_t bytes) -> lbm_status {
    if (!bytes) return LBM_OK;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, b->stream) == hipSuccess ? LBM_OK
                                                                                           : LBM_ERR_DEVICE;
  };
  if (s == LBM_OK) s = copy(c->coefs, b->coefs, sizeof(DevCoef) * count);
  for (int k = 0; k < 2 && s == LBM_OK; ++k) {
    if (b->f64[k]) {
      if (k == 1) s = ensure_second_buffer(c, false);
      if (s == LBM_OK) s = copy(c->f64[k], b->f64[k], sizeof(double) * b->n64);
    }
    if (b->f32[k] && s == LBM_OK) {
      if (k == 1) s = ensure_second_buffer(c, true);
      if (s == LBM_OK) s = copy(c->f32[k], b->f32[k], sizeof(float) * b->n32);
    }
  }
  if (s == LBM_OK && hipStreamSynchronize(b->stream) != hipSuccess) s = LBM_ERR_DEVICE;
  if (s != LBM_OK) {
    destroy_batch(c);
    return s;
  }
  *out = c;
  return LBM_OK;
}

// device time (ms) of one pass of `probe` steps with knobs k: best of two after a warm-up pass
lbm_status time_knobs(lbm_batch_s* c, const Knobs& k, int64_t probe, double* ms) {
  set_knobs(c, k);
  std::vector<int64_t> st(c->inst.size(), probe);
  double best = 1e300;
  for (int r = 0; r < 3; ++r) {
    lbm_status s = advance(c, st.data());
    if (s != LBM_OK) return s;
    LBM_HIP(hipEventSynchronize(c->ev1));
    float t = 0.0f;
    LBM_HIP(hipEventElapsedTime(&t, c->ev0, c->ev1));
    if (r > 0) best = std::min(best, (double)t);
  }
  *ms = best;
  return LBM_OK;
}

lbm_status autotune(lbm_batch_s* b, int64_t probe, lbm_tuning* out) {
  const int count = (int)b->inst.size();
  bool any_fit = false, any_big = false;
  double nodes = 0.0;
  int64_t minn = INT64_MAX;
  for (const HostInst& h : b->inst) {
    const bool f = fits_resident(b, h);
    any_fit |= f;
    any_big |= !f;
    nodes += h.n;
    minn = std::min<int64_t>(minn, h.n);
  }
  lbm_batch_s* c = nullptr;
  lbm_status s = clone_for_tuning(b, &c);
  if (s != LBM_OK) return s;
  int tried = 0;
  Knobs best{0, 0, 0, 0, 0};
  double best_ms = 0.0, default_ms = 0.0;
  s = time_knobs(c, best, probe, &default_ms);
  best_ms = default_ms;
  ++tried;
  auto consider = [&](const Knobs& k) {
    if (s != LBM_OK) return;
    double ms = 0.0;
    s = time_knobs(c, k, probe, &ms);
    ++tried;
    if (s == LBM_OK && ms < kTuneMargin * best_ms) {   // clear wins only, not timing noise
      best_ms = ms;
      best = k;
    }
  };
  // 1. temporal blocking: steps per launch x workgroups per CU
  if (any_big || minn >= 1024) {
    static const int kTiles[][2] = {{8, 2}, {16, 2}, {32, 2}, {64, 2}, {16, 1}, {32, 1}, {64, 1}};
    const int path = any_big ? best.path : 3;   // instances that fit: try them tiled as well
    for (const auto& t : kTiles) consider(Knobs{path, t[0], t[1], 0, 0});
    if (!any_big) consider(Knobs{3, 0, 0, 0, 0});
  }
  // 2. resident step chunks
  if (any_fit && best.path != 3) {
    static const int kChunks[] = {1, 4, 8, 16, 32};
    const Knobs base = best;
    for (int ch : kChunks) consider(Knobs{base.path, base.tile_steps, base.tile_wgs, 0, ch});
  }
  // 3. HBM streaming, one launch per step: only for a few instances
  if (count <= 16 && nodes * (double)probe <= 2.5e8) consider(Knobs{1, 0, 0, 0, 0});
  destroy_batch(c);
  if (s != LBM_OK) return s;
  set_knobs(b, best);
  if (out) {
    out->path = best.path;
    out->tile_steps = best.tile_steps;
    out->tile_wgs = best.tile_wgs;
    out->res_chunks = best.res_chunks;
    out->candidates = tried;
    out->pad_ = 0;
    out->best_node_updates_per_s = nodes * (double)probe / (best_ms * 1e-3);
    out->default_node_updates_per_s = nodes * (double)probe / (default_ms * 1e-3);
  }
  return LBM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* lbm_status_str(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID_ARG: return "invalid argument";
    case LBM_ERR_UNSUPPORTED: return "unsupported";
    case LBM_ERR_SINGULAR_TAU: return "singular relaxation polynomial tau_k";
    case LBM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case LBM_ERR_DEVICE: return "HIP runtime error";
    case LBM_ERR_NONFINITE: return "non-finite state";
    case LBM_ERR_BUSY: return "busy";
    case LBM_ERR_TIMEOUT: return "device wait timed out";
  }
  return "unknown status";
}

const char* lbm_version(void) { return "lbmhpde 0.1 gfx950"; }

int64_t lbm_row_stride(int64_t n) { return (n + 63) / 64 * 64; }

lbm_status lbm_validate(const lbm_desc* d) {
  if (!d) return LBM_ERR_INVALID_ARG;
  Model m;
  return build_model(*d, &m);
}

lbm_status lbm_coefficients(const lbm_desc* d, double* G, int32_t cap, int32_t* q_out, int32_t* degree_out) {
  if (!d || !G || !q_out || !degree_out) return LBM_ERR_INVALID_ARG;
  Model m;
  lbm_status s = build_model(*d, &m);
  if (s != LBM_OK) return s;
  if (m.gF > 0) return LBM_ERR_UNSUPPORTED;   // not a polynomial in phi
  if (cap < m.q * (m.D + 1)) return LBM_ERR_INVALID_ARG;
  for (int j = 0; j < m.q; ++j)
    for (int p = 0; p <= m.D; ++p) G[j * (m.D + 1) + p] = m.G[j][p];
  *q_out = m.q;
  *degree_out = m.D;
  return LBM_OK;
}

lbm_status lbm_coefficients_general(const lbm_desc* d, double* nu, double* G, int32_t cap, int32_t* classes_out,
                                    int32_t* q_out, int32_t* degree_out) {
  if (!d || !nu || !G || !classes_out || !q_out || !degree_out) return LBM_ERR_INVALID_ARG;
  Model m;
  lbm_status s = build_model(*d, &m);
  if (s != LBM_OK) return s;
  const int F = m.gF > 0 ? m.gF : 1;
  if (cap < F * m.q * (m.D + 1)) return LBM_ERR_INVALID_ARG;
  for (int c = 0; c < F; ++c) {
    nu[c] = m.gF > 0 ? m.gnu[c] : 0.0;
    for (int j = 0; j < m.q; ++j)
      for (int p = 0; p <= m.D; ++p) G[(c * m.q + j) * (m.D + 1) + p] = m.gF > 0 ? m.gG[c][j][p] : m.G[j][p];
  }
  *classes_out = F;
  *q_out = m.q;
  *degree_out = m.D;
  return LBM_OK;
}

lbm_status lbm_stability(const lbm_desc* d, double phi_min, double phi_max, int64_t steps,
                         double* growth_per_step, double* amplification) {
  if (!d || !growth_per_step || steps < 0 || !(phi_min <= phi_max) || !std::isfinite(phi_min) ||
      !std::isfinite(phi_max))
    return LBM_ERR_INVALID_ARG;
  Model m;
  lbm_status s = build_model(*d, &m);
  if (s != LBM_OK) return s;
  if (m.gF > 1 && phi_min <= 0) return LBM_ERR_INVALID_ARG;   // real powers: phi > 0 only
  const double g = stability_growth(m, phi_min, phi_max);
  *growth_per_step = g;
  if (amplification) *amplification = std::pow(g, (double)steps);
  return LBM_OK;
}

lbm_status lbm_required_bytes(const lbm_desc* d, size_t* bytes) {
  if (!d || !bytes) return LBM_ERR_INVALID_ARG;
  Model m;
  lbm_status s = build_model(*d, &m);
  if (s != LBM_OK) return s;
  size_t es = d->prec == LBM_F64 ? sizeof(double) : sizeof(float);
  *bytes = (size_t)m.q * (size_t)lbm_row_stride(d->n) * es;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_desc* d, void* stream, void* dev_buf, size_t buf_bytes, lbm_problem* out) {
  if (!d || !out) return LBM_ERR_INVALID_ARG;
  lbm_batch_s* b = nullptr;
  lbm_status s = create_batch(d, 1, stream, dev_buf, buf_bytes, &b);
  if (s != LBM_OK) return s;
  lbm_problem_s* p = new (std::nothrow) lbm_problem_s();
  if (!p) {
    destroy_batch(b);
    return LBM_ERR_OUT_OF_MEMORY;
  }
  p->b = b;
  *out = p;
  return LBM_OK;
}

lbm_status lbm_load_phi(lbm_problem h, const double* phi, int phi_on_device) {
  if (!h || !phi) return LBM_ERR_INVALID_ARG;
  return load_phi_one(h->b, 0, phi, phi_on_device);
}

lbm_status lbm_advance(lbm_problem h, int64_t steps) {
  if (!h || steps < 0) return LBM_ERR_INVALID_ARG;
  return advance(h->b, &steps);
}

// lbm_create + lbm_load_phi + lbm_advance + lbm_read_phi of one periodic
// problem whose state fits one workgroup's LDS, with every device buffer in
// the fixed per-device scratch (noalloc.hip): the same kernels (k_init, one
// resident launch per 2^30 steps, k_phi), so the result is bitwise that of the
// handle path.  Host-side buffers live on this call's stack.
lbm_status lbm_advance_noalloc(const lbm_desc* d, const double* phi0, int64_t steps, double* phi, void* stream) {
  if (!d || !phi0 || !phi || steps < 0 || d->n < 1 || d->n > kNoAllocMaxNodes) return LBM_ERR_INVALID_ARG;
  if (d->bc != LBM_BC_PERIODIC) return LBM_ERR_INVALID_ARG;
  const hipStream_t st = (hipStream_t)stream;
  HostInst h;
  lbm_status s = prepare_one(*d, &h);
  if (s != LBM_OK) return s;
  const DeviceLimits lim = query_limits();
  if (!lim.ok) return LBM_ERR_DEVICE;
  const size_t es = elem_size(h);
  const size_t lds = ((size_t)lds_stride(h.q) * h.n * es + 15) / 16 * 16;
  if ((size_t)h.q * h.stride * es > kNoAllocStateBytes || lds + resident_static_lds(h.q, h.prec, h.D) > lim.lds_max)
    return LBM_ERR_INVALID_ARG;
  void* base = nullptr;
  LBM_HIP(noalloc_scratch(&base));
  // tables at the start of the scratch, the state after them
  static_assert(sizeof(DevCoef) <= 12288, "coefficient table outgrew its scratch region");
  unsigned char* bytes = (unsigned char*)base;
  DevCoef* dcoef = (DevCoef*)bytes;
  DevJob* djob = (DevJob*)(bytes + 12288);
  DevJobInst* dji = (DevJobInst*)(bytes + 12288 + 256);
  int* ints = (int*)(bytes + 12288 + 512);   // queue counter, slot, done, status, non-finite flag
  void* f = bytes + kNoAllocTableBytes;
  // phi0 on the host: the checks of lbm_load_phi and the rest state (mean of phi0)
  double host[kNoAllocMaxNodes];
  LBM_HIP(hipMemcpyAsync(host, phi0, sizeof(double) * h.n, hipMemcpyDeviceToHost, st));
  LBM_HIP(hipStreamSynchronize(st));
  long double sum = 0;
  for (int i = 0; i < h.n; ++i) {
    if (!std::isfinite(host[i]) || (h.mdl.gF > 1 && host[i] < 0)) return LBM_ERR_INVALID_ARG;
    sum += host[i];
  }
  if (h.f32) set_rest_state(&h.mdl, (double)(sum / h.n));
  DevCoef cf;
  fill_devcoef(h, &cf);
  // one job of one instance: a wave per 64 nodes, at most 16
  const int waves = std::max(1, std::min(16, (h.n + 63) / 64));
  DevJob jb{0, 1, 0, h.D, 0, 0};
  DevJobInst ji{};
  ji.addr = (uint64_t)(uintptr_t)f;
  ji.n = h.n;
  ji.stride = h.stride;
  ji.degree = h.D;
  ji.nt = 64 * waves;
  LBM_HIP(hipMemcpyAsync(dcoef, &cf, sizeof(cf), hipMemcpyHostToDevice, st));
  LBM_HIP(hipMemcpyAsync(dji, &ji, sizeof(ji), hipMemcpyHostToDevice, st));
  LBM_HIP(launch_zero_ints(ints, 5, st));
  LBM_HIP(launch_init(h.q, h.Dinit, h.prec, phi0, f, h.n, h.stride, dcoef, st));
  for (int64_t left = steps; left > 0;) {
    const int64_t now = std::min(left, kMaxStepsPerLaunch);
    left -= now;
    jb.steps = (int)now;
    LBM_HIP(hipMemcpyAsync(djob, &jb, sizeof(jb), hipMemcpyHostToDevice, st));
    LBM_HIP(hipStreamSynchronize(st));   // jb is reused by the next launch
    LBM_HIP(launch_zero_ints(ints, 3, st));
    LBM_HIP(launch_resident(h.q, h.prec, h.D, djob, dji, 1, 1, ints, ints + 1, ints + 2, dcoef, ints + 3, 0, -1, 1,
                            ji.nt, lds, st));
  }
  LBM_HIP(launch_phi(h.prec, f, phi, h.n, h.stride, h.q, h.f32 ? h.mdl.phi_rest : 0.0, ints + 4, st));
  int flags[2] = {0, 0};
  LBM_HIP(hipMemcpyAsync(flags, ints + 3, sizeof(flags), hipMemcpyDeviceToHost, st));
  LBM_HIP(hipStreamSynchronize(st));
  if (flags[0] & 6) return LBM_ERR_TIMEOUT;
  return (flags[0] || flags[1]) ? LBM_ERR_NONFINITE : LBM_OK;
}

}  // extern "C"

namespace {
// Where the boundary rows of a bounded call come from: host arrays (copied),
// or travelling waves evaluated on the device.
struct RowSource {
  const double* const* host = nullptr;   // per instance
  const lbm_wave* waves = nullptr;       // per instance
};

bool valid_wave(const lbm_wave* w) {
  if (!w) return false;
  if (w->shape < LBM_WAVE_SECH || w->shape > LBM_WAVE_COS) return false;
  const double v[] = {w->a, w->b, w->p, w->d, w->r, w->k, w->xc, w->c, w->x_first, w->t0};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  if (w->p < 0.0 || w->r < 0.0) return false;
  // tanh may be negative: integer exponents only
  if (w->shape == LBM_WAVE_TANH && (w->p != std::floor(w->p) || w->r != std::floor(w->r))) return false;
  return true;
}

// rows [steps][2 layers] of instance i into device memory dst (on b->stream)
lbm_status fill_rows(lbm_batch_s* b, int i, const RowSource& src, double* dst, int64_t steps, int layers) {
  const HostInst& h = b->inst[i];
  const size_t rows = (size_t)steps * 2 * layers;
  if (src.host) {
    LBM_HIP(hipMemcpy(dst, src.host[i], sizeof(double) * rows, hipMemcpyHostToDevice));
  } else {
    LBM_HIP(launch_wave_rows(dst, steps, layers, h.n, h.desc.dx, h.desc.dt, src.waves[i], b->stream));
  }
  return LBM_OK;
}

// Bounded instances of a batch advance `steps` (<= kMaxStepsPerLaunch) steps on
// the resident path, their boundary layers reset in LDS after every step;
// rows [steps][2 layers] of bounded instance i from `src`.
lbm_status advance_bounded_resident(lbm_batch_s* b, int64_t steps, const RowSource& src, int layers) {
  const int count = (int)b->inst.size();
  int nb = 0;
  for (int i = 0; i < count; ++i) nb += b->inst[i].desc.bc != LBM_BC_PERIODIC;
  const size_t rows = (size_t)steps * 2 * layers;
  const size_t need = rows * (size_t)nb;
  // a synchronous copy: earlier launches have read the buffer by the time it lands
  LBM_HIP(hipStreamSynchronize(b->stream));
  if (need > b->bound_cap) {
    hipFree(b->bound);
    b->bound = nullptr;
    b->bound_cap = 0;
    if (hipMalloc(&b->bound, sizeof(double) * need) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
    b->bound_cap = need;
  }
  b->bnd_ptr.assign(count, 0);
  for (int i = 0, k = 0; i < count; ++i) {
    if (b->inst[i].desc.bc == LBM_BC_PERIODIC) continue;
    double* dst = b->bound + (size_t)k++ * rows;
    lbm_status s = fill_rows(b, i, src, dst, steps, layers);
    if (s != LBM_OK) return s;
    b->bnd_ptr[i] = (uint64_t)(uintptr_t)dst;
  }
  b->bnd_active = true;
  b->bnd_layers = layers;
  std::vector<int64_t> st(count, steps);
  lbm_status s = advance_pass(b, st.data());
  b->bnd_active = false;
  return s;
}
lbm_status batch_advance_bounded(lbm_batch_s* b, int64_t steps, const RowSource& src, int layers) {
  if (steps < 0 || steps > kMaxStepsPerLaunch) return LBM_ERR_INVALID_ARG;
  int hmax = 0;
  for (const HostInst& h : b->inst)
    if (h.desc.bc != LBM_BC_PERIODIC) hmax = std::max(hmax, h.q / 2);
  if (layers == 0) layers = hmax;
  if (layers < hmax || layers > 32) return LBM_ERR_INVALID_ARG;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    const HostInst& h = b->inst[i];
    if (h.desc.bc == LBM_BC_PERIODIC) continue;
    if (src.host && steps > 0 && !src.host[i]) return LBM_ERR_INVALID_ARG;
    if (src.waves && !valid_wave(&src.waves[i])) return LBM_ERR_INVALID_ARG;
    if (h.n < 2 * layers + 2) return LBM_ERR_INVALID_ARG;
  }
  if (steps == 0) return LBM_OK;
  return advance_bounded_resident(b, steps, src, layers);
}

// device rows buffer of at least steps * 2 layers doubles (b->bound), no
// earlier launch still reading it
lbm_status bound_rows_buffer(lbm_batch_s* b, size_t need) {
  LBM_HIP(hipStreamSynchronize(b->stream));
  if (need > b->bound_cap) {
    hipFree(b->bound);
    b->bound = nullptr;
    b->bound_cap = 0;
    if (hipMalloc(&b->bound, sizeof(double) * need) != hipSuccess) return LBM_ERR_OUT_OF_MEMORY;
    b->bound_cap = need;
  }
  return LBM_OK;
}

// single bounded problem: `layers` resolved and checked against the problem
lbm_status bounded_layers(const HostInst& in, int32_t* layers) {
  if (in.desc.bc != LBM_BC_DIRICHLET_EQ && in.desc.bc != LBM_BC_DIRICHLET_NEE) return LBM_ERR_INVALID_ARG;
  const int H = in.q / 2;
  if (*layers == 0) *layers = H;
  if (*layers < H || *layers > 32 || in.n < 2 * *layers + 2) return LBM_ERR_INVALID_ARG;
  return LBM_OK;
}

lbm_status advance_bounded_one(lbm_batch_s* b, int64_t steps, const RowSource& src, int32_t layers) {
  HostInst& in = b->inst[0];
  lbm_status s = bounded_layers(in, &layers);
  if (s != LBM_OK) return s;
  if (src.waves && !valid_wave(src.waves)) return LBM_ERR_INVALID_ARG;
  if (steps == 0) return LBM_OK;
  // LDS-resident unless the streaming path is asked for or the state does not fit
  if ((b->path == 0 || b->path == 2) && fits_resident(b, in) && steps <= kMaxStepsPerLaunch)
    return advance_bounded_resident(b, steps, src, layers);
  s = ensure_second_buffer(b, in.f32);
  if (s != LBM_OK) return s;
  const size_t need = (size_t)steps * 2 * layers;
  s = bound_rows_buffer(b, need);
  if (s != LBM_OK) return s;
  s = fill_rows(b, 0, src, b->bound, steps, layers);
  if (s != LBM_OK) return s;
  const int kind = in.desc.bc == LBM_BC_DIRICHLET_EQ ? 1 : 2;
  LBM_HIP(hipEventRecord(b->ev0, b->stream));
  for (int64_t t = 0; t < steps; ++t) {
    LBM_HIP(launch_stream(in.q, in.D, in.prec, state_cur(b, in), state_other(b, in), in.n, in.stride, b->coefs,
                          b->stream));
    in.cur = 1 - in.cur;
    LBM_HIP(launch_bound(in.q, in.Dinit, in.prec, state_cur(b, in), in.n, in.stride, layers, kind,
                         b->bound + (size_t)t * 2 * layers, b->coefs, b->stream));
  }
  LBM_HIP(hipEventRecord(b->ev1, b->stream));
  in.steps_done += steps;
  return LBM_OK;
}
}  // namespace

extern "C" {

lbm_status lbm_batch_advance_bounded(lbm_batch b, int64_t steps, const double* const* phib, int32_t layers) {
  if (!b) return LBM_ERR_INVALID_ARG;
  for (const HostInst& h : b->inst)
    if (h.desc.bc != LBM_BC_PERIODIC && steps > 0 && !phib) return LBM_ERR_INVALID_ARG;
  RowSource src;
  src.host = phib;
  return batch_advance_bounded(b, steps, src, layers);
}

lbm_status lbm_batch_advance_bounded_wave(lbm_batch b, int64_t steps, const lbm_wave* waves, int32_t layers) {
  if (!b || !waves) return LBM_ERR_INVALID_ARG;
  RowSource src;
  src.waves = waves;
  return batch_advance_bounded(b, steps, src, layers);
}

lbm_status lbm_advance_bounded(lbm_problem h, int64_t steps, const double* phib, int32_t layers) {
  if (!h || steps < 0 || (steps > 0 && !phib)) return LBM_ERR_INVALID_ARG;
  const double* rows[1] = {phib};
  RowSource src;
  src.host = rows;
  return advance_bounded_one(h->b, steps, src, layers);
}

lbm_status lbm_advance_bounded_wave(lbm_problem h, int64_t steps, const lbm_wave* w, int32_t layers) {
  if (!h || steps < 0 || !w) return LBM_ERR_INVALID_ARG;
  RowSource src;
  src.waves = w;
  return advance_bounded_one(h->b, steps, src, layers);
}

lbm_status lbm_wave_rows(lbm_problem h, int64_t steps, const lbm_wave* w, int32_t layers, double* out) {
  if (!h || steps < 0 || !w || (steps > 0 && !out) || !valid_wave(w)) return LBM_ERR_INVALID_ARG;
  lbm_batch_s* b = h->b;
  lbm_status s = bounded_layers(b->inst[0], &layers);
  if (s != LBM_OK) return s;
  if (steps == 0) return LBM_OK;
  const size_t need = (size_t)steps * 2 * layers;
  s = bound_rows_buffer(b, need);
  if (s != LBM_OK) return s;
  RowSource src;
  src.waves = w;
  s = fill_rows(b, 0, src, b->bound, steps, layers);
  if (s != LBM_OK) return s;
  LBM_HIP(hipStreamSynchronize(b->stream));
  LBM_HIP(hipMemcpy(out, b->bound, sizeof(double) * need, hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_read_phi(lbm_problem h, double* out, int out_on_device) {
  if (!h || !out) return LBM_ERR_INVALID_ARG;
  return read_phi(h->b, 0, out, out_on_device, nullptr);
}

lbm_status lbm_sum_phi(lbm_problem h, double* total) {
  if (!h || !total) return LBM_ERR_INVALID_ARG;
  lbm_batch_s* b = h->b;
  HostInst& hi = b->inst[0];
  lbm_status s = phi_to_scratch(b, 0);
  if (s != LBM_OK) return s;
  // deterministic FP64 reduction: fixed partition on the device, fixed order on the host
  const int parts = 64;
  double* part = b->scratch + hi.n;
  LBM_HIP(launch_sum(b->scratch, hi.n, part, parts, b->stream));
  double hp[parts];
  LBM_HIP(hipMemcpyAsync(hp, part, sizeof(hp), hipMemcpyDeviceToHost, b->stream));
  LBM_HIP(hipStreamSynchronize(b->stream));
  double t = 0.0;
  for (int i = 0; i < parts; ++i) t += hp[i];
  *total = t;
  return std::isfinite(t) ? LBM_OK : LBM_ERR_NONFINITE;
}

lbm_status lbm_state_bytes(lbm_problem h, size_t* bytes) {
  if (!h || !bytes) return LBM_ERR_INVALID_ARG;
  const HostInst& hi = h->b->inst[0];
  *bytes = 32 + (size_t)hi.q * hi.n * elem_size(hi);
  return LBM_OK;
}

lbm_status lbm_save_f(lbm_problem h, void* host_buf, size_t bytes) {
  if (!h || !host_buf) return LBM_ERR_INVALID_ARG;
  lbm_batch_s* b = h->b;
  HostInst& hi = b->inst[0];
  size_t need = 0;
  lbm_state_bytes(h, &need);
  if (bytes < need) return LBM_ERR_INVALID_ARG;
  unsigned char* p = (unsigned char*)host_buf;
  uint64_t hdr[4] = {kMagic, (uint64_t)hi.steps_done, (uint64_t)hi.q | ((uint64_t)hi.f32 << 32), (uint64_t)hi.n};
  std::memcpy(p, hdr, 32);
  const size_t row = (size_t)hi.n * elem_size(hi);
  for (int j = 0; j < hi.q; ++j) {
    const void* src = hi.f32 ? (const void*)(f32_cur(b, hi) + (size_t)j * hi.stride)
                             : (const void*)(f64_cur(b, hi) + (size_t)j * hi.stride);
    LBM_HIP(hipMemcpyAsync(p + 32 + j * row, src, row, hipMemcpyDeviceToHost, b->stream));
  }
  LBM_HIP(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

lbm_status lbm_load_f(lbm_problem h, const void* host_buf, size_t bytes) {
  if (!h || !host_buf) return LBM_ERR_INVALID_ARG;
  lbm_batch_s* b = h->b;
  HostInst& hi = b->inst[0];
  size_t need = 0;
  lbm_state_bytes(h, &need);
  if (bytes < need) return LBM_ERR_INVALID_ARG;
  const unsigned char* p = (const unsigned char*)host_buf;
  uint64_t hdr[4];
  std::memcpy(hdr, p, 32);
  if (hdr[0] != kMagic || hdr[2] != ((uint64_t)hi.q | ((uint64_t)hi.f32 << 32)) || hdr[3] != (uint64_t)hi.n)
    return LBM_ERR_INVALID_ARG;
  const size_t row = (size_t)hi.n * elem_size(hi);
  for (int j = 0; j < hi.q; ++j) {
    void* dst = hi.f32 ? (void*)(f32_cur(b, hi) + (size_t)j * hi.stride)
                       : (void*)(f64_cur(b, hi) + (size_t)j * hi.stride);
    LBM_HIP(hipMemcpyAsync(dst, p + 32 + j * row, row, hipMemcpyHostToDevice, b->stream));
  }
  LBM_HIP(hipMemsetAsync(b->status, 0, sizeof(int), b->stream));
  LBM_HIP(hipStreamSynchronize(b->stream));
  hi.steps_done = (int64_t)hdr[1];
  return LBM_OK;
}

lbm_status lbm_set_path(lbm_problem h, int32_t path) {
  if (!h || path < 0 || path > 4) return LBM_ERR_INVALID_ARG;
  h->b->path = path;
  return LBM_OK;
}

lbm_status lbm_last_advance_ms(lbm_problem h, float* ms) {
  if (!h || !ms) return LBM_ERR_INVALID_ARG;
  return lbm_batch_last_advance_ms(h->b, ms);
}

lbm_status lbm_destroy(lbm_problem h) {
  if (!h) return LBM_ERR_INVALID_ARG;
  destroy_batch(h->b);
  delete h;
  return LBM_OK;
}

lbm_status lbm_batch_create(const lbm_desc* descs, int32_t count, void* stream, lbm_batch* out) {
  return create_batch(descs, count, stream, nullptr, 0, out);
}

lbm_status lbm_batch_load_phi(lbm_batch b, const double* const* phi0) {
  if (!b || !phi0) return LBM_ERR_INVALID_ARG;
  for (size_t i = 0; i < b->inst.size(); ++i)
    if (!phi0[i]) return LBM_ERR_INVALID_ARG;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    lbm_status s = load_phi_one(b, (int)i, phi0[i], 0);
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

lbm_status lbm_batch_advance(lbm_batch b, const int64_t* steps) {
  if (!b) return LBM_ERR_INVALID_ARG;
  if (!steps) return LBM_OK;
  return advance(b, steps);
}

lbm_status lbm_batch_read_phi(lbm_batch b, int32_t i, double* out, lbm_status* inst_status) {
  if (!b || !out || i < 0 || i >= (int32_t)b->inst.size()) return LBM_ERR_INVALID_ARG;
  lbm_status s = read_phi(b, i, out, 0, inst_status);
  return (s == LBM_ERR_NONFINITE || s == LBM_ERR_TIMEOUT) ? LBM_OK : s;
}

lbm_status lbm_batch_last_advance_ms(lbm_batch b, float* ms) {
  if (!b || !ms) return LBM_ERR_INVALID_ARG;
  LBM_HIP(hipEventSynchronize(b->ev1));
  LBM_HIP(hipEventElapsedTime(ms, b->ev0, b->ev1));
  return LBM_OK;
}

lbm_status lbm_batch_set_path(lbm_batch b, int32_t path) {
  if (!b || path < 0 || path > 4) return LBM_ERR_INVALID_ARG;
  b->path = path;
  return LBM_OK;
}

lbm_status lbm_batch_set_tiling(lbm_batch b, int32_t steps_per_launch, int32_t wgs_per_cu) {
  if (!b || steps_per_launch < 0 || steps_per_launch > 4096 || wgs_per_cu < 0 || wgs_per_cu > 8)
    return LBM_ERR_INVALID_ARG;
  b->tile_steps = steps_per_launch;
  b->tile_wgs = wgs_per_cu;
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch b, int64_t probe_steps, lbm_tuning* out) {
  if (!b || probe_steps < 1 || probe_steps > kMaxStepsPerLaunch) return LBM_ERR_INVALID_ARG;
  if (b->arena[0]) return LBM_ERR_UNSUPPORTED;   // server-owned batches re-plan every block
  return autotune(b, probe_steps, out);
}

lbm_status lbm_batch_set_resident(lbm_batch b, int32_t max_workgroups, int32_t chunks) {
  if (!b || max_workgroups < 0 || max_workgroups > kMaxResidentGrid || chunks < 0 || chunks > kMaxChunks)
    return LBM_ERR_INVALID_ARG;
  b->res_grid = max_workgroups;
  b->res_chunks = chunks;
  return LBM_OK;
}

lbm_status lbm_batch_set_lanes(lbm_batch b, int32_t lanes) {
  if (!b || lanes < 0 || lanes > kAuxStreams) return LBM_ERR_INVALID_ARG;
  b->lanes = lanes;
  return LBM_OK;
}

lbm_status lbm_batch_test_stall(lbm_batch b, int32_t what, int64_t wait_us) {
  if (!b || what < 0 || what > 2 || wait_us < 0 || wait_us > (int64_t(1) << 40)) return LBM_ERR_INVALID_ARG;
  b->test_stall = what;
  b->test_wait_us = wait_us;
  return LBM_OK;
}

lbm_status lbm_set_tiling(lbm_problem h, int32_t steps_per_launch, int32_t wgs_per_cu) {
  if (!h) return LBM_ERR_INVALID_ARG;
  return lbm_batch_set_tiling(h->b, steps_per_launch, wgs_per_cu);
}

lbm_status lbm_batch_destroy(lbm_batch b) {
  if (!b) return LBM_ERR_INVALID_ARG;
  destroy_batch(b);
  return LBM_OK;
}

}  // extern "C"

// ===========================================================================
// Serving: continuous batching of solve requests
// ===========================================================================
namespace {

// first-fit allocator over [0, size) in 256-byte units
struct Arena {
  struct Block { size_t off, len; };
  std::vector<Block> free;
  size_t size = 0;
  void init(size_t bytes) {
    size = bytes / 256 * 256;
    free.assign(1, Block{0, size});
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) / 256 * 256;
    for (size_t i = 0; i < free.size(); ++i) {
      if (free[i].len >= bytes) {
        *off = free[i].off;
        free[i].off += bytes;
        free[i].len -= bytes;
        if (free[i].len == 0) free.erase(free.begin() + i);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    size_t i = 0;
    while (i < free.size() && free[i].off < off) ++i;
    free.insert(free.begin() + i, Block{off, bytes});
    if (i + 1 < free.size() && free[i].off + free[i].len == free[i + 1].off) {
      free[i].len += free[i + 1].len;
      free.erase(free.begin() + i + 1);
    }
    if (i > 0 && free[i - 1].off + free[i - 1].len == free[i].off) {
      free[i - 1].len += free[i].len;
      free.erase(free.begin() + i);
    }
  }
  size_t available() const {
    size_t t = 0;
    for (const Block& b : free) t += b.len;
    return t;
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id;
  lbm_desc desc;
  std::vector<double> phi0;
  int64_t steps;
};

struct Slot {
  bool active = false;
  int64_t id = -1;
  int64_t remaining = 0;
  size_t off = 0, bytes = 0;
};

struct Result {
  std::vector<double> phi;
  lbm_status status;
  double t_submit = 0.0, t_admit = 0.0, t_retire = 0.0;   // host steady clock
};

size_t state_bytes_of(const lbm_desc& d) {
  const int q = resolved_lattice(d);
  const size_t es = d.prec == LBM_F64 ? sizeof(double) : sizeof(float);
  return (size_t)q * (size_t)lbm_row_stride(d.n) * es;
}

}  // namespace

struct lbm_server_s {
  lbm_batch_s* b = nullptr;
  Arena arena;
  int block = 1000;
  int64_t max_n = 0;
  int64_t next_id = 1;
  std::vector<Request> queue;        // FIFO
  std::vector<Slot> slots;
  std::vector<Result> results;       // indexed by id - 1 (kept until polled)
  std::vector<char> done;
  std::vector<int64_t> steps_buf;
  double node_updates = 0.0;
  double device_ms = 0.0;
  // a round launched and not yet retired (lbm_server_pump): its node updates
  bool inflight = false;
  bool inflight_empty = false;   // the round advanced nothing (only zero-step requests)
  double inflight_nu = 0.0;
};

extern "C" {

lbm_status lbm_server_create(void* stream, size_t budget_bytes, int32_t max_slots, int64_t max_n,
                             int32_t block_steps, lbm_server* out) {
  if (!out || max_slots <= 0 || max_slots > 65536 || max_n < 5 || max_n > (int64_t(1) << 30) ||
      block_steps <= 0 || budget_bytes < 4096)
    return LBM_ERR_INVALID_ARG;
  lbm_server_s* sv = new (std::nothrow) lbm_server_s();
  if (!sv) return LBM_ERR_OUT_OF_MEMORY;
  lbm_batch_s* b = new (std::nothrow) lbm_batch_s();
  if (!b) {
    delete sv;
    return LBM_ERR_OUT_OF_MEMORY;
  }
  sv->b = b;
  b->stream = (hipStream_t)stream;
  b->lim = query_limits();
  b->inst.resize(max_slots);
  lbm_status s = b->lim.ok ? LBM_OK : LBM_ERR_DEVICE;
  // two mirrored arenas: the current state and the other buffer of the tiled path
  sv->arena.init(budget_bytes);
  for (int k = 0; k < 2 && s == LBM_OK; ++k)
    if (hipMalloc(&b->arena[k], sv->arena.size) != hipSuccess) s = LBM_ERR_OUT_OF_MEMORY;
  if (s == LBM_OK) {
    b->f64[0] = (double*)b->arena[0];
    b->f32[0] = (float*)b->arena[0];
    b->f64[1] = (double*)b->arena[1];
    b->f32[1] = (float*)b->arena[1];
    b->n64 = sv->arena.size / sizeof(double);
    b->n32 = sv->arena.size / sizeof(float);
    s = alloc_tables(b, (size_t)max_n);
  }
  if (s != LBM_OK) {
    destroy_batch(b);
    delete sv;
    return s;
  }
  sv->block = block_steps;
  sv->max_n = max_n;
  sv->slots.resize(max_slots);
  sv->steps_buf.assign(max_slots, 0);
  *out = sv;
  return LBM_OK;
}

lbm_status lbm_server_submit(lbm_server sv, const lbm_desc* d, const double* phi0, int64_t steps, int64_t* id) {
  if (!sv || !d || !phi0 || !id || steps < 0) return LBM_ERR_INVALID_ARG;
  // the checks admission repeats: the model, its kernel variant and phi0
  HostInst probe;
  lbm_status s = prepare_one(*d, &probe);
  if (s != LBM_OK) return s;
  if (d->n > sv->max_n) return LBM_ERR_INVALID_ARG;
  if (d->bc != LBM_BC_PERIODIC) return LBM_ERR_UNSUPPORTED;   // requests carry no boundary data
  if (state_bytes_of(*d) > sv->arena.size) return LBM_ERR_OUT_OF_MEMORY;
  for (int64_t i = 0; i < d->n; ++i)
    if (!std::isfinite(phi0[i]) || (probe.mdl.gF > 1 && phi0[i] < 0)) return LBM_ERR_INVALID_ARG;
  Request r;
  r.id = sv->next_id++;
  r.desc = *d;
  r.phi0.assign(phi0, phi0 + d->n);
  r.steps = steps;
  sv->queue.push_back(std::move(r));
  sv->results.emplace_back();
  sv->results.back().t_submit = now_s();
  sv->done.push_back(0);
  *id = sv->queue.back().id;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Admission: queued requests in arrival order while a slot and arena space
// are free (f := f_eq(phi0) on the stream, which it synchronises).
void server_admit(lbm_server_s* sv) {
  lbm_batch_s* b = sv->b;
  size_t qi = 0;
  for (; qi < sv->queue.size(); ++qi) {
    Request& r = sv->queue[qi];
    int slot = -1;
    for (size_t k = 0; k < sv->slots.size(); ++k)
      if (!sv->slots[k].active) {
        slot = (int)k;
        break;
      }
    if (slot < 0) break;
    const size_t bytes = state_bytes_of(r.desc);
    size_t off = 0;
    if (!sv->arena.alloc(bytes, &off)) break;   // FIFO: wait for space
    HostInst& h = b->inst[slot];
    lbm_status s = prepare_one(r.desc, &h);
    if (s == LBM_OK) {
      h.off = (int64_t)(off / (h.f32 ? sizeof(float) : sizeof(double)));
      s = load_phi_one(b, slot, r.phi0.data(), 0);
    }
    Result& res = sv->results[r.id - 1];
    res.t_admit = now_s();
    if (s != LBM_OK) {
      // submission ran the same checks, so this is a device error: the request
      // retires with it (no phi) and the queue moves on
      sv->arena.release(off, bytes);
      h = HostInst();
      res.status = s;
      res.t_retire = res.t_admit;
      sv->done[r.id - 1] = 1;
      continue;
    }
    Slot& sl = sv->slots[slot];
    sl.active = true;
    sl.id = r.id;
    sl.remaining = r.steps;
    sl.off = off;
    sl.bytes = bytes;
  }
  sv->queue.erase(sv->queue.begin(), sv->queue.begin() + qi);
}

// One block for every active request in one planner pass (asynchronous on
// the stream).  A round lasts as long as its slowest request's block;
// requests whose steps take less time take proportionally more steps in the
// same round, up to 8 blocks.  A step's time is estimated as its arithmetic
// per node (lattice size x polynomial degree) times the node sweeps of one
// workgroup (1024 threads; larger grids are spread over several).
lbm_status server_launch(lbm_server_s* sv, int* act_out) {
  lbm_batch_s* b = sv->b;
  auto step_cost = [&](size_t k) {
    const HostInst& h = b->inst[k];
    const int sweeps = (std::min(h.n, 4096) + 1023) / 1024;
    return (double)h.q * ((h.D & 0xff) + 3) * sweeps;
  };
  double cmax = 0.0;
  for (size_t k = 0; k < sv->slots.size(); ++k)
    if (sv->slots[k].active) cmax = std::max(cmax, step_cost(k));
  int act = 0;
  double nu = 0.0;
  for (size_t k = 0; k < sv->slots.size(); ++k) {
    const Slot& sl = sv->slots[k];
    const double scale = sl.active ? std::min(8.0, std::max(1.0, cmax / step_cost(k))) : 1.0;
    sv->steps_buf[k] = sl.active ? std::min<int64_t>(sl.remaining, (int64_t)(sv->block * scale)) : 0;
    if (sl.active) {
      ++act;
      nu += (double)sv->steps_buf[k] * b->inst[k].n;
    }
  }
  *act_out = act;
  if (!act) return LBM_OK;
  sv->inflight_empty = nu == 0.0;
  if (!sv->inflight_empty) {
    lbm_status s = advance(b, sv->steps_buf.data());
    if (s != LBM_OK) return s;
  }
  sv->inflight = true;
  sv->inflight_nu = nu;
  return LBM_OK;
}

// The launched round has finished on the device: account for it, retire the
// requests it completed (phi read out, space released).
lbm_status server_finish(lbm_server_s* sv, int* retired) {
  lbm_batch_s* b = sv->b;
  if (!sv->inflight_empty) {
    float ms = 0.0f;
    LBM_HIP(hipEventSynchronize(b->ev1));
    if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) sv->device_ms += ms;
  }
  sv->node_updates += sv->inflight_nu;
  sv->inflight = false;
  sv->inflight_nu = 0.0;
  int ret = 0;
  for (size_t k = 0; k < sv->slots.size(); ++k) {
    Slot& sl = sv->slots[k];
    if (!sl.active) continue;
    sl.remaining -= sv->steps_buf[k];
    sv->steps_buf[k] = 0;
    if (sl.remaining > 0) continue;
    Result& res = sv->results[sl.id - 1];
    res.phi.resize(b->inst[k].n);
    lbm_status st = LBM_OK;
    lbm_status s = read_phi(b, (int)k, res.phi.data(), 0, &st);
    if (s != LBM_OK && s != LBM_ERR_NONFINITE && s != LBM_ERR_TIMEOUT) return s;
    res.status = st;
    res.t_retire = now_s();
    sv->done[sl.id - 1] = 1;
    sv->arena.release(sl.off, sl.bytes);
    sl = Slot();
    ++ret;
  }
  *retired = ret;
  return LBM_OK;
}

void server_counts(const lbm_server_s* sv, int32_t* active, int32_t* queued) {
  int act = 0;
  for (const Slot& sl : sv->slots) act += sl.active ? 1 : 0;
  if (active) *active = act;
  if (queued) *queued = (int32_t)sv->queue.size();
}

}  // namespace

extern "C" {

// One synchronous scheduling round: finish a round a pump left running,
// admit, advance every active request by one block (all concurrent on the
// device), wait, retire.
lbm_status lbm_server_step(lbm_server sv, int32_t* active, int32_t* queued, int32_t* retired) {
  if (!sv) return LBM_ERR_INVALID_ARG;
  int ret = 0, r = 0, act = 0;
  if (sv->inflight) {
    lbm_status s = server_finish(sv, &r);
    if (s != LBM_OK) return s;
    ret += r;
  }
  server_admit(sv);
  lbm_status s = server_launch(sv, &act);
  if (s != LBM_OK) return s;
  if (sv->inflight) {
    s = server_finish(sv, &r);
    if (s != LBM_OK) return s;
    ret += r;
  }
  server_counts(sv, active, queued);
  if (retired) *retired = ret;
  return LBM_OK;
}

// Continuous batching without blocking the caller: while a round runs on the
// device, return at once (*running = 1); once it has finished, retire what it
// completed, admit queued requests and launch the next round.
lbm_status lbm_server_pump(lbm_server sv, int32_t* running, int32_t* active, int32_t* queued, int32_t* retired) {
  if (!sv) return LBM_ERR_INVALID_ARG;
  int ret = 0, act = 0;
  if (sv->inflight && !sv->inflight_empty) {
    const hipError_t q = hipEventQuery(sv->b->ev1);
    if (q == hipErrorNotReady) {
      if (running) *running = 1;
      server_counts(sv, active, queued);
      if (retired) *retired = 0;
      return LBM_OK;
    }
    if (q != hipSuccess) return LBM_ERR_DEVICE;
  }
  if (sv->inflight) {
    lbm_status s = server_finish(sv, &ret);
    if (s != LBM_OK) return s;
  }
  server_admit(sv);
  lbm_status s = server_launch(sv, &act);
  if (s != LBM_OK) return s;
  if (running) *running = sv->inflight ? 1 : 0;
  server_counts(sv, active, queued);
  if (retired) *retired = ret;
  return LBM_OK;
}

lbm_status lbm_server_timing(lbm_server sv, int64_t id, double* queue_s, double* service_s) {
  if (!sv || id < 1 || id >= sv->next_id) return LBM_ERR_INVALID_ARG;
  if (sv->done[id - 1] == 0) return LBM_ERR_BUSY;
  const Result& r = sv->results[id - 1];
  if (queue_s) *queue_s = r.t_admit - r.t_submit;
  if (service_s) *service_s = r.t_retire - r.t_admit;
  return LBM_OK;
}

lbm_status lbm_server_poll(lbm_server sv, int64_t id, double* out, int64_t n, lbm_status* inst_status) {
  if (!sv || id < 1 || id >= sv->next_id) return LBM_ERR_INVALID_ARG;
  if (sv->done[id - 1] != 1) return sv->done[id - 1] == 2 ? LBM_ERR_INVALID_ARG : LBM_ERR_BUSY;
  Result& r = sv->results[id - 1];
  if (!out || n < (int64_t)r.phi.size()) return LBM_ERR_INVALID_ARG;
  std::memcpy(out, r.phi.data(), sizeof(double) * r.phi.size());
  if (inst_status) *inst_status = r.status;
  r.phi.clear();
  r.phi.shrink_to_fit();
  sv->done[id - 1] = 2;   // delivered
  return LBM_OK;
}

lbm_status lbm_server_stats(lbm_server sv, double* node_updates, double* device_ms, size_t* free_bytes) {
  if (!sv) return LBM_ERR_INVALID_ARG;
  if (node_updates) *node_updates = sv->node_updates;
  if (device_ms) *device_ms = sv->device_ms;
  if (free_bytes) *free_bytes = sv->arena.available();
  return LBM_OK;
}

lbm_status lbm_server_destroy(lbm_server sv) {
  if (!sv) return LBM_ERR_INVALID_ARG;
  destroy_batch(sv->b);
  delete sv;
  return LBM_OK;
}

}  // extern "C"
