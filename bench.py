"""Throughput of the batched LBGK hot path on one MI355X.

Workload: 4096 independent KdV / mKdV solitons (N log-uniform in [256, 4096],
periodic, 5000 time steps each, seeded).  One bench "step" advances the whole
batch by its 5000 lattice steps (one pass of the hot path over the batch).

Reported:
  value                 lattice-node updates per second of the batched FP32
                        deviation path (all instances, wall clock of the timed
                        passes, inputs resident in HBM)
  fp32_error            error of that FP32 path: against the FP64 batch on all
                        4096 instances after one pass, and against the CPU
                        oracle on the instances the CPU baseline runs
  fp64_batched          the same batch stored and computed in FP64
  plain_fp64            one instance at a time, one fused collide+stream launch
                        per step, FP64 (sampled instances)
  roofline              the dominant kernel (the persistent LDS-resident batch
                        kernel) against the VALU issue peak in the operation
                        count of one node update (FMA = 1 operation), timed with
                        HIP events on the launch stream; roofline_flops gives
                        the same in flops (FMA = 2) against 78.6 TFLOP/s
  hbm_stream            the fused collide+stream path on a 2^25-node grid:
                        algorithmic HBM GB/s against 8 TB/s and a device copy
  ks_batches            the 1024-run Kuramoto-Sivashinsky batches at N = 1024,
                        4096, 8192 to t = 20, FP64 and FP32, device time after
                        the autotuner has timed planner settings on a copy; FP32
                        error against FP64 on every run and both against the
                        stored oracle references
  kawahara_k22_batch    the 512-instance Kawahara + K(2,2) batch for 5000 steps
                        (autotuned likewise), the same measurements plus the
                        closed-form errors
  serving               a sweep of Poisson arrival rates of mixed solve requests
                        through the continuous-batching server (non-blocking
                        rounds): p50/p99 latency, queue wait and node updates/s
                        per rate; sampled served results checked bit for bit
                        against solo solves and FP32 ones against FP64
  autotune              the planner settings the autotuner kept for each batch
  next_rows             the extensions beyond the periodic batch, each timed on the
                        device: the bounded Table VIII example as a 256-tau sweep
                        in one batch (resident, boundary layers reset in LDS) and
                        on the per-step streaming path; real-power equilibria;
                        the D1Q4 / D1Q6 lattices
  cpu_baseline          the CPU oracle on a sample of the same instances

    python bench.py [--gpus 1] [--steps K] [--warmup W]

The process runs with GPU_MAX_HW_QUEUES = 16 (--hw-queues; HIP's default is 4): the
library spreads a pass's launches over one stream per hardware queue.
"""
import argparse
import dataclasses
import hashlib
import json
import multiprocessing as mp
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_0907_1720_amd import workloads as W  # noqa: E402

COUNT = 4096
LB_STEPS = 5000
PEAK_VALU_TFLOPS = 78.6      # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 flop/FMA (FP64 = non-packed FP32)
PEAK_VALU_TOPS = 39.3        # the same issue rate counted in operations (FMA = 1): 3.93e13 lane ops/s
GOLDEN = os.path.join(ROOT, "tests", "golden", "long_horizon.npz")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_counters_kdv_mkdv_batch4096.md")
KERNEL_SOURCES = ("kernels_body.hpp", "kernels_q.hip", "kernels.hip", "device.hpp", "kernels.hpp", "runtime.cpp")


def kernel_source_digest() -> str:
    """sha256 over the sources that decide what the resident kernels read and write."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0907_1720_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per FP32 pass from the committed FETCH_SIZE / WRITE_SIZE record,
    or None when the kernel sources changed since the counters were taken."""
    try:
        text = open(TRAFFIC_RECORD).read()
    except OSError:
        return None
    dig = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    val = re.search(r"hbm_bytes_per_pass:\s*([0-9.eE+]+)", text)
    if not dig or not val or dig.group(1) != kernel_source_digest():
        return None
    return float(val.group(1))


def algorithmic_flops_per_nu(G: np.ndarray) -> int:
    """Arithmetic of one node update for the equilibrium polynomials G (q x (D+1)):
    phi = sum_j f_j (q - 1 adds); per population the polynomial by Horner over
    its nonzero structure and the BGK update with omega folded in (1 FMA).
    Dense: D FMAs.  Odd in phi (every nonzero degree odd, e.g. mKdV): one shared
    phi^2, (D-1)/2 FMAs in phi^2 and one multiply by phi.  An FMA is 2 flops."""
    q, D = G.shape[0], G.shape[1] - 1
    odd = not np.any(G[:, 0::2])
    if odd:
        K = (D + 1) // 2
        return (q - 1) + 1 + q * (2 * (K - 1) + 1 + 2)
    return (q - 1) + q * (2 * D + 2)


def algorithmic_ops_per_nu(G: np.ndarray) -> int:
    """Operations of one node update (FMA = 1, as the VALU issues it), the
    count the roofline is taken in: phi = sum_j f_j (q - 1 adds); per population
    the equilibrium polynomial by Horner over its nonzero structure and the
    BGK update f + omega (f_eq - f) (2 operations).  Dense: D FMAs; odd in phi
    (e.g. mKdV): one shared phi^2, (D-1)/2 FMAs in phi^2 and one multiply by
    phi.  D1Q5 KdV (D = 5): 39; mKdV (D = 9, odd): 40."""
    q, D = G.shape[0], G.shape[1] - 1
    if not np.any(G[:, 0::2]):
        K = (D + 1) // 2
        return (q - 1) + 1 + q * ((K - 1) + 1 + 2)
    return (q - 1) + q * (D + 2)


def error_stats(got, want) -> dict:
    """Relative L2 and max-abs (relative to max |want|) over pairs of arrays."""
    r2 = np.array([np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(got, want)])
    rm = np.array([np.max(np.abs(a - b)) / np.max(np.abs(b)) for a, b in zip(got, want)])
    return {"instances": int(len(r2)), "max_rel2": float(r2.max()), "median_rel2": float(np.median(r2)),
            "max_maxabs": float(rm.max()), "median_maxabs": float(np.median(rm))}


def algorithmic_flops_power_sum(nu: np.ndarray, G: np.ndarray) -> int:
    """Arithmetic of one node update for an equilibrium with real powers,
    f_eq_j = sum_c phi^nu_c sum_d G[c, j, d] phi^d (G: F x q x (D+1)), counted
    for the cheapest evaluation of each class: its nonzero degrees lie on
    d0 + s i (i < K), so phi^(nu_c + d0) times a Horner of K terms in phi^s.
    Per node: the phi sum (q - 1 adds) and, per class, the products forming
    phi^s and phi^d0 (s - 1 and d0 - 1 multiplies, one more to apply phi^nu_c);
    per population and class K - 1 FMAs and one FMA (or multiply) applying the
    class factor; per population the BGK FMA.  The powers phi^nu (square roots,
    or exp2/log2) are not counted."""
    F, q = G.shape[0], G.shape[1]
    flops = q - 1
    for c in range(F):
        degs = [d for d in range(G.shape[2]) if np.any(G[c, :, d])]
        if not degs:
            continue
        d0 = degs[0]
        s = int(np.gcd.reduce([d - d0 for d in degs[1:]])) if len(degs) > 1 else 1
        K = (degs[-1] - d0) // s + 1
        flops += max(s - 1, 0) + max(d0 - 1, 0) + (1 if c > 0 else 0)
        flops += q * (2 * (K - 1) + 2)
    return flops + 2 * q


def serving_knee(sweep, frac: float = 0.8):
    """The first arrival rate of a serving sweep at which the work finished
    while the arrivals lasted falls below `frac` of the work arriving.  The
    drain after the last arrival (a few tenths of a second for the largest
    requests) is not counted: it would put every rate near 80% of a 1.5 s
    window.  What the largest requests still have to do when the arrivals end
    is up to ~15% of the window's work below saturation, hence 80%."""
    return next((r["rate_per_s"] for r in sweep
                 if (r["window_node_updates_per_s"] or 0) < frac * (r["offered_node_updates_per_s"] or 0)), None)


def _oracle_one(args):
    i, steps = args
    from oracle import lbm_oracle as O
    inst = W.config2_instance(i)
    t0 = time.perf_counter()
    phi = O.run(inst.problem, inst.phi0, steps)
    return inst.problem.n * steps, time.perf_counter() - t0, phi


def cpu_baseline(sample: int = 32, steps: int = LB_STEPS):
    """The oracle timed on the host cores over a sample of the batch; its
    results also give the GPU paths' error against the oracle."""
    workers = min(16, os.cpu_count() or 1, sample)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_one, [(i, steps) for i in range(sample)])
    wall = time.perf_counter() - t0
    nu = sum(r[0] for r in res)
    out = {"value": nu / wall, "unit": "node-updates/s", "cores": workers, "kind": "oracle",
           "sample": f"instances 0..{sample - 1} of the 4096-instance batch, {steps} steps each, "
                     f"numpy FP64 oracle, one process per core ({workers} processes), wall clock",
           "host": host_cpu()}
    return out, [r[2] for r in res]


def host_cpu() -> dict:
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return {"model": model, "logical_cpus": os.cpu_count(), "affinity_cpus": allowed}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--count", type=int, default=COUNT)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--serve-rates", type=str, default="32,64,128,256,512,1024",
                    help="Poisson arrival rates (requests/s) of the serving sweep")
    ap.add_argument("--serve-window", type=float, default=1.5,
                    help="seconds of arrivals per rate (at least 64 requests)")
    ap.add_argument("--serve-block", type=int, default=1000)
    ap.add_argument("--serve-budget-gb", type=int, default=16)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB device to device first (reference kernel for HBM counters)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's automatic settings instead of autotuning the batch first")
    ap.add_argument("--stream-only", action="store_true",
                    help="time only the HBM-streaming path on one large grid (for profiler runs)")
    ap.add_argument("--large-only", action="store_true",
                    help="time only the large-grid workloads (for profiler runs); prints a reduced line")
    ap.add_argument("--next-only", action="store_true",
                    help="time only the extension workloads (bounded sweep, real powers, D1Q4/D1Q6)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving measurement (Poisson request streams)")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the FP32 batch (for profiler runs); prints a reduced line")
    ap.add_argument("--fp64-batch-only", action="store_true",
                    help="time only the FP64 batch (for profiler runs); prints a reduced line")
    ap.add_argument("--powers-only", action="store_true",
                    help="time only the real-power batches, FP64 then FP32 (for profiler runs)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="GPU_MAX_HW_QUEUES for this process (hardware queues the launch lanes map to; 1..16)")
    ap.add_argument("--config4-only", action="store_true",
                    help="time only the Kawahara + K(2,2) batch (for profiler runs)")
    args = ap.parse_args()
    # HIP runs a process's streams on GPU_MAX_HW_QUEUES hardware queues (4 by
    # default); the library spreads a pass's launches over one lane per queue,
    # at most 16, and a serving round holds up to ~16 small launches (one per
    # lattice, precision and variant, resident and slab).  HIP reads the
    # variable once, when its runtime starts: before anything touches the GPU.
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.gpus != 1:
        print("bench.py measures one GPU: the instances are independent, so several GPUs would each "
              "run a share of the batch with no communication; multi-GPU runs are not part of this "
              "build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0907_1720_amd import lbm

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def read_all(b, n):
        """phi and status of every instance."""
        out = [b.read_phi(i) for i in range(n)]
        return [o[0] for o in out], all(o[1] == lbm.OK for o in out)

    def build_batch(prec):
        insts = [W.config2_instance(i, prec=prec, steps=LB_STEPS) for i in range(args.count)]
        b = lbm.Batch([x.problem for x in insts], stream=stream.cuda_stream)
        b.load_phi([x.phi0 for x in insts])
        return insts, b

    def run(prec, tune=True, keep_phi=True):
        insts, b = build_batch(prec)
        tuning = None if (args.no_autotune or not tune) else b.autotune(LB_STEPS)
        nu_pass = sum(x.problem.n for x in insts) * LB_STEPS
        per = {}
        for x in insts:
            if x.problem.name not in per:
                G = lbm.coefficients(x.problem)
                per[x.problem.name] = (algorithmic_flops_per_nu(G), algorithmic_ops_per_nu(G))
        flops_pass = sum(x.problem.n * LB_STEPS * per[x.problem.name][0] for x in insts)
        ops_pass = sum(x.problem.n * LB_STEPS * per[x.problem.name][1] for x in insts)
        for _ in range(args.warmup):
            b.advance(LB_STEPS)
        torch.cuda.synchronize()
        kern_ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.advance(LB_STEPS)
            kern_ms.append(b.last_advance_ms())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        _, ok_timed = read_all(b, len(insts))
        phis = None
        if keep_phi:
            # one pass from phi0: the configuration's 5000 steps, for the error statements
            b.load_phi([x.phi0 for x in insts])
            b.advance(LB_STEPS)
            phis, ok1 = read_all(b, len(insts))
            ok_timed = ok_timed and ok1
        b.close()
        return {"nu_pass": nu_pass, "flops_pass": flops_pass, "ops_pass": ops_pass, "wall_s": wall,
                "kernel_ms": kern_ms, "nu_per_s": nu_pass * args.steps / wall, "status_ok": ok_timed,
                "tuning": tuning, "phis": phis}

    gold = dict(np.load(GOLDEN)) if os.path.exists(GOLDEN) else {}

    def vs_gold(got, key):
        if key not in gold:
            return None
        e = error_stats([got], [gold[key]])
        return {"rel2": e["max_rel2"], "maxabs": e["max_maxabs"]}

    def ks_batches():
        """Config 3 whole: 1024 perturbed KS runs at each N to t = 20, FP64 and FP32."""
        out = {"workload": "Kuramoto-Sivashinsky on [0, 32 pi), 1024 runs at each of N = 1024, 4096, 8192, "
                           "cos(x/16)(1 + sin(x/16)) + N(0, 1e-3^2), to t = 20 (tau, dt = (2, 2.9e-4), "
                           "(10, 3.1e-4), (20, 1.7e-4))"}
        tot_nu, tot_ms = {0: 0.0, 1: 0.0}, {0: 0.0, 1: 0.0}
        for n in (1024, 4096, 8192):
            res = {}
            for prec, tag in ((W.F64, "fp64"), (W.F32_DEV, "fp32")):
                insts = [W.config3_instance(n, i, prec=prec) for i in range(1024)]
                steps = insts[0].steps
                b = lbm.Batch([x.problem for x in insts], stream=stream.cuda_stream)
                b.load_phi([x.phi0 for x in insts])
                # planner settings timed on a copy of the batch (1000-step probes)
                tuning = None if args.no_autotune else b.autotune(1000)
                torch.cuda.synchronize()
                b.advance(steps)
                ms = b.last_advance_ms()
                phis, ok = read_all(b, len(insts))
                b.close()
                nu = n * 1024 * steps
                tot_nu[prec] += nu
                tot_ms[prec] += ms
                res[tag] = {"steps": steps, "kernel_ms": ms, "node_updates_per_s": nu / (ms * 1e-3), "status_ok": ok,
                            "autotune": tuning,
                            "vs_oracle_inst0_t20": vs_gold(phis[0], f"ks_n{n}_i0_t20"),
                            "vs_oracle_inst1023_t20": vs_gold(phis[1023], f"ks_n{n}_i1023_t20")}
                res[tag + "_phis"] = phis
            res["fp32_vs_fp64_all_runs_t20"] = error_stats(res.pop("fp32_phis"), res.pop("fp64_phis"))
            out[f"n{n}"] = res
        out["fp64_node_updates_per_s"] = tot_nu[0] / (tot_ms[0] * 1e-3)
        out["fp32_node_updates_per_s"] = tot_nu[1] / (tot_ms[1] * 1e-3)
        out["node_updates_per_precision"] = tot_nu[0]
        return out

    def kawahara_k22_batch():
        """Config 4 whole: 512 Kawahara / K(2,2) instances, N in {2048, 16384}, 5000 steps."""
        out = {"workload": "128 x {Kawahara (D1Q7), K(2,2) (D1Q5)} x N {2048, 16384} on [-60, 60), 5000 steps"}
        phis = {}
        insts = {}
        for prec, tag in ((W.F64, "fp64"), (W.F32_DEV, "fp32")):
            xs = [W.config4_instance(i, prec=prec) for i in range(512)]
            insts[tag] = xs
            b = lbm.Batch([x.problem for x in xs], stream=stream.cuda_stream)
            b.load_phi([x.phi0 for x in xs])
            tuning = None if args.no_autotune else b.autotune(1000)
            b.advance(16)                  # warm-up (planner tables, code objects)
            b.load_phi([x.phi0 for x in xs])
            torch.cuda.synchronize()
            b.advance(5000)
            ms = b.last_advance_ms()
            phis[tag], ok = read_all(b, len(xs))
            b.close()
            nu = sum(x.problem.n for x in xs) * 5000
            ops = 0
            for name in ("kawahara", "k22"):
                x = next(x for x in xs if x.problem.name == name)
                ops += sum(y.problem.n for y in xs if y.problem.name == name) * 5000 * \
                    algorithmic_ops_per_nu(lbm.coefficients(x.problem))
            out[tag] = {"kernel_ms": ms, "node_updates_per_s": nu / (ms * 1e-3), "status_ok": ok,
                        "alu_ops_frac": ops / (ms * 1e-3) / 1e12 / PEAK_VALU_TOPS, "autotune": tuning,
                        "vs_oracle": [vs_gold(phis[tag][i], f"c4_i{i}") for i in range(4)],
                        "vs_closed_form_rel2": [float(np.linalg.norm(phis[tag][i] - xs[i].exact(5000 * xs[i].problem.dt))
                                                      / np.linalg.norm(xs[i].exact(5000 * xs[i].problem.dt)))
                                                for i in range(4)]}
        out["node_updates"] = nu
        out["fp32_vs_fp64_all_instances"] = error_stats(phis["fp32"], phis["fp64"])
        return out

    def large_grids():
        return {"ks_batches": ks_batches(), "kawahara_k22_batch": kawahara_k22_batch()}

    def hbm_stream():
        """The plain fused collide+stream path on one grid far larger than the caches
        (2^25 nodes: 1.34 GB per FP64 buffer), against HBM peak and a device copy."""
        out = {}
        n, steps = 1 << 25, 128
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        out["copy_gb_per_s"] = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
        x = -20.0 + 40.0 / n * np.arange(n)
        for prec, tag, es in ((W.F64, "fp64", 8), (W.F32_DEV, "fp32", 4)):
            p = W.kdv(1.0, n, 40.0 / n, 0.05 * (40.0 / n) ** 3, 2.0, -20.0, prec=prec)
            s = lbm.Solver(p, stream=stream.cuda_stream)
            s.set_path(lbm.PATH_STREAM)
            s.load_phi(W.kdv_soliton(x, 0.0, 1.0, 1.0, -5.0, period=40.0))
            s.advance(steps)
            torch.cuda.synchronize()
            s.advance(steps)
            ms = s.last_advance_ms()
            nbytes = 2 * p.lattice() * es * n * steps
            out[tag] = {"node_updates_per_s": n * steps / (ms * 1e-3), "algorithmic_gb_per_s": nbytes / (ms * 1e-3) / 1e9,
                        "frac_of_8tb": nbytes / (ms * 1e-3) / 8e12, "kernel_ms": ms, "nodes": n, "steps": steps}
            out[tag + "_phi"] = s.read_phi()
            s.close()
        out["fp32_vs_fp64"] = error_stats([out.pop("fp32_phi")], [out.pop("fp64_phi")])
        return out

    def timed_batch(insts, steps, label, keep_phi=False):
        """Device rate of one pass (after a warm-up pass) of a periodic batch."""
        b = lbm.Batch([x.problem for x in insts], stream=stream.cuda_stream)
        b.load_phi([x.phi0 for x in insts])
        b.advance(steps)
        b.load_phi([x.phi0 for x in insts])
        torch.cuda.synchronize()
        b.advance(steps)
        ms = b.last_advance_ms()
        phis, ok = read_all(b, len(insts))
        b.close()
        nu = sum(x.problem.n for x in insts) * steps
        out = {"workload": label, "instances": len(insts), "steps": steps, "node_updates": nu,
               "kernel_ms": ms, "node_updates_per_s": nu / (ms * 1e-3), "status_ok": ok}
        fl = 0
        for x in insts:
            nu, G = lbm.coefficients_general(x.problem)
            f = algorithmic_flops_per_nu(G[0]) if len(nu) == 1 else algorithmic_flops_power_sum(nu, G)
            fl += x.problem.n * steps * f
        out["alu_frac"] = fl / (ms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS
        return (out, phis) if keep_phi else out

    def next_rows():
        out = {}
        # bounded (Sec. IV boundaries) x tau sweep: Table VIII to t = 150 at 256 taus
        p0, x, ex = W.table8_bounded()
        steps, layers = 15000, 2
        xb = np.concatenate([x[:layers], x[-layers:]])
        phib = np.stack([ex(xb, s * p0.dt) for s in range(1, steps + 1)])
        taus = np.linspace(0.97, 2.5, 256)
        probs = [dataclasses.replace(p0, tau=float(t)) for t in taus]
        b = lbm.Batch(probs, stream=stream.cuda_stream)
        b.load_phi([ex(x, 0.0)] * len(probs))
        b.advance_bounded([phib[:200]] * len(probs))            # warm-up
        b.load_phi([ex(x, 0.0)] * len(probs))
        b.advance_bounded([phib] * len(probs))
        ms = b.last_advance_ms()
        res = [b.read_phi(i) for i in range(len(probs))]
        b.close()
        err = [float(np.sum(np.abs(r[0] - ex(x, steps * p0.dt))) / np.sum(np.abs(ex(x, steps * p0.dt))))
               if r[1] == lbm.OK else float("inf") for r in res]
        nu = len(probs) * p0.n * steps
        fl = nu * algorithmic_flops_per_nu(lbm.coefficients(p0))
        out["bounded_tau_sweep"] = {
            "workload": "Table VIII KdV-Burgers on [-4, 4] (801 nodes, D1Q5, NEE boundaries), 256 taus in "
                        "[0.97, 2.5], 15000 steps (t = 150) in one batch",
            "node_updates": nu, "kernel_ms": ms, "node_updates_per_s": nu / (ms * 1e-3),
            "alu_frac": fl / (ms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS,
            "tau_opt": float(taus[int(np.argmin(err))]), "E_at_tau_opt": float(min(err)),
            "status_ok": all(r[1] == lbm.OK for r in res)}
        # the same sweep with the boundary values evaluated on the device from the
        # front's closed form (no host rows): wall clock of the call, rows included
        wv = W.table8_wave()
        wave = lbm.make_wave(wv["shape"], wv["a"], wv["b"], wv["p"], wv["k"], wv["xc"], wv["c"], float(x[0]))
        b = lbm.Batch(probs, stream=stream.cuda_stream)
        b.load_phi([ex(x, 0.0)] * len(probs))
        b.advance_bounded_wave([wave] * len(probs), 200)        # warm-up
        b.load_phi([ex(x, 0.0)] * len(probs))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.advance_bounded_wave([wave] * len(probs), steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        msw = b.last_advance_ms()
        resw = [b.read_phi(i) for i in range(len(probs))]
        b.close()
        errw = [float(np.sum(np.abs(r[0] - ex(x, steps * p0.dt))) / np.sum(np.abs(ex(x, steps * p0.dt))))
                if r[1] == lbm.OK else float("inf") for r in resw]
        out["bounded_tau_sweep_device_rows"] = {
            "workload": "the same sweep, boundary rows evaluated on the device from the front's closed form",
            "kernel_ms": msw, "wall_ms": wall * 1e3, "node_updates_per_s": nu / wall,
            "E_at_tau_opt": float(errw[int(np.argmin(err))]), "status_ok": all(r[1] == lbm.OK for r in resw)}
        # the same problem on the per-step streaming path (one collide+stream and
        # one boundary launch per step)
        s = lbm.Solver(p0, stream=stream.cuda_stream)
        s.set_path(lbm.PATH_STREAM)
        s.load_phi(ex(x, 0.0))
        s.advance_bounded(phib[:200])
        torch.cuda.synchronize()
        s.advance_bounded(phib[200:2200])
        ms1 = s.last_advance_ms()
        s.close()
        out["bounded_streaming_single"] = {"workload": "the same problem at tau = 0.97, 2000 steps, one instance",
                                           "kernel_ms": ms1, "node_updates_per_s": p0.n * 2000 / (ms1 * 1e-3)}
        out["real_powers"], out["real_powers_fp32"] = real_powers()
        out["d1q4"] = timed_batch([W.even_lattice_instance(i, 4) for i in range(1024)], 2000,
                                  "1024 D1Q4 KdV-Burgers, N log-uniform [256, 4096], FP64")
        out["d1q6"] = timed_batch([W.even_lattice_instance(i, 6) for i in range(1024)], 2000,
                                  "1024 D1Q6 fifth-order dissipative equations, N log-uniform [256, 4096], FP64")
        return out

    def real_powers():
        rp, ph64 = timed_batch([W.power_batch_instance(i) for i in range(1024)], 2000,
                               "1024 periodic phi_t + phi^n phi_x + delta phi_xxx = 0, n in {0.5, 1.5}, "
                               "N log-uniform [256, 4096], FP64, D1Q5", keep_phi=True)
        rp32, ph32 = timed_batch([W.power_batch_instance(i, prec=W.F32_DEV) for i in range(1024)],
                                 2000, "the same, FP32 deviation storage", keep_phi=True)
        rp32["fp32_vs_fp64_all_instances"] = error_stats(ph32, ph64)
        return rp, rp32

    def solo(p, phi0, steps):
        s = lbm.Solver(p, stream=stream.cuda_stream)
        s.load_phi(phi0)
        s.advance(steps)
        out = s.read_phi(allow_nonfinite=True)
        s.close()
        return out

    def serve():
        """Sweep of Poisson arrival rates of the mixed request stream (7 equation
        families, N log-uniform [128, 16384], steps log-uniform [1e3, 1e5],
        FP32/FP64) through the server's non-blocking rounds."""
        from paper_0907_1720_amd import serving
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        counts = [max(64, int(round(r * args.serve_window))) for r in rates]
        reqs = [W.serving_request(i) for i in range(max(counts))]
        sweep = []
        check = None
        for rate, cnt in zip(rates, counts):
            srv = lbm.Server(args.serve_budget_gb << 30, max_slots=1024, max_n=16384, block_steps=args.serve_block,
                             stream=stream.cuda_stream)
            keep = check is None and rate >= 256
            r = serving.run_poisson(srv, reqs[:cnt], rate=rate, seed=1, keep_results=keep)
            srv.close()
            if keep:
                check = (cnt, r.pop("results"))
                for k in ("latency", "queue_wait", "statuses"):
                    r.pop(k)
            sweep.append({k: r[k] for k in ("rate_per_s", "requests", "arrival_span_s", "offered_node_updates_per_s",
                                            "node_updates_per_s", "window_node_updates_per_s", "wall_s",
                                            "p50_latency_s", "p99_latency_s",
                                            "mean_queue_wait_s", "p99_queue_wait_s", "p50_service_s", "nonfinite")})
        knee = serving_knee(sweep)
        out = {"workload": "Poisson arrivals of the 7-family request mix (N log-uniform [128, 16384], steps "
                           "log-uniform [1e3, 1e5], FP32 / FP64), " f"{args.serve_window} s of arrivals per rate "
                           "(at least 64 requests), non-blocking rounds (lbm_server_pump)",
               "block_steps": args.serve_block, "budget_bytes": args.serve_budget_gb << 30,
               "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]), "sweep": sweep,
               "knee_rate_per_s": knee}
        if check:
            cnt, results = check
            # served results against solo solves (bit for bit), and the FP32
            # ones against the FP64 solve of the same request
            idx = list(range(min(8, cnt)))
            big = max(range(cnt), key=lambda i: reqs[i].problem.n * reqs[i].steps)
            if big not in idx:
                idx.append(big)
            same = all(np.array_equal(results[i], solo(reqs[i].problem, reqs[i].phi0, reqs[i].steps)) for i in idx)
            f32 = [i for i in range(min(cnt, 48)) if reqs[i].problem.prec != W.F64 and reqs[i].problem.name != "ks"][:6]
            errs = error_stats([results[i] for i in f32],
                               [solo(dataclasses.replace(reqs[i].problem, prec=W.F64), reqs[i].phi0, reqs[i].steps)
                                for i in f32]) if f32 else None
            out["check"] = {"rate_per_s": next(s_["rate_per_s"] for s_ in sweep if s_["requests"] == cnt),
                            "bitwise_vs_solo": bool(same), "requests_checked": [int(i) for i in idx],
                            "largest_checked": {"n": reqs[big].problem.n, "steps": reqs[big].steps},
                            "fp32_vs_fp64_solo": errs}
        return out

    if args.serving_only:
        print(json.dumps({"metric": "serving latency only", "serving": serve()}))
        return
    if args.next_only:
        print(json.dumps({"metric": "extensions (next rows) only", "next_rows": next_rows()}))
        return
    if args.stream_only:
        print(json.dumps({"metric": "HBM streaming path", "hbm_stream": hbm_stream()}))
        return
    if args.large_only:
        print(json.dumps({"metric": "lattice-node updates/s (large grids only)", "large_grids": large_grids()}))
        return
    if args.config4_only:
        print(json.dumps({"metric": "Kawahara + K(2,2) batch only", "kawahara_k22_batch": kawahara_k22_batch()}))
        return
    if args.powers_only:
        rp, rp32 = real_powers()
        print(json.dumps({"metric": "real-power batches only", "real_powers": rp, "real_powers_fp32": rp32}))
        return
    if args.fp64_batch_only:
        r64 = run(W.F64, keep_phi=False)
        print(json.dumps({"metric": "lattice-node updates/s (FP64 batch only)", "value": r64["nu_per_s"],
                          "unit": "node-updates/s", "steps": args.steps, "warmup": args.warmup,
                          "kernel_ms": r64["kernel_ms"], "status_ok": r64["status_ok"]}))
        return
    r32 = run(W.F32_DEV, keep_phi=not args.batch_only)
    if args.batch_only:
        print(json.dumps({"metric": "lattice-node updates/s (FP32 batch only)", "value": r32["nu_per_s"],
                          "unit": "node-updates/s", "steps": args.steps, "warmup": args.warmup,
                          "kernel_ms": r32["kernel_ms"], "status_ok": r32["status_ok"]}))
        return
    r64 = run(W.F64)
    r32a = run(W.F32_DEV_ARITH32)
    lg = large_grids()
    hs = hbm_stream()
    nx = next_rows()

    # plain FP64 path: one instance at a time, one launch per step
    sample = np.linspace(0, args.count - 1, args.plain_sample).astype(int)
    nu, secs = 0, 0.0
    for i in sample:
        inst = W.config2_instance(int(i))
        s = lbm.Solver(inst.problem, stream=stream.cuda_stream)
        s.set_path(lbm.PATH_STREAM)
        s.load_phi(inst.phi0)
        s.advance(50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(LB_STEPS)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        nu += inst.problem.n * LB_STEPS
        s.close()
    plain = nu / secs

    srv_out = serve()

    k_ms = float(np.mean(r32["kernel_ms"]))
    # the HBM record was taken with the planner's automatic settings
    t = r32["tuning"]
    default_plan = t is None or all(t[k] == 0 for k in ("path", "tile_steps", "tile_wgs", "res_chunks"))
    traffic = measured_traffic() if default_plan else None
    achieved_ops = r32["ops_pass"] / (k_ms * 1e-3) / 1e12
    achieved = r32["flops_pass"] / (k_ms * 1e-3) / 1e12
    kernel = "k_resident<5, D, P, float, double>: KdV (D 5) and mKdV (D 9, odd) launches of one pass"
    roofline = {"bound": "alu", "achieved": achieved_ops, "peak": PEAK_VALU_TOPS, "unit": "Tops/s",
                "frac": achieved_ops / PEAK_VALU_TOPS, "traffic": traffic, "traffic_unit": "HBM bytes per pass",
                "accounting": "VALU lane operations of one node update (FMA = 1): 39 per KdV, 40 per mKdV node "
                              "update; peak 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz",
                "kernel": kernel, "kernel_ms": k_ms, "ops_per_pass": r32["ops_pass"]}
    roofline_flops = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                      "frac": achieved / PEAK_VALU_TFLOPS, "kernel": kernel, "kernel_ms": k_ms,
                      "flops_per_pass": r32["flops_pass"]}
    fp32_err = {"vs_fp64_batch_all_instances": error_stats(r32["phis"], r64["phis"]),
                "fp32_relaxation_vs_fp64_batch": error_stats(r32a["phis"], r64["phis"]),
                "after_steps": LB_STEPS}
    out = {
        "metric": "lattice-node updates/s, batched FP32 vs plain FP64 on 1 GPU; p50/p99 latency",
        "value": r32["nu_per_s"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["wall_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "f32 deviation from rest equilibrium",
        "data": "synthetic",
        "config": {"workload": f"{args.count} periodic KdV/mKdV solitons, N log-uniform [256, 4096], "
                               f"{LB_STEPS} steps each, D1Q5, tau = 2, dt = 0.05 dx^3/delta",
                   "instances": args.count, "lattice_steps_per_step": LB_STEPS,
                   "node_updates_per_step": r32["nu_pass"]},
        "fp32_error": fp32_err,
        "fp64_batched": {"value": r64["nu_per_s"], "ms_per_step": r64["wall_s"] / args.steps * 1e3,
                         "kernel_ms": float(np.mean(r64["kernel_ms"])), "autotune": r64["tuning"]},
        "fp32_arith_batched": {"value": r32a["nu_per_s"], "ms_per_step": r32a["wall_s"] / args.steps * 1e3,
                               "kernel_ms": float(np.mean(r32a["kernel_ms"])),
                               "precision": "FP32 deviation storage and FP32 relaxation (LBM_F32_DEV_ARITH32)"},
        "autotune": r32["tuning"],
        "plain_fp64": {"value": plain, "sample_instances": int(len(sample)),
                       "path": "one fused collide+stream launch per step (64-step blocks replayed from a HIP graph), "
                               "one instance at a time"},
        "speedup_vs_plain_fp64": r32["nu_per_s"] / plain,
        "hbm_stream": {"workload": "one periodic KdV grid of 2^25 nodes, 128 steps on the plain fused "
                                   "collide+stream path; algorithmic bytes 2 q s per node update", **hs},
        "large_grids": lg,
        "next_rows": nx,
        "status_ok": bool(r32["status_ok"] and r64["status_ok"] and r32a["status_ok"]),
        "roofline": roofline,
        "roofline_flops": roofline_flops,
        "serving": srv_out,
    }
    if not args.no_cpu:
        cb, oracle_phis = cpu_baseline()
        out["cpu_baseline"] = cb
        k = len(oracle_phis)
        fp32_err["vs_oracle_sample"] = error_stats(r32["phis"][:k], oracle_phis)
        fp32_err["fp64_vs_oracle_sample"] = error_stats(r64["phis"][:k], oracle_phis)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
