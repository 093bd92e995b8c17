"""Throughput of the batched LBGK hot path on one MI355X.

Workload: 4096 independent KdV / mKdV solitons (N log-uniform in [256, 4096],
periodic, 5000 time steps each, seeded).  One bench "step" advances the whole
batch by its 5000 lattice steps (one pass of the hot path over the batch).

Reported:
  value                 lattice-node updates per second of the batched FP32
                        deviation path (all instances, wall clock of the timed
                        passes, inputs resident in HBM)
  fp64_batched          the same batch stored and computed in FP64
  plain_fp64            one instance at a time, one fused collide+stream launch
                        per step, FP64 (sampled instances)
  roofline              the dominant kernel (the persistent LDS-resident batch
                        kernel) against the VALU peak, timed with HIP events on
                        the launch stream
  hbm_stream            the fused collide+stream path on a 2^25-node grid:
                        algorithmic HBM GB/s against 8 TB/s and a device copy
  large_grids           device rate of the workloads whose grids exceed one
                        workgroup's LDS (slabs over co-resident workgroups):
                        Kuramoto-Sivashinsky N = 8192 and Kawahara / K(2,2)
  serving               p50/p99 latency and throughput of a Poisson stream of
                        mixed solve requests through the continuous-batching server
  autotune              the planner settings the autotuner kept for each batch
  next_rows             the extensions beyond the periodic batch, each timed on the
                        device: the bounded Table VIII example as a 64-tau sweep
                        in one batch (resident, boundary layers reset in LDS) and
                        on the per-step streaming path; real-power equilibria;
                        the D1Q4 / D1Q6 lattices
  cpu_baseline          the CPU oracle on a sample of the same instances

    python bench.py [--gpus 1] [--steps K] [--warmup W]
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


def _oracle_one(args):
    i, steps = args
    from oracle import lbm_oracle as O
    inst = W.config2_instance(i)
    t0 = time.perf_counter()
    O.run(inst.problem, inst.phi0, steps)
    return inst.problem.n * steps, time.perf_counter() - t0


def cpu_baseline(sample: int = 32, steps: int = LB_STEPS):
    workers = min(16, os.cpu_count() or 1, sample)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_one, [(i, steps) for i in range(sample)])
    wall = time.perf_counter() - t0
    nu = sum(r[0] for r in res)
    return {"value": nu / wall, "unit": "node-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"instances 0..{sample - 1} of the 4096-instance batch, {steps} steps each, "
                      f"numpy FP64 oracle, one process per core ({workers} processes), wall clock",
            "host": host_cpu()}


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
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=256.0)
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
                    help="run only the serving measurement (Poisson request stream)")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the FP32 batch (for profiler runs); prints a reduced line")
    args = ap.parse_args()
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

    def build_batch(prec):
        insts = [W.config2_instance(i, prec=prec, steps=LB_STEPS) for i in range(args.count)]
        b = lbm.Batch([x.problem for x in insts], stream=stream.cuda_stream)
        b.load_phi([x.phi0 for x in insts])
        return insts, b

    def run(prec):
        insts, b = build_batch(prec)
        tuning = None if args.no_autotune else b.autotune(LB_STEPS)
        nu_pass = sum(x.problem.n for x in insts) * LB_STEPS
        fpn = {}
        for x in insts:
            if x.problem.name not in fpn:
                fpn[x.problem.name] = algorithmic_flops_per_nu(lbm.coefficients(x.problem))
        flops_pass = sum(x.problem.n * LB_STEPS * fpn[x.problem.name] for x in insts)
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
        st = [b.read_phi(i)[1] for i in (0, args.count - 1)]
        b.close()
        return {"nu_pass": nu_pass, "flops_pass": flops_pass, "wall_s": wall, "kernel_ms": kern_ms,
                "nu_per_s": nu_pass * args.steps / wall, "status_ok": all(s == lbm.OK for s in st),
                "tuning": tuning}

    def large(insts, steps):
        """Device rate of one pass over instances too large for one workgroup's LDS."""
        b = lbm.Batch([x.problem for x in insts], stream=stream.cuda_stream)
        b.load_phi([x.phi0 for x in insts])
        b.advance(16)
        torch.cuda.synchronize()
        b.advance(steps)
        ms = b.last_advance_ms()
        st = all(b.read_phi(i)[1] == lbm.OK for i in (0, len(insts) - 1))
        b.close()
        return {"node_updates_per_s": sum(x.problem.n for x in insts) * steps / (ms * 1e-3), "kernel_ms": ms,
                "instances": len(insts), "steps": steps, "status_ok": st}

    def large_grids():
        out = {}
        for prec, tag in ((W.F64, "fp64"), (W.F32_DEV, "fp32")):
            out[f"ks_n8192_{tag}"] = large([W.config3_instance(8192, i, prec=prec) for i in range(256)], 640)
            out[f"kawahara_k22_{tag}"] = large([W.config4_instance(i, prec=prec) for i in range(512)], 500)
        return out

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
            s.close()
        return out

    def timed_batch(insts, steps, label):
        """Device rate of one pass (after a warm-up pass) of a periodic batch."""
        b = lbm.Batch([x.problem for x in insts], stream=stream.cuda_stream)
        b.load_phi([x.phi0 for x in insts])
        b.advance(steps)
        torch.cuda.synchronize()
        b.advance(steps)
        ms = b.last_advance_ms()
        ok = all(b.read_phi(i)[1] == lbm.OK for i in range(len(insts)))
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
        return out

    def next_rows():
        out = {}
        # bounded (Sec. IV boundaries) x tau sweep: Table VIII to t = 150 at 64 taus
        p0, x, ex = W.table8_bounded()
        steps, layers = 15000, 2
        xb = np.concatenate([x[:layers], x[-layers:]])
        phib = np.stack([ex(xb, s * p0.dt) for s in range(1, steps + 1)])
        taus = np.linspace(0.97, 2.5, 64)
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
            "workload": "Table VIII KdV-Burgers on [-4, 4] (801 nodes, D1Q5, NEE boundaries), 64 taus in "
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
        out["real_powers"] = timed_batch([W.power_batch_instance(i) for i in range(1024)], 2000,
                                         "1024 periodic phi_t + phi^n phi_x + delta phi_xxx = 0, n in {0.5, 1.5}, "
                                         "N log-uniform [256, 4096], FP64, D1Q5")
        out["real_powers_fp32"] = timed_batch([W.power_batch_instance(i, prec=W.F32_DEV) for i in range(1024)],
                                              2000, "the same, FP32 deviation storage")
        out["d1q4"] = timed_batch([W.even_lattice_instance(i, 4) for i in range(1024)], 2000,
                                  "1024 D1Q4 KdV-Burgers, N log-uniform [256, 4096], FP64")
        out["d1q6"] = timed_batch([W.even_lattice_instance(i, 6) for i in range(1024)], 2000,
                                  "1024 D1Q6 fifth-order dissipative equations, N log-uniform [256, 4096], FP64")
        return out

    def serve():
        # Poisson arrivals of the mixed request stream (7 equation families,
        # N log-uniform [128, 16384], steps log-uniform [1e3, 1e5], FP32/FP64)
        from paper_0907_1720_amd import serving
        reqs = [W.serving_request(i) for i in range(args.serve_requests)]
        srv = lbm.Server(args.serve_budget_gb << 30, max_slots=1024, max_n=16384, block_steps=args.serve_block,
                         stream=stream.cuda_stream)
        r = serving.run_poisson(srv, reqs, rate=args.serve_rate, seed=1)
        srv.close()
        return {"requests": r["requests"], "arrival_rate_per_s": r["rate_per_s"],
                "p50_latency_s": r["p50_latency_s"], "p99_latency_s": r["p99_latency_s"],
                "node_updates_per_s": r["node_updates_per_s"], "wall_s": r["wall_s"],
                "nonfinite": r["nonfinite"], "block_steps": args.serve_block,
                "budget_bytes": args.serve_budget_gb << 30}

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
    r32 = run(W.F32_DEV)
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
    achieved = r32["flops_pass"] / (k_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_VALU_TFLOPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per pass",
                "kernel": "k_resident<5, D, P, float, double>: KdV (D 5) and mKdV (D 9, odd) launches of one pass",
                "kernel_ms": k_ms, "flops_per_pass": r32["flops_pass"]}
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
        "large_grids": {"workload": "Kuramoto-Sivashinsky N = 8192 (256 instances, 640 steps) and "
                                    "Kawahara/K(2,2) N in {2048, 16384} (512 instances, 500 steps), device time",
                        **lg},
        "next_rows": nx,
        "status_ok": bool(r32["status_ok"] and r64["status_ok"] and r32a["status_ok"]),
        "roofline": roofline,
        "serving": srv_out,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
