"""Benchmark: thread-safe regularized LB sweep, D3Q19 512^3 FP32 on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512]

Workload: D3Q19, 512^3 periodic 3D Taylor-Green vortex (u0 = 0.02,
tau = 0.55, rho0 = 1), FP32 shifted population storage and FP32 arithmetic,
synthetic seeded input.  A step is the whole hot path: the moments sweep and
the fused stream-collide sweep (boundaries fused).  The state is resident in
HBM before the timed region; K steps are timed between two device
synchronisations.  Prints one JSON line.

Roofline: algorithmic bytes per lattice update = Q reads + M writes
(moments) + M reads + Q writes (stream-collide) = 116 + 116 B for D3Q19 FP32.
The dominant kernel's achieved bandwidth uses its average launch time from
HIP events recorded on the launch stream during the timed region.  The HBM
traffic counters (FETCH_SIZE / WRITE_SIZE) come from separate rocprofv3 runs
kept under profiles/; they are reported only while the kernel source they
were taken on is unchanged.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS + % HBM roofline, D3Q19 512^3 FP32; p50/p99 solve latency"
KERNEL_SOURCES = ["paper_2304_06437_amd/csrc/kernels.hpp", "paper_2304_06437_amd/csrc/lattice.hpp",
                  "paper_2304_06437_amd/csrc/storage.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_d3q19_512_traffic.md")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(Q: int, M: int, ssize: int, csize: int):
    """Bytes per lattice update of (moments, stream-collide)."""
    k1 = Q * ssize + M * csize
    k2 = M * csize + Q * ssize
    return k1, k2


def read_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary, or None when
    the summary is missing or was taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(rf"{kernel}_hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    return float(m.group(1)) if m else None


def cpu_baseline(seconds_hint: float = 15.0):
    """Time the FP64 CPU oracle on a bounded sample of the same workload."""
    import oracle
    from paper_2304_06437_amd import inputs

    n = 128
    p = oracle.Params(lattice=19, nx=n, ny=n, nz=n, tau=0.55)
    rho, u = inputs.taylor_green_3d(n, n, n, 0.02)
    f = oracle.init(p, rho, u)
    t = time.perf_counter()
    oracle.run(p, f, 1)
    one = time.perf_counter() - t
    steps = max(1, min(200, int(seconds_hint / max(one, 1e-3))))
    t = time.perf_counter()
    oracle.run(p, f, steps)
    dt = time.perf_counter() - t
    return {
        "value": n ** 3 * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"D3Q19 {n}^3 periodic Taylor-Green (u0 0.02, tau 0.55), FP64 two-array "
                  f"oracle, {steps} steps ({dt:.1f} s); same per-node work as the 512^3 workload",
    }


def serving(torch, jobs: int, rate: float, budget_gb: float):
    """Continuous batching of a seeded Poisson request stream: D2Q9/D3Q19,
    Taylor-Green or channel, FP32 or shifted-FP16 storage, edge
    log-uniform 64..256 (n^2 or n^3), 200-2000 steps, admitted by an HBM
    budget.  Time-to-solution = arrival to moments on the host."""
    from paper_2304_06437_amd.serving import GpuBackend, Server, poisson_mix

    specs = poisson_mix(jobs, rate=rate, seed=2026)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        be = GpuBackend()
        rep = Server(be, hbm_budget=int(budget_gb * 1e9), chunk_steps=200).run(specs)
        be.close()
    torch.cuda.synchronize()
    s = rep.summary()
    s.update({"rate_per_s": rate, "budget_GB": budget_gb,
              "mix": "D2Q9/D3Q19 x TG/channel x f32/f16s, edge 64..256 log-uniform, "
                     "200-2000 steps, seeded Poisson arrivals"})
    return s


def copy_ceiling(torch, nbytes: int = 4 << 30, reps: int = 10):
    """Device-to-device copy kernel bandwidth (read + write bytes / time)."""
    from paper_2304_06437_amd import lb

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream().cuda_stream
    lb.lb_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lb.lb_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="cube edge (512 is the workload)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16s", "bf16s"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=96,
                    help="requests in the serving measurement (0 to skip)")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="mean arrivals per second")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_06437_amd import inputs, lb
    from paper_2304_06437_amd.sim import Simulation, make_params

    lb.load()
    n = args.n
    N = n ** 3
    params = make_params(lattice=19, shape=(n, n, n), tau=0.55, storage=args.storage)
    rho, u = inputs.taylor_green_3d(n, n, n, 0.02)

    copy_gbs = copy_ms = None
    if not args.no_copy:
        copy_gbs, copy_ms = copy_ceiling(torch)

    sim = Simulation(params)
    sim.init(rho, u)
    del rho, u
    sim.step(args.warmup)
    sim.synchronize()

    lb.lb_timing_begin(sim.handle, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, klaunch = lb.lb_timing_end(sim.handle)
    elapsed = t1 - t0
    check = sim.moments(rho=False, u=False, pineq=False)["conserved"]
    sim.close()

    ms_per_step = elapsed * 1e3 / args.steps
    mlups = N * args.steps / elapsed / 1e6
    ssize = {"f32": 4, "f16s": 2, "bf16s": 2}[args.storage]
    b1, b2 = algorithmic_bytes(19, 10, ssize, 4)
    avg = [kms[i] / max(klaunch[i], 1) for i in range(2)]
    names = ["moments", "stream_collide"]
    dom = 0 if avg[0] > avg[1] else 1
    bytes_launch = [b1 * N, b2 * N]
    achieved = bytes_launch[dom] / (avg[dom] * 1e-3) / 1e9
    traffic = read_traffic(names[dom]) if args.storage == "f32" and n == 512 else None

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"D3Q19 {n}^3 periodic 3D Taylor-Green (u0 0.02, tau 0.55, rho0 1), "
                        f"{args.storage} population storage, f32 arithmetic",
            "lattice": "D3Q19", "nodes": N, "storage": args.storage, "compute": "f32",
            "bytes_per_update": b1 + b2,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": names[dom],
            "bytes_per_launch": bytes_launch[dom],
        },
        "kernels": {
            names[i]: {"avg_ms": round(avg[i], 4), "launches": klaunch[i],
                       "algorithmic_GBs": round(bytes_launch[i] / (avg[i] * 1e-3) / 1e9, 1)}
            for i in range(2)
        },
        "step_GBs": round((b1 + b2) * N / (ms_per_step * 1e-3) / 1e9, 1),
        "step_frac_of_peak": round((b1 + b2) * N / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_ceiling_GBs": round(copy_gbs, 1) if copy_gbs else None,
        "mass_finite": bool(np.isfinite(check[0])),
    }
    if args.serve_jobs > 0:
        out["serving"] = serving(torch, args.serve_jobs, args.serve_rate, args.serve_budget_gb)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
