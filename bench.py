"""Benchmark: thread-safe regularized LB sweep, D3Q19 512^3 FP32 on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512]

Workload: D3Q19, 512^3 periodic 3D Taylor-Green vortex (u0 = 0.02,
tau = 0.55, rho0 = 1), FP32 shifted population storage and FP32 arithmetic,
synthetic seeded input.  A step is the whole hot path: every node's moments,
post-collision populations and streaming (boundaries fused), through the
path lb_step takes by default: the fused step where the shape allows it
(one launch that keeps the moments in registers), else the moments sweep
and the stream-collide sweep.  The state is resident in HBM before the
timed region; K steps are timed between two device synchronisations.  The
same handle is then timed on the two-sweep path for comparison.  Prints one
JSON line.

Roofline: algorithmic bytes per lattice update of the fused step = Q reads
+ Q writes = 152 B for D3Q19 FP32; of the two sweeps = Q reads + M writes
(moments) + M reads + Q writes (stream-collide) = 116 + 116 B.  The dominant
kernel's achieved bandwidth uses its average launch time from HIP events
recorded on the launch stream during the timed region.  The HBM traffic
counters (FETCH_SIZE / WRITE_SIZE) come from separate rocprofv3 runs kept
under profiles/; they are reported only while the kernel source they were
taken on is unchanged.

Memory: the handle's device footprint (lb_required_bytes) per node, and
the footprint of a handle holding the population set alone (keep_moments =
0, fused step only) where the shape has a fused step.
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
                  "paper_2304_06437_amd/csrc/storage.hpp", "paper_2304_06437_amd/csrc/fused.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_d3q19_512_traffic.md")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(Q: int, M: int, ssize: int, csize: int, ref: int = 0):
    """Bytes per lattice update of (moments, stream-collide); ref: the
    reference-colour byte of two species, read by the moments sweep and
    written by stream-collide."""
    k1 = Q * ssize + M * csize + ref
    k2 = M * csize + Q * ssize + ref
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


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload: str = "d3q19_tg", seconds_hint: float = 15.0):
    """Time the FP64 CPU oracle on a bounded sample of the same workload: the
    same lattice, flow and parameters on a smaller domain (the per-node work
    does not depend on the domain size)."""
    import oracle

    w = WORKLOADS[workload]
    n = {9: 1024, 19: 128, 27: 96}[w["lattice"]]
    if w["species"] == 2:
        n = 96
    shape = (n, n, 1) if w["lattice"] == 9 else (n, n, n)
    kw = dict(lattice=w["lattice"], nx=shape[0], ny=shape[1], nz=shape[2], tau=w["tau"],
              order=w["order"], species=w["species"])
    if w["flow"] == "channel":
        kw.update(force=(1e-6, 0.0, 0.0), bb=(0, 0, 1))
    if w["flow"] == "cavity":
        kw.update(bb=(1, 1, 0), wall_u=lid_walls())
    if w["species"] == 2:
        kw.update(sigma=0.03, beta=0.7)
    p = oracle.Params(**kw)
    sub = dict(w, n=n)
    if w["flow"] == "droplets":
        from paper_2304_06437_amd import inputs

        centres = inputs.droplet_centres(n, 3, 12.0, gap=2.0, seed=7)
        rho, u, phi = inputs.droplets(n, centres, 12.0)
    else:
        rho, u, phi = workload_fields(sub, n)
    f = oracle.init(p, rho, u, phi)
    t = time.perf_counter()
    oracle.run(p, f, 1)
    one = time.perf_counter() - t
    steps = max(1, min(200, int(seconds_hint / max(one, 1e-3))))
    t = time.perf_counter()
    oracle.run(p, f, steps)
    dt = time.perf_counter() - t
    nodes = shape[0] * shape[1] * shape[2]
    return {
        "value": nodes * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": (w["desc"].format(n=n) if w["flow"] != "droplets" else
                   f"two-species D3Q19 {n}^3 periodic, 3 droplets radius 12, tau 1.0, "
                   "sigma 0.03, beta 0.7") +
                  f"; FP64 two-array oracle, {steps} steps ({dt:.1f} s) on a {n}-edge "
                  "domain; same per-node work as the benchmark",
        "host_cpu": cpu_model(),
        "nproc": os.cpu_count(),
    }


def serving(torch, jobs: int, rate: float, budget_gb: float, overlap: bool = True):
    """Continuous batching of a seeded Poisson request stream: D2Q9/D3Q19,
    Taylor-Green or channel, FP32 or shifted-FP16 storage, edge
    log-uniform 64..256 (n^2 or n^3), 200-2000 steps, admitted by an HBM
    budget.  Time-to-solution = arrival to moments on the host.  Set-up and
    read-back overlap the batch's steps (worker thread, own stream)."""
    from paper_2304_06437_amd.serving import GpuBackend, Server, poisson_mix

    specs = poisson_mix(jobs, rate=rate, seed=2026)
    side = torch.cuda.Stream()
    last = [time.perf_counter()]

    def progress(c):
        # one line on stderr every 20 s of a long serving run
        if time.perf_counter() - last[0] >= 20.0:
            last[0] = time.perf_counter()
            print(f"serving {jobs} requests at {rate}/s: t {c['t']:.0f} s, chunk {c['chunks']}, "
                  f"active {c['active']}, finished {c['finished']}", file=sys.stderr, flush=True)

    with torch.cuda.stream(side):
        be = GpuBackend()
        rep = Server(be, hbm_budget=int(budget_gb * 1e9), chunk_steps=200,
                     overlap=overlap, progress=progress).run(specs)
        be.close()
    torch.cuda.synchronize()
    s = rep.summary()
    s.update({"requests": jobs, "rate_per_s": rate, "budget_GB": budget_gb, "overlap": overlap,
              "mix": "D2Q9/D3Q19 x TG/channel x f32/f16s, edge 64..256 log-uniform, "
                     "200-2000 steps, seeded Poisson arrivals"})
    return s


def copy_ceilings(torch, nbytes: int = 4 << 30, reps: int = 10):
    """Device-to-device copy bandwidth (read + write bytes / time) of 4 GiB by
    three independent routes: the library's one-pass copy kernel, the HIP
    runtime's hipMemcpyAsync, and torch's copy_.  All timed with events on
    the current stream."""
    import ctypes

    from paper_2304_06437_amd import lb

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream().cuda_stream
    hip = ctypes.CDLL("libamdhip64.so")  # the runtime torch has loaded
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_int, ctypes.c_void_p]
    hip.hipMemcpyAsync.restype = ctypes.c_int
    hip_d2d = 3  # hipMemcpyDeviceToDevice

    def memcpy():
        rc = hip.hipMemcpyAsync(dst.data_ptr(), src.data_ptr(), nbytes, hip_d2d, stream)
        if rc != 0:
            raise RuntimeError(f"hipMemcpyAsync failed: {rc}")

    routes = {
        "lb_copy_kernel": lambda: lb.lb_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream),
        "hipMemcpyAsync_d2d": memcpy,
        "torch_copy_": lambda: dst.copy_(src),
    }
    out = {}
    for name, fn in routes.items():
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    out["best"] = max(out.values())
    out["bytes"] = nbytes
    return out


# name -> problem statement (all synthetic, seeded)
WORKLOADS = {
    "d3q19_tg": dict(lattice=19, n=512, tau=0.55, flow="tg3d", order=2, species=1,
                     desc="D3Q19 {n}^3 periodic 3D Taylor-Green (u0 0.02, tau 0.55, rho0 1)"),
    "d3q19_channel": dict(lattice=19, n=256, tau=0.6, flow="channel", order=2, species=1,
                          desc="D3Q19 {n}^3 channel: walls in z, periodic x/y, force 1e-6 along x, "
                               "tau 0.6, rho 1 + 1e-4 seeded noise"),
    "d3q27_tg3": dict(lattice=27, n=512, tau=0.55, flow="tg3d", order=3, species=1,
                      desc="D3Q27 third-order Hermite {n}^3 periodic 3D Taylor-Green (u0 0.02, "
                           "tau 0.55)"),
    "two_species": dict(lattice=19, n=256, tau=1.0, flow="droplets", order=2, species=2,
                        desc="two-species D3Q19 {n}^3 periodic, 64 droplets radius 12 at seeded "
                             "non-overlapping positions, density ratio 1, tau 1.0, sigma 0.03, "
                             "beta 0.7"),
    "d2q9_tg": dict(lattice=9, n=4096, tau=0.8, flow="tg2d", order=2, species=1,
                    desc="D2Q9 {n}^2 periodic 2D Taylor-Green (u0 0.01, tau 0.8)"),
    "d2q9_cavity": dict(lattice=9, n=4096, tau=0.6, flow="cavity", order=2, species=1,
                        desc="D2Q9 {n}^2 lid-driven cavity: bounce-back walls on all four "
                             "sides, lid (high y) moving along x at 0.05, tau 0.6, fluid at rest"),
}

LID = 0.05

# The paper's own single-component thread-safe numbers (Section 6, CUDA
# Fortran, FP32), other hardware: context for the workload of the same
# lattice and shape, never a target (the paper reports no 512^3 figure).
PAPER_CONTEXT = {
    "D3Q19 3D": {"value": 3600.0, "unit": "MLUPS", "hardware": "RTX 3090 (CUDA Fortran)",
                 "workload": "3D 256^3, single component, FP32"},
    "D2Q9 2D": {"value": 6100.0, "unit": "MLUPS", "hardware": "RTX 3090 (CUDA Fortran)",
                "workload": "2D 4096^2, single component, FP32"},
}


def lid_walls():
    """wall velocity [axis][low, high][component] of the cavity lid."""
    wu = [[[0.0] * 3 for _ in range(2)] for _ in range(3)]
    wu[1][1][0] = LID
    return wu


def workload_fields(w, n):
    from paper_2304_06437_amd import inputs

    if w["flow"] == "tg3d":
        return inputs.taylor_green_3d(n, n, n, 0.02) + (None,)
    if w["flow"] == "tg2d":
        return inputs.taylor_green_2d(n, n, 0.01) + (None,)
    if w["flow"] == "channel":
        return inputs.channel_noise(n, n, n, 3) + (None,)
    if w["flow"] == "droplets":
        centres = inputs.droplet_centres(n, 64, 12.0, gap=2.0, seed=7)
        return inputs.droplets(n, centres, 12.0)
    if w["flow"] == "cavity":
        D = 2 if w["lattice"] == 9 else 3
        N = n * n * (1 if D == 2 else n)
        return np.ones(N), np.zeros((D, N)), None
    raise ValueError(w["flow"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="d3q19_tg", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=0, help="domain edge (0: the workload's own)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16s", "bf16s"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=96,
                    help="requests in the serving measurement (0 to skip)")
    ap.add_argument("--serve-rates", default="50,5",
                    help="mean arrivals per second, comma-separated: the first is reported as "
                         "'serving' (saturating load), the second as 'serving_below_saturation'")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-serial", action="store_true",
                    help="serving loop without set-up / read-back overlap")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_06437_amd import inputs, lb
    from paper_2304_06437_amd.sim import Simulation, make_params

    lb.load()
    w = WORKLOADS[args.workload]
    n = args.n or w["n"]
    shape = (n, n, 1) if w["lattice"] == 9 else (n, n, n)
    N = shape[0] * shape[1] * shape[2]
    kw = dict(lattice=w["lattice"], shape=shape, tau=w["tau"], order=w["order"],
              storage=args.storage, species=w["species"])
    if w["flow"] == "channel":
        kw.update(force=(1e-6, 0.0, 0.0), bc=(0, 0, 1))
    if w["flow"] == "cavity":
        kw.update(bc=(1, 1, 0), wall_velocity=lid_walls())
    if w["species"] == 2:
        kw.update(sigma=0.03, beta=0.7)
    params = make_params(**kw)
    # device footprint, and without moment arrays where the shape has a fused
    # step (lb_params.keep_moments = 0: the population set alone)
    lean = make_params(keep_moments=0, **kw)
    memory = {"device_bytes": lb.lb_required_bytes(params),
              "bytes_per_node": round(lb.lb_required_bytes(params) / N, 2),
              "population_set_only": None}
    if lb.lb_validate(lean) == lb.LB_OK:
        memory["population_set_only"] = {
            "device_bytes": lb.lb_required_bytes(lean),
            "bytes_per_node": round(lb.lb_required_bytes(lean) / N, 2)}
    rho, u, phi = workload_fields(w, n)
    copies = copy_ceilings(torch) if not args.no_copy else None

    sim = Simulation(params)
    sim.init(rho, u, phi)
    del rho, u, phi
    path, z_tiles = lb.lb_get_step_path(sim.handle)
    fused = path == lb.LB_PATH_FUSED

    def timed(steps, warmup):
        sim.step(warmup)
        sim.synchronize()
        lb.lb_timing_begin(sim.handle, steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kms, klaunch = lb.lb_timing_end(sim.handle)
        return t1 - t0, kms, klaunch

    elapsed, kms, klaunch = timed(args.steps, args.warmup)
    check = sim.moments(rho=False, u=False, pineq=False)["conserved"]
    ssize = {"f32": 4, "f16s": 2, "bf16s": 2}[args.storage]
    Q = w["lattice"]
    D = 2 if Q == 9 else 3
    M = 1 + D + D * (D + 1) // 2 + (1 if w["species"] == 2 else 0)
    b1, b2 = algorithmic_bytes(Q * w["species"], M, ssize, 4, ref=1 if w["species"] == 2 else 0)
    bf = 2 * Q * ssize  # fused step: Q in, Q out
    two_sweep = None
    if fused:
        # the same state, on the two-sweep path
        lb.lb_set_step_path(sim.handle, lb.LB_PATH_TWO_SWEEP, 0)
        e2, k2, l2 = timed(args.steps, args.warmup)
        a2 = [k2[i] / max(l2[i], 1) for i in range(2)]
        two_sweep = {
            "value": round(N * args.steps / e2 / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(e2 * 1e3 / args.steps, 4),
            "bytes_per_update": b1 + b2,
            "step_GBs": round((b1 + b2) * N / (e2 / args.steps) / 1e9, 1),
            "kernels": {nm: {"avg_ms": round(a2[i], 4),
                             "algorithmic_GBs": round(bb * N / (a2[i] * 1e-3) / 1e9, 1)}
                        for i, (nm, bb) in enumerate((("moments", b1), ("stream_collide", b2)))},
        }
    sim.close()

    ms_per_step = elapsed * 1e3 / args.steps
    mlups = N * args.steps / elapsed / 1e6
    avg = [kms[i] / max(klaunch[i], 1) for i in range(2)]
    if fused:
        names, bytes_launch, dom, kidx = ["fused_step"], [bf * N], 0, [1]
        b_update = bf
    else:
        names, bytes_launch, kidx = ["moments", "stream_collide"], [b1 * N, b2 * N], [0, 1]
        dom = 0 if avg[0] > avg[1] else 1
        b_update = b1 + b2
    achieved = bytes_launch[dom] / (avg[kidx[dom]] * 1e-3) / 1e9
    headline = args.workload == "d3q19_tg" and args.storage == "f32" and n == 512
    traffic = read_traffic(names[dom]) if headline else None

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
            "workload": w["desc"].format(n=n) + f", {args.storage} population storage, "
                        "f32 arithmetic",
            "name": args.workload, "lattice": f"D{D}Q{Q}", "nodes": N,
            "storage": args.storage, "compute": "f32", "bytes_per_update": b_update,
            "path": "fused" if fused else "two_sweep", "z_tiles": z_tiles,
        },
        "memory": memory,
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
            names[i]: {"avg_ms": round(avg[kidx[i]], 4), "launches": klaunch[kidx[i]],
                       "algorithmic_GBs": round(bytes_launch[i] / (avg[kidx[i]] * 1e-3) / 1e9, 1),
                       "vs_best_copy": (round(bytes_launch[i] / (avg[kidx[i]] * 1e-3) / 1e9 /
                                              copies["best"], 4) if copies else None)}
            for i in range(len(names))
        },
        "step_GBs": round(b_update * N / (ms_per_step * 1e-3) / 1e9, 1),
        "step_frac_of_peak": round(b_update * N / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "two_sweep": two_sweep,
        "copy_ceilings_GBs": copies,
        "dominant_vs_best_copy": (round(achieved / copies["best"], 4) if copies else None),
        "mass_finite": bool(np.isfinite(check[0])),
    }
    ctx = PAPER_CONTEXT.get("D3Q19 3D" if Q == 19 and w["species"] == 1 else
                            "D2Q9 2D" if Q == 9 and w["species"] == 1 else "")
    if ctx:
        out["paper_context"] = dict(ctx, note="other hardware and domain size; context only")
    if args.serve_jobs > 0:
        rates = [float(r) for r in args.serve_rates.split(",") if r.strip()]
        for key, rate in zip(("serving", "serving_below_saturation"), rates):
            out[key] = serving(torch, args.serve_jobs, rate, args.serve_budget_gb,
                               overlap=not args.serve_serial)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
