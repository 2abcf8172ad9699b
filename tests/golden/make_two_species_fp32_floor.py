"""Write two_species_fp32_floor.json: the float32 rounding floor of the
two-species colour-gradient step (Section 2.1) on the GPU parity cases.

For each case the oracle's numpy twin runs the same conventional two-array
step with every array and constant in float32 (oracle.twoarray.simulate,
dtype float32) and is compared with the FP64 C oracle: the max-relative
velocity error, the largest phase-field error and, for the conservation
case, the per-node drift of each species' mass.  These are what plain
float32 arithmetic of the method gives; the GPU FP32 tests are held to them.

    python tests/golden/make_two_species_fp32_floor.py

Calls only oracle/ (and the seeded input generators).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from oracle import twoarray  # noqa: E402
from two_species_cases import (CASES, CONSERVATION, FLOW_CASES, flow_state,  # noqa: E402
                               sharp_state)

OUT = os.path.join(HERE, "two_species_fp32_floor.json")


def max_rel(a, ref):
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300))


def floor_of(p, rho, u, phi, steps):
    ref = oracle.simulate(p, rho, u, steps, phi=phi)
    f32 = twoarray.simulate(p, rho, u, steps, phi=phi, dtype=np.float32)
    return {"u_max_rel": max_rel(f32["u"], ref["u"]),
            "phi_max_abs": float(np.abs(f32["phi"] - ref["phi"]).max()),
            "steps": steps}


def main():
    out = {"source": "oracle.twoarray.simulate(dtype=float32) vs oracle.simulate (FP64 C)",
           "cases": {}, "flow_cases": {}}
    for name, (lattice, shape, tau, steps, bc, sigma, beta) in CASES.items():
        t = time.time()
        rho, u, phi = sharp_state(lattice, shape, 3)
        p = oracle.Params(lattice=lattice, nx=shape[0], ny=shape[1], nz=shape[2], tau=tau,
                          bb=bc, species=2, sigma=sigma, beta=beta)
        out["cases"][name] = floor_of(p, rho, u, phi, steps)
        print(name, out["cases"][name], f"{time.time() - t:.0f}s", flush=True)
    for name, (lattice, shape, tau, steps, sigma, beta) in FLOW_CASES.items():
        t = time.time()
        rho, u, phi = flow_state(lattice, shape)
        p = oracle.Params(lattice=lattice, nx=shape[0], ny=shape[1], nz=shape[2], tau=tau,
                          species=2, sigma=sigma, beta=beta)
        out["flow_cases"][name] = floor_of(p, rho, u, phi, steps)
        print(name, out["flow_cases"][name], f"{time.time() - t:.0f}s", flush=True)
    lattice, shape, tau, steps, sigma, beta = CONSERVATION
    rho, u, phi = sharp_state(lattice, shape, 9)
    p = oracle.Params(lattice=lattice, nx=shape[0], ny=shape[1], nz=shape[2], tau=tau,
                      species=2, sigma=sigma, beta=beta)
    N = shape[0] * shape[1] * shape[2]
    f32 = twoarray.simulate(p, rho, u, steps, phi=phi, dtype=np.float32)
    out["conservation"] = {
        "red_drift_per_node": abs(f32["mass_red"] - float((rho * (1 + phi) / 2).sum())) / N,
        "blue_drift_per_node": abs(f32["mass_blue"] - float((rho * (1 - phi) / 2).sum())) / N,
        "steps": steps,
    }
    print("conservation", out["conservation"], flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
