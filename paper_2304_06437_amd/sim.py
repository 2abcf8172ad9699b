"""One simulation on the GPU: liblb.so handle + PyTorch-owned device memory.

PyTorch supplies the device buffer (``lb_required_bytes`` bytes) and the
stream; every step runs in the library's HIP kernels.  This is marshalling
only.
"""
from __future__ import annotations

import numpy as np

from . import lb


def make_params(lattice=19, shape=(32, 32, 32), tau=0.6, rho0=1.0, force=(0.0, 0.0, 0.0),
                bc=(0, 0, 0), order=2, storage="f32", species=1, sigma=0.0, beta=0.0,
                wall_velocity=None, nci_strength=0.0, nci_eps=0.1, nci_reach=1, keep_moments=1):
    """lb_params for a problem; wall_velocity[axis][low, high][component]
    gives moving walls on bounce-back faces; nci_* the near-contact
    interactions of two species; keep_moments=0 holds the population set
    only (fused step only)."""
    st = lb.STORAGE[storage] if isinstance(storage, str) else int(storage)
    compute = lb.LB_COMPUTE_F64 if st == lb.LB_STORE_F64 else lb.LB_COMPUTE_F32
    kw = {} if wall_velocity is None else dict(wall_velocity=wall_velocity)
    kw.update(nci_strength=nci_strength, nci_eps=nci_eps, nci_reach=nci_reach,
              keep_moments=keep_moments)
    return lb.lb_params_default(lattice=lattice, nx=shape[0], ny=shape[1], nz=shape[2], tau=tau,
                                rho0=rho0, force=tuple(force), bc=tuple(bc),
                                hermite_order=order, storage=st, compute=compute,
                                species=species, sigma=sigma, beta=beta, **kw)


class Simulation:
    """Handle lifetime bound to a torch device buffer on the current stream."""

    def __init__(self, params: lb.lb_params, device=None, stream=None):
        import torch

        self.params = params
        self.nbytes = lb.lb_required_bytes(params)
        if self.nbytes == 0:
            raise lb.LbError(lb.lb_validate(params), "lb_required_bytes")
        dev = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        self.handle = lb.lb_create(params, self.buffer.data_ptr(), self.nbytes,
                                   self.stream.cuda_stream)

    @property
    def N(self) -> int:
        p = self.params
        return p.nx * p.ny * p.nz

    @property
    def D(self) -> int:
        return 2 if self.params.lattice == lb.LB_D2Q9 else 3

    def init(self, rho, u, phi=None):
        lb.lb_init(self.handle, rho, u, phi)

    def step(self, n: int):
        lb.lb_step(self.handle, n)

    def synchronize(self):
        lb.lb_synchronize(self.handle)

    def set_stream(self, stream):
        """Enqueue later work on another torch stream (the caller orders it)."""
        lb.lb_set_stream(self.handle, stream.cuda_stream)
        self.stream = stream

    def moments(self, **kw):
        return lb.lb_moments(self.handle, self.params, **kw)

    def close(self):
        if self.handle is not None:
            lb.lb_destroy(self.handle)
            self.handle = None
            self.buffer = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(params: lb.lb_params, rho, u, nsteps: int, phi=None, phi_out=False, **moment_kw):
    """Initialise, step and read back; returns the moments dict."""
    with Simulation(params) as sim:
        sim.init(rho, u, phi)
        sim.step(nsteps)
        return sim.moments(phi=phi_out, **moment_kw)


def max_rel(a: np.ndarray, ref: np.ndarray) -> float:
    """max |a - ref| / max |ref| over all components."""
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300))
