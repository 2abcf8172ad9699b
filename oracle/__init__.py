"""FP64 CPU oracle for the regularized lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2304_06437_amd``) never imports, links or executes anything here, and
this package imports nothing from the product.

Two independent implementations live here:

* ``lbref.c`` (wrapped below): plain C, FP64, the conventional regularized
  step -- collide every node, push every post-collision population to its
  neighbour, two population arrays.  The thread-safe reordering of Section 3
  of the paper reaches exactly this result (up to rounding order).
* ``twoarray.py``: the same conventional step written with numpy array
  operations (``np.roll`` streaming), used on tiny grids to cross-check the C
  code.

Array conventions (shared with the C file): node index n = x + nx*(y + ny*z);
populations f[species][a][n]; velocity u[alpha][n] (alpha < D); the
non-equilibrium stress pineq[k][n] with k ordered xx, yy, (zz), xy, (xz, yz).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbref.c")
_LIB_PATH = os.path.join(_HERE, "_lbref.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile lbref.c into _lbref.so (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("bb", ctypes.c_int32 * 3),
        ("species", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("sigma", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("wall_u", ctypes.c_double * 18),
        ("nci_strength", ctypes.c_double),
        ("nci_eps", ctypes.c_double),
        ("nci_reach", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


@dataclass
class Params:
    """Problem statement of one simulation (Sections 2-3 of the paper)."""
    lattice: int = 19            # 9 (D2Q9), 19 (D3Q19), 27 (D3Q27)
    nx: int = 8
    ny: int = 8
    nz: int = 8
    tau: float = 0.8
    rho0: float = 1.0
    force: tuple = (0.0, 0.0, 0.0)
    bb: tuple = (0, 0, 0)        # per axis: 1 = halfway bounce-back walls
    order: int = 2
    species: int = 1
    sigma: float = 0.0
    beta: float = 0.0
    wall_u: tuple = None         # [axis][low, high][component] wall velocities
    nci_strength: float = 0.0    # near-contact force constant (two species); 0 = off
    nci_eps: float = 0.1         # bulk threshold: phi < -1 + nci_eps
    nci_reach: int = 1           # sampling distance along lattice directions

    @property
    def D(self) -> int:
        return 2 if self.lattice == 9 else 3

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def _c(self) -> _Params:
        p = _Params()
        p.lattice = self.lattice
        p.order = self.order
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        for i in range(3):
            p.bb[i] = int(self.bb[i])
            p.force[i] = float(self.force[i])
        p.species = self.species
        p.tau = self.tau
        p.rho0 = self.rho0
        p.sigma = self.sigma
        p.beta = self.beta
        if self.wall_u is not None:
            wu = np.asarray(self.wall_u, dtype=np.float64).reshape(18)
            for i in range(18):
                p.wall_u[i] = float(wu[i])
        p.nci_strength = self.nci_strength
        p.nci_eps = self.nci_eps
        p.nci_reach = self.nci_reach
        return p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.ref_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    dp, ctypes.POINTER(ctypes.c_int)]
        lib.ref_init.argtypes = [pp, dp, dp, dp, dp]
        lib.ref_run.argtypes = [pp, dp, ctypes.c_int64]
        lib.ref_moments.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.ref_collide_node.argtypes = [pp, dp, dp]
        lib.ref_equilibrium_node.argtypes = [pp, ctypes.c_double, dp, dp]
        lib.ref_threads.argtypes = []
        lib.ref_nci.argtypes = [pp, dp, ctypes.POINTER(ctypes.c_uint8), dp]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice(kind: int):
    """Velocity set of a lattice: (c[Q,3] int, w[Q] float64, opp[Q] int)."""
    lib = _load()
    q, d = ctypes.c_int(), ctypes.c_int()
    c = (ctypes.c_int * 81)()
    w = np.zeros(27)
    opp = (ctypes.c_int * 27)()
    if lib.ref_lattice(kind, ctypes.byref(q), ctypes.byref(d), c, _ptr(w), opp) != 0:
        raise ValueError(f"unknown lattice {kind}")
    Q = q.value
    cc = np.array(c[: 3 * Q], dtype=np.int64).reshape(Q, 3)
    return cc, w[:Q].copy(), np.array(opp[:Q], dtype=np.int64)


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().ref_threads())


def init(p: Params, rho, u, phi=None) -> np.ndarray:
    """Equilibrium populations f[species*Q*N] for the given fields."""
    lib = _load()
    Q = len(lattice(p.lattice)[1])
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    assert rho.size == p.N and u.size == p.D * p.N
    if p.species == 2:
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        assert phi.size == p.N
    f = np.empty(p.species * Q * p.N)
    pc = p._c()
    if lib.ref_init(ctypes.byref(pc), _ptr(rho), _ptr(u), _ptr(phi) if p.species == 2 else None,
                    _ptr(f)) != 0:
        raise ValueError("invalid parameters")
    return f


def run(p: Params, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance f in place by nsteps regularized steps; returns f."""
    lib = _load()
    pc = p._c()
    rc = lib.ref_run(ctypes.byref(pc), _ptr(f), int(nsteps))
    if rc != 0:
        raise RuntimeError(f"ref_run failed ({rc})")
    return f


def moments(p: Params, f: np.ndarray) -> dict:
    """rho[N], u[D,N], pineq[K,N] (and phi[N] for two species) of f."""
    lib = _load()
    N, D = p.N, p.D
    K = 3 if D == 2 else 6
    rho = np.empty(N)
    u = np.empty(D * N)
    pineq = np.empty(K * N)
    phi = np.empty(N) if p.species == 2 else None
    pc = p._c()
    if lib.ref_moments(ctypes.byref(pc), _ptr(f), _ptr(rho), _ptr(u), _ptr(pineq),
                       _ptr(phi)) != 0:
        raise ValueError("invalid parameters")
    out = {"rho": rho, "u": u.reshape(D, N), "pineq": pineq.reshape(K, N)}
    if phi is not None:
        out["phi"] = phi
    return out


def simulate(p: Params, rho, u, nsteps: int, phi=None) -> dict:
    """Initialise at equilibrium, run nsteps, return the moments."""
    f = init(p, rho, u, phi)
    run(p, f, nsteps)
    return moments(p, f)


def collide_node(p: Params, f) -> np.ndarray:
    """Regularized post-collision populations of a single node (one species)."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    pc = p._c()
    if lib.ref_collide_node(ctypes.byref(pc), _ptr(f), _ptr(out)) != 0:
        raise ValueError("invalid parameters")
    return out


def equilibrium_node(p: Params, rho: float, u) -> np.ndarray:
    """Equilibrium populations of a single node."""
    lib = _load()
    Q = len(lattice(p.lattice)[1])
    uu = np.zeros(3)
    uu[: len(u)] = u
    out = np.empty(Q)
    pc = p._c()
    if lib.ref_equilibrium_node(ctypes.byref(pc), float(rho), _ptr(uu), _ptr(out)) != 0:
        raise ValueError("invalid parameters")
    return out


def nci(p: Params, f: np.ndarray):
    """Near-contact flags[N] (bool) and forces[D, N] of the current
    two-species populations (Section 2.2, flagging pass and force)."""
    lib = _load()
    N = p.N
    flag = np.zeros(N, dtype=np.uint8)
    force = np.empty(3 * N)
    pc = p._c()
    if lib.ref_nci(ctypes.byref(pc), _ptr(f), flag.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                   _ptr(force)) != 0:
        raise ValueError("invalid parameters")
    return flag.astype(bool), force.reshape(3, N)[: p.D]
