"""ctypes binding of liblb.so (include/lb.h): argument marshalling only.

Every entry point keeps the C name.  Device memory and streams may come from
PyTorch (``torch.empty(..., device='cuda')`` and
``torch.cuda.current_stream().cuda_stream``); all computation runs in the HIP
kernels of liblb.so.  There is no fallback: if the library is not built,
loading it raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblb.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lb.h")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EUNSUPPORTED, LB_EDEVICE, LB_ENONFINITE = 0, -1, -2, -3, -4, -5
LB_D2Q9, LB_D3Q19, LB_D3Q27 = 9, 19, 27
LB_PERIODIC, LB_BOUNCEBACK = 0, 1
LB_STORE_F64, LB_STORE_F32, LB_STORE_F16S, LB_STORE_BF16S = 0, 1, 2, 3
LB_COMPUTE_F64, LB_COMPUTE_F32 = 0, 1

STORAGE = {"f64": LB_STORE_F64, "f32": LB_STORE_F32, "f16s": LB_STORE_F16S,
           "bf16s": LB_STORE_BF16S}


class lb_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_size_t),
        ("lattice", ctypes.c_int32),
        ("hermite_order", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("bc", ctypes.c_int32 * 3),
        ("species", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("sigma", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("compute", ctypes.c_int32),
        ("wall_velocity", ctypes.c_double * 18),   # [axis][low, high][component]
        ("nci_strength", ctypes.c_double),
        ("nci_eps", ctypes.c_double),
        ("nci_reach", ctypes.c_int32),
        ("nci_reserved_", ctypes.c_int32),
        ("keep_moments", ctypes.c_int32),
        ("keep_moments_reserved_", ctypes.c_int32),
    ]


# struct_size of the earlier versions of lb_params (include/lb.h)
LB_PARAMS_SIZE_V1 = lb_params.wall_velocity.offset
LB_PARAMS_SIZE_V2 = lb_params.nci_strength.offset
LB_PARAMS_SIZE_V3 = lb_params.keep_moments.offset


class LbError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lb_strerror(status)} ({status})")


_lib = None


def load():
    """Open liblb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2304_06437_amd.build")
    # PyTorch ships its own HIP runtime.  Loaded first, it is the runtime
    # liblb.so binds to (same library name), so the streams and device
    # memory torch hands over belong to the library's runtime; loaded after
    # liblb.so, a second runtime would come up beside the system one and
    # torch's streams would be invalid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(lb_params)
    H = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.lb_params_default.argtypes = [P]
    lib.lb_params_default.restype = None
    lib.lb_required_bytes.argtypes = [P]
    lib.lb_required_bytes.restype = ctypes.c_size_t
    lib.lb_validate.argtypes = [P]
    lib.lb_create.argtypes = [P, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                              ctypes.POINTER(H)]
    lib.lb_init.argtypes = [H, dp, dp, dp]
    lib.lb_step.argtypes = [H, ctypes.c_int64]
    lib.lb_synchronize.argtypes = [H]
    lib.lb_set_stream.argtypes = [H, ctypes.c_void_p]
    lib.lb_moments.argtypes = [H, dp, dp, dp, dp, dp]
    lib.lb_step_count.argtypes = [H]
    lib.lb_step_count.restype = ctypes.c_int64
    lib.lb_destroy.argtypes = [H]
    lib.lb_strerror.argtypes = [ctypes.c_int]
    lib.lb_strerror.restype = ctypes.c_char_p
    lib.lb_timing_begin.argtypes = [H, ctypes.c_int64]
    lib.lb_timing_end.argtypes = [H, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.lb_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.lb_check_division.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    lib.lb_sweep.argtypes = [H, ctypes.c_int]
    lib.lb_set_sweep_order.argtypes = [H, ctypes.c_int]
    lib.lb_set_step_path.argtypes = [H, ctypes.c_int, ctypes.c_int64]
    lib.lb_get_step_path.argtypes = [H, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.lb_set_fused_wait_limit.argtypes = [H, ctypes.c_int64]
    lib.lb_layout.argtypes = [H, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)]
    lib.lb_batch_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.lb_step_batch.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.c_int]
    lib.lb_step_batch_noalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.lb_batch_step.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.lb_batch_set_graphs.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.lb_batch_conserved.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.c_int, dp]
    lib.lb_batch_destroy.argtypes = [ctypes.c_void_p]
    _lib = lib
    return lib


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/lb.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", text)))


def _check(status: int, where: str):
    if status != LB_OK:
        raise LbError(status, where)


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- entry points -----------------------------------------------------------

def lb_params_default(**overrides) -> lb_params:
    p = lb_params()
    load().lb_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if k in ("bc", "force"):
            for i in range(3):
                getattr(p, k)[i] = v[i]
        elif k == "wall_velocity":
            flat = [float(x) for x in np.asarray(v, dtype=np.float64).reshape(18)]
            for i in range(18):
                p.wall_velocity[i] = flat[i]
        else:
            setattr(p, k, v)
    return p


def lb_required_bytes(p: lb_params) -> int:
    return int(load().lb_required_bytes(ctypes.byref(p)))


def lb_validate(p: lb_params) -> int:
    return int(load().lb_validate(ctypes.byref(p)))


def lb_create(p: lb_params, dev_mem: int = 0, dev_bytes: int = 0, hip_stream: int = 0):
    h = ctypes.c_void_p()
    _check(load().lb_create(ctypes.byref(p), ctypes.c_void_p(dev_mem or None), dev_bytes,
                            ctypes.c_void_p(hip_stream or None), ctypes.byref(h)), "lb_create")
    return h


def lb_init(h, rho, u, phi=None):
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    if phi is not None:
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
    _check(load().lb_init(h, _dptr(rho), _dptr(u), _dptr(phi)), "lb_init")


def lb_step(h, nsteps: int):
    _check(load().lb_step(h, int(nsteps)), "lb_step")


def lb_sweep(h, which: int):
    _check(load().lb_sweep(h, int(which)), "lb_sweep")


def lb_set_sweep_order(h, order: int):
    """0 natural, 1 reversed, 2 strided order of the stream-collide
    sweep's wavefronts (results are bitwise the same)."""
    _check(load().lb_set_sweep_order(h, int(order)), "lb_set_sweep_order")


LB_PATH_AUTO, LB_PATH_TWO_SWEEP, LB_PATH_FUSED = 0, 1, 2


def lb_set_step_path(h, path: int, z_tiles: int = 0):
    """Path of lb_step: LB_PATH_AUTO, LB_PATH_TWO_SWEEP or LB_PATH_FUSED
    (z_tiles runs of planes per row, 0 to choose)."""
    _check(load().lb_set_step_path(h, int(path), int(z_tiles)), "lb_set_step_path")


def lb_set_fused_wait_limit(h, polls: int):
    """Polls before a wait of the fused step gives up (tests of that path)."""
    _check(load().lb_set_fused_wait_limit(h, int(polls)), "lb_set_fused_wait_limit")


def lb_get_step_path(h):
    """(path lb_step takes: LB_PATH_TWO_SWEEP or LB_PATH_FUSED, z_tiles)."""
    path = ctypes.c_int(0)
    zt = ctypes.c_int64(0)
    _check(load().lb_get_step_path(h, ctypes.byref(path), ctypes.byref(zt)), "lb_get_step_path")
    return path.value, zt.value


def lb_check_division(stream=None):
    """Mismatches of the short division against the IEEE one over every
    finite FP32 input, for the divisors (3, 9, 27)."""
    out = (ctypes.c_uint64 * 3)()
    _check(load().lb_check_division(stream, out), "lb_check_division")
    return tuple(int(v) for v in out)


def lb_layout(h):
    """(population byte offset, moment byte offset, block size B in nodes,
    padded storage node count, row pitch px): node (x, y, z) is storage node
    n = x + px (y + ny z), and element (a, n) of a region of NA arrays sits
    at element (n // B) * NA * B + a * B + n % B of that region."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    c, d, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().lb_layout(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                            ctypes.byref(e)), "lb_layout")
    return a.value, b.value, c.value, d.value, e.value


def lb_synchronize(h):
    _check(load().lb_synchronize(h), "lb_synchronize")


def lb_set_stream(h, stream: int):
    """Rebind handle h to another HIP stream (the caller orders the work)."""
    _check(load().lb_set_stream(h, ctypes.c_void_p(stream)), "lb_set_stream")


def lb_moments(h, p: lb_params, rho=True, u=True, pineq=True, phi=False, conserved=True,
               allow_nonfinite=False):
    """Returns dict of numpy arrays: rho[N], u[D,N], pineq[K,N], phi[N], conserved[6]."""
    N = p.nx * p.ny * p.nz
    D = 2 if p.lattice == LB_D2Q9 else 3
    K = D * (D + 1) // 2
    out = {}
    a_rho = np.empty(N) if rho else None
    a_u = np.empty(D * N) if u else None
    a_pi = np.empty(K * N) if pineq else None
    a_phi = np.empty(N) if phi else None
    a_c = np.empty(6) if conserved else None
    st = load().lb_moments(h, _dptr(a_rho), _dptr(a_u), _dptr(a_pi), _dptr(a_phi), _dptr(a_c))
    if not (allow_nonfinite and st == LB_ENONFINITE):
        _check(st, "lb_moments")
    if rho:
        out["rho"] = a_rho
    if u:
        out["u"] = a_u.reshape(D, N)
    if pineq:
        out["pineq"] = a_pi.reshape(K, N)
    if phi:
        out["phi"] = a_phi
    if conserved:
        out["conserved"] = a_c
    out["status"] = st
    return out


def lb_step_count(h) -> int:
    return int(load().lb_step_count(h))


def lb_destroy(h):
    _check(load().lb_destroy(h), "lb_destroy")


def lb_strerror(status: int) -> str:
    return load().lb_strerror(int(status)).decode()


def lb_timing_begin(h, max_steps: int):
    _check(load().lb_timing_begin(h, int(max_steps)), "lb_timing_begin")


def lb_timing_end(h):
    """Returns ([ms_moments, ms_stream_collide], [launches, launches])."""
    ms = (ctypes.c_double * 2)()
    n = (ctypes.c_int64 * 2)()
    _check(load().lb_timing_end(h, ms, n), "lb_timing_end")
    return [ms[0], ms[1]], [n[0], n[1]]


def lb_copy(dst: int, src: int, nbytes: int, hip_stream: int = 0):
    _check(load().lb_copy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes,
                          ctypes.c_void_p(hip_stream or None)), "lb_copy")


def lb_batch_create(hip_stream: int = 0):
    b = ctypes.c_void_p()
    _check(load().lb_batch_create(ctypes.c_void_p(hip_stream or None), ctypes.byref(b)),
           "lb_batch_create")
    return b


def lb_batch_step(b, handles, nsteps):
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[h.value for h in handles])
    ns = (ctypes.c_int64 * n)(*[int(k) for k in nsteps])
    _check(load().lb_batch_step(b, hs, ns, n), "lb_batch_step")


def lb_step_batch(handles, nsteps):
    """One-shot batched step of handles on one stream (see lb_batch_step)."""
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[h.value for h in handles])
    ns = (ctypes.c_int64 * n)(*[int(k) for k in nsteps])
    _check(load().lb_step_batch(hs, ns, n), "lb_step_batch")


LB_NOALLOC_MAX_HANDLES = 1024
LB_NOALLOC_SCRATCH_BYTES = 1 << 20


def lb_step_batch_noalloc(handles, nsteps):
    """Batched step of handles on one stream without any allocation: the
    descriptor tables go to the library's fixed per-device array; returns
    without waiting."""
    n = len(handles)
    hs = (ctypes.c_void_p * max(n, 1))(*[h.value for h in handles])
    ns = (ctypes.c_int64 * max(n, 1))(*[int(k) for k in nsteps])
    _check(load().lb_step_batch_noalloc(hs, ns, n), "lb_step_batch_noalloc")


def lb_batch_conserved(b, handles):
    """FP64 conservation sums of several handles in one round trip:
    (array[count, 6] of mass, j (3), red mass, blue mass; status), status
    LB_ENONFINITE when some row is not finite."""
    n = len(handles)
    out = np.empty((max(n, 1), 6))
    hs = (ctypes.c_void_p * max(n, 1))(*[h.value for h in handles])
    st = load().lb_batch_conserved(b, hs, n, _dptr(out))
    if st not in (LB_OK, LB_ENONFINITE):
        _check(st, "lb_batch_conserved")
    return out[:n], st


def lb_batch_set_graphs(b, enable: bool):
    _check(load().lb_batch_set_graphs(b, 1 if enable else 0), "lb_batch_set_graphs")


def lb_batch_destroy(b):
    _check(load().lb_batch_destroy(b), "lb_batch_destroy")
