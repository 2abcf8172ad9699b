"""Host-side checks of the C ABI (no GPU needed: nothing here launches work)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2304_06437_amd import lb

HERE = os.path.dirname(os.path.abspath(__file__))


def test_library_exports_every_declared_function():
    lib = lb.load()
    declared = lb.header_functions()
    assert "lb_create" in declared and "lb_step" in declared and "lb_moments" in declared
    nm = subprocess.run(["nm", "-D", "--defined-only", lb.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = {line.split()[-1] for line in nm.splitlines() if line.strip()}
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name), name


def test_params_default_is_valid():
    p = lb.lb_params_default()
    assert lb.lb_validate(p) == lb.LB_OK
    assert (p.lattice, p.nx, p.ny, p.nz, p.species) == (lb.LB_D3Q19, 32, 32, 32, 1)
    assert p.storage == lb.LB_STORE_F32 and p.compute == lb.LB_COMPUTE_F32


def test_struct_size_matches_c_layout():
    import ctypes
    p = lb.lb_params_default()
    assert p.struct_size == ctypes.sizeof(lb.lb_params)


@pytest.mark.parametrize("field,value", [
    ("tau", 0.5), ("tau", float("nan")), ("rho0", 0.0), ("lattice", 15),
    ("hermite_order", 4), ("nx", 0), ("storage", 9), ("compute", 5),
])
def test_invalid_parameters_rejected(field, value):
    p = lb.lb_params_default(**{field: value})
    assert lb.lb_validate(p) == lb.LB_EINVAL
    assert lb.lb_required_bytes(p) == 0
    with pytest.raises(lb.LbError) as e:
        lb.lb_create(p)
    assert e.value.status == lb.LB_EINVAL


def test_invalid_combinations_rejected():
    assert lb.lb_validate(lb.lb_params_default(hermite_order=3)) == lb.LB_EINVAL  # D3Q19
    assert lb.lb_validate(lb.lb_params_default(lattice=27, hermite_order=3)) == lb.LB_OK
    assert lb.lb_validate(lb.lb_params_default(lattice=9, nz=2)) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(lattice=9, nz=1)) == lb.LB_OK
    assert lb.lb_validate(lb.lb_params_default(lattice=9, nz=1, bc=(0, 0, 1))) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(storage=lb.LB_STORE_F64)) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(storage=lb.LB_STORE_F64,
                                               compute=lb.LB_COMPUTE_F64)) == lb.LB_OK
    assert lb.lb_validate(lb.lb_params_default(storage=lb.LB_STORE_F16S,
                                               compute=lb.LB_COMPUTE_F64)) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(bc=(2, 0, 0))) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(force=(float("inf"), 0, 0))) == lb.LB_EINVAL
    p = lb.lb_params_default()
    p.struct_size = 8
    assert lb.lb_validate(p) == lb.LB_EINVAL
    two = dict(species=2, sigma=0.03, beta=0.7)
    assert lb.lb_validate(lb.lb_params_default(**two)) == lb.LB_OK
    assert lb.lb_validate(lb.lb_params_default(lattice=9, nz=1, **two)) == lb.LB_OK
    assert lb.lb_validate(lb.lb_params_default(lattice=27, **two)) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(storage=lb.LB_STORE_BF16S, **two)) == lb.LB_EUNSUPPORTED
    assert lb.lb_validate(lb.lb_params_default(species=2, sigma=-1.0, beta=0.7)) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(species=2, sigma=0.03, beta=1.5)) == lb.LB_EINVAL
    assert lb.lb_validate(lb.lb_params_default(species=3)) == lb.LB_EINVAL


def _golden_arrays():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "memory_arrays.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, ts, ff, save = line.split()
        rows[name] = (int(ts), int(ff), int(save))
    return rows


def test_required_bytes_match_paper_array_counts():
    """Section 4: 15 (D2Q9) and 29 (D3Q19) single-precision arrays per node."""
    g = _golden_arrays()
    for name, lattice, nz in (("D2Q9", 9, 1), ("D3Q19", 19, 256)):
        p = lb.lb_params_default(lattice=lattice, nx=256, ny=256, nz=nz)
        N = 256 * 256 * nz
        arrays = g[name][0]
        extra = lb.lb_required_bytes(p) - arrays * 4 * N
        # only the FP64 reduction scratch (64 KiB), the fused step's progress
        # words (one per row and plane, 3D rows of 256 nodes) and alignment
        # remain
        words = 4 * (256 * nz + 3) if nz > 1 else 0
        assert 0 <= extra - words <= 64 * 1024 + 256 * (arrays + 3), (name, extra)
        # saving against the flip-flop layout, bytes per node (Section 4)
        assert (g[name][1] - arrays) * 4 == g[name][2]


def test_required_bytes_scale_with_precision():
    base = dict(nx=128, ny=128, nz=128)
    b32 = lb.lb_required_bytes(lb.lb_params_default(**base))
    b16 = lb.lb_required_bytes(lb.lb_params_default(storage=lb.LB_STORE_F16S, **base))
    b64 = lb.lb_required_bytes(lb.lb_params_default(storage=lb.LB_STORE_F64,
                                                    compute=lb.LB_COMPUTE_F64, **base))
    N = 128 ** 3
    words = 4 * (128 * 128 + 3)  # the fused step's progress words: FP32 and 16-bit only
    assert abs((b32 - b16) - 19 * 2 * N) < 4096
    assert abs((b64 - (b32 - words)) - 29 * 4 * N) < 4096


def test_strerror_and_null_destroy():
    for st in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(lb.lb_strerror(st), str) and lb.lb_strerror(st)
    assert lb.load().lb_destroy(None) == lb.LB_OK
    assert lb.load().lb_step(None, 1) == lb.LB_EINVAL
    assert lb.load().lb_moments(None, None, None, None, None, None) == lb.LB_EINVAL
    assert lb.load().lb_copy(None, None, 16, None) == lb.LB_EINVAL
    assert lb.load().lb_set_stream(None, None) == lb.LB_EINVAL
    assert lb.load().lb_set_step_path(None, 0, 0) == lb.LB_EINVAL
    assert lb.load().lb_set_fused_wait_limit(None, 1) == lb.LB_EINVAL
    assert lb.load().lb_check_division(None, None) == lb.LB_EINVAL


def _fused_rows(kw):
    """The fused step's shapes (lb_set_step_path): one species, D3Q19 or
    D3Q27, FP32 or 16-bit storage, nx = 128, 256, 512 (D3Q27: 128, 256)."""
    if kw.get("species", 1) != 1 or kw.get("lattice", 19) == 9:
        return False
    if kw.get("storage", lb.LB_STORE_F32) == lb.LB_STORE_F64:
        return False
    sizes = (128, 256) if kw.get("lattice", 19) == 27 else (128, 256, 512)
    return kw.get("nx", 32) in sizes


def _blocked_bytes(Q, M, NS, ssize, csize, species=1, rows=0):
    """Footprint of the documented blocked layout over NS storage nodes:
    block B = 32 KiB of population storage (at least 1024 nodes, at most the
    next power of two >= NS), node count padded to a multiple of B, each
    region 256-byte aligned, plus (two species) one reference-colour byte per
    padded node, plus 64 KiB of FP64 reduction partials, plus (shapes of the
    fused step) a 4-byte progress word per row (rows = ny nz) and 3 more."""
    B = 1024
    while B < NS and B * ssize < 32768:
        B *= 2
    npad = -(-NS // B) * B
    al = lambda v: -(-v // 256) * 256
    ref = al(npad) if species == 2 else 0
    sync = al(4 * (rows + 3)) if rows else 0
    return (al(species * Q * npad * ssize) + al(M * npad * csize) + ref + al(1024 * 8 * 8) + sync,
            B, npad)


def test_required_bytes_of_ragged_domains():
    """Storage nodes = px ny nz with the row pitch px: nx rounded up to the
    stream-collide sweep's vector chunk, where the sweep takes the narrowest
    lane vector V that needs no more 64-lane wavefronts per row than its
    widest one (D3Q19 FP32: V <= 4 in chunks of 2; 16-bit D3Q19 / D2Q9:
    V <= 8 in one chunk; D3Q27 FP32: V <= 4 in one chunk; two species FP32:
    V <= 4, FP64: V <= 2)."""
    f16, f64 = lb.LB_STORE_F16S, lb.LB_STORE_F64
    cases = [
        # (params, Q, M, storage bytes, compute bytes, species, row pitch)
        (dict(lattice=19, nx=37, ny=5, nz=7), 19, 10, 4, 4, 1, 37),       # V = 1
        (dict(lattice=19, nx=100, ny=90, nz=3), 19, 10, 4, 4, 1, 100),    # V = 2
        (dict(lattice=9, nx=300, ny=70, nz=1, storage=f16), 9, 6, 2, 4, 1, 304),  # V = 8
        (dict(lattice=27, nx=20, ny=19, nz=18, hermite_order=3, storage=f64,
              compute=lb.LB_COMPUTE_F64), 27, 10, 8, 8, 1, 20),
        (dict(lattice=19, nx=24, ny=20, nz=18, species=2, sigma=0.03, beta=0.7), 19, 11, 4, 4, 2,
         24),
        (dict(lattice=19, nx=1, ny=1, nz=1), 19, 10, 4, 4, 1, 1),
        (dict(lattice=19, nx=97, ny=6, nz=5), 19, 10, 4, 4, 1, 98),       # V = 2
        (dict(lattice=19, nx=131, ny=5, nz=4), 19, 10, 4, 4, 1, 132),     # V = 4 = 2 x 2
        (dict(lattice=19, nx=161, ny=4, nz=3, storage=f16), 19, 10, 2, 4, 1, 164),  # V = 4
        (dict(lattice=27, nx=197, ny=4, nz=3, hermite_order=3), 27, 10, 4, 4, 1, 200),
        (dict(lattice=19, nx=197, ny=6, nz=5, species=2, sigma=0.03, beta=0.7), 19, 11, 4, 4, 2,
         200),
        (dict(lattice=19, nx=131, ny=6, nz=5, species=2, sigma=0.03, beta=0.7, storage=f64,
              compute=lb.LB_COMPUTE_F64), 19, 11, 8, 8, 2, 132),
        (dict(lattice=19, nx=511, ny=3, nz=2), 19, 10, 4, 4, 1, 512),     # V = 4
        (dict(lattice=19, nx=64, ny=3, nz=2, storage=f16), 19, 10, 2, 4, 1, 64),   # V = 1
        # shapes of the fused step: progress words
        (dict(lattice=19, nx=128, ny=7, nz=5), 19, 10, 4, 4, 1, 128),
        (dict(lattice=19, nx=512, ny=3, nz=9, storage=f16), 19, 10, 2, 4, 1, 512),
        (dict(lattice=27, nx=256, ny=4, nz=6, hermite_order=3), 27, 10, 4, 4, 1, 256),
        (dict(lattice=27, nx=512, ny=4, nz=6), 27, 10, 4, 4, 1, 512),
        (dict(lattice=19, nx=256, ny=5, nz=3, storage=f64, compute=lb.LB_COMPUTE_F64), 19, 10,
         8, 8, 1, 256),
    ]
    for kw, Q, M, ss, cs, sp, px in cases:
        p = lb.lb_params_default(**kw)
        rows = p.ny * p.nz if _fused_rows(kw) else 0
        want, B, npad = _blocked_bytes(Q, M, px * p.ny * p.nz, ss, cs, sp, rows)
        assert lb.lb_required_bytes(p) == want, (kw, px, B, npad)


def test_wall_velocity_validation():
    def wv(axis, side, comp, v=0.05):
        w = np.zeros((3, 2, 3))
        w[axis, side, comp] = v
        return w
    ok = lb.lb_params_default(lattice=9, nx=32, ny=32, nz=1, bc=(1, 1, 0),
                              wall_velocity=wv(1, 1, 0))
    assert lb.lb_validate(ok) == lb.LB_OK
    assert lb.lb_required_bytes(ok) == lb.lb_required_bytes(
        lb.lb_params_default(lattice=9, nx=32, ny=32, nz=1, bc=(1, 1, 0)))
    # normal component, periodic axis, z component in 2D, non-finite
    for bad in (wv(1, 1, 1), wv(0, 0, 1, 0.0) + wv(2, 0, 0), wv(1, 0, 2), wv(1, 1, 0, np.nan)):
        p = lb.lb_params_default(lattice=9, nx=32, ny=32, nz=1, bc=(1, 1, 0), wall_velocity=bad)
        assert lb.lb_validate(p) == lb.LB_EINVAL
    p3 = lb.lb_params_default(lattice=19, bc=(0, 0, 1), wall_velocity=wv(2, 1, 0) + wv(2, 0, 1))
    assert lb.lb_validate(p3) == lb.LB_OK
    p3b = lb.lb_params_default(lattice=19, bc=(0, 0, 1), wall_velocity=wv(1, 1, 0))
    assert lb.lb_validate(p3b) == lb.LB_EINVAL
    two = lb.lb_params_default(lattice=19, bc=(0, 0, 1), species=2, sigma=0.03, beta=0.7,
                               wall_velocity=wv(2, 1, 0))
    assert lb.lb_validate(two) == lb.LB_EUNSUPPORTED


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before torch must not bring up a second HIP
    runtime (torch's streams would be invalid in it)."""
    code = (
        "from paper_2304_06437_amd import lb\n"
        "lb.load()\n"
        "import torch\n"
        "maps = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
        "print(len(maps))\n"
    )
    root = os.path.dirname(HERE)
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1", out.stdout


def test_noalloc_batch_limits_checked_before_any_device_call():
    import ctypes
    lib = lb.load()
    n = lb.LB_NOALLOC_MAX_HANDLES + 1
    hs = (ctypes.c_void_p * n)()
    ns = (ctypes.c_int64 * n)()
    assert lib.lb_step_batch_noalloc(hs, ns, n) == lb.LB_ENOMEM
    assert lib.lb_step_batch_noalloc(hs, ns, -1) == lb.LB_EINVAL
    assert lib.lb_step_batch_noalloc(None, None, 0) == lb.LB_OK
    assert lib.lb_step_batch_noalloc(hs, ns, 1) == lb.LB_EINVAL  # NULL handle
    hdr = open(lb.HEADER).read()
    assert f"#define LB_NOALLOC_MAX_HANDLES {lb.LB_NOALLOC_MAX_HANDLES}" in hdr
    assert "#define LB_NOALLOC_SCRATCH_BYTES (1u << 20)" in hdr
    assert lb.LB_NOALLOC_SCRATCH_BYTES == 1 << 20


def test_params_struct_versions():
    """Callers built against the earlier, shorter lb_params (no moving walls;
    no near-contact fields) are accepted; unknown sizes are not."""
    import ctypes
    assert (lb.LB_PARAMS_SIZE_V1 < lb.LB_PARAMS_SIZE_V2 < lb.LB_PARAMS_SIZE_V3
            < ctypes.sizeof(lb.lb_params))
    full = lb.lb_params_default(lattice=19, nx=24, ny=20, nz=16)
    want = lb.lb_required_bytes(full)
    for size in (lb.LB_PARAMS_SIZE_V1, lb.LB_PARAMS_SIZE_V2, lb.LB_PARAMS_SIZE_V3):
        p = lb.lb_params_default(lattice=19, nx=24, ny=20, nz=16)
        # the tail beyond the caller's size is garbage the library must not read
        raw = (ctypes.c_ubyte * ctypes.sizeof(lb.lb_params)).from_buffer(p)
        for i in range(size, ctypes.sizeof(lb.lb_params)):
            raw[i] = 0xFF
        p.struct_size = size
        assert lb.lb_validate(p) == lb.LB_OK
        assert lb.lb_required_bytes(p) == want
    for bad in (0, 8, lb.LB_PARAMS_SIZE_V1 - 8, ctypes.sizeof(lb.lb_params) + 8):
        p = lb.lb_params_default()
        p.struct_size = bad
        assert lb.lb_validate(p) == lb.LB_EINVAL
        assert lb.lb_required_bytes(p) == 0


def test_population_set_only_parameters():
    """keep_moments 0: the population set alone plus a staging buffer of at
    most 256 MiB in place of the moment arrays (Section 4's count without
    the M moments), only for shapes with a fused step."""
    assert lb.lb_params_default().keep_moments == 1
    for v in (-1, 2):
        assert lb.lb_validate(lb.lb_params_default(nx=128, keep_moments=v)) == lb.LB_EINVAL
    for kw in (dict(lattice=9, nx=128, ny=64, nz=1), dict(nx=96), dict(nx=1024),
               dict(nx=128, storage=lb.LB_STORE_F64, compute=lb.LB_COMPUTE_F64),
               dict(nx=128, species=2, sigma=0.03, beta=0.7)):
        p = lb.lb_params_default(keep_moments=0, **kw)
        assert lb.lb_validate(p) == lb.LB_EUNSUPPORTED, kw
        assert lb.lb_required_bytes(p) == 0, kw
    al = lambda v: -(-v // 256) * 256
    for (nx, ny, nz, st, ss) in ((128, 24, 20, lb.LB_STORE_F32, 4),
                                 (256, 40, 33, lb.LB_STORE_F16S, 2),
                                 (512, 512, 512, lb.LB_STORE_F32, 4)):
        kw = dict(lattice=19, nx=nx, ny=ny, nz=nz, storage=st)
        full, B, npad = _blocked_bytes(19, 10, nx * ny * nz, ss, 4, rows=ny * nz)
        assert lb.lb_required_bytes(lb.lb_params_default(**kw)) == full
        lean = lb.lb_required_bytes(lb.lb_params_default(keep_moments=0, **kw))
        stage = min(10 * npad * 4, 256 << 20)
        assert lean == full - al(10 * npad * 4) + al(stage), (nx, ny, nz)
    # D3Q19 FP32 at 512^3: 76 B per node plus the bounded staging buffer
    # (29 arrays of 4 B with the moments)
    assert abs(lean / 512 ** 3 - 76) < 2.1 and abs(full / 512 ** 3 - 116) < 0.1


def test_near_contact_parameters():
    two = dict(species=2, sigma=0.03, beta=0.7)
    assert lb.lb_validate(lb.lb_params_default(nci_strength=0.1, **two)) == lb.LB_OK
    assert lb.lb_validate(lb.lb_params_default(nci_strength=0.1)) == lb.LB_EINVAL  # one species
    for kw in (dict(nci_strength=-0.1), dict(nci_strength=float("nan")),
               dict(nci_strength=0.1, nci_eps=0.0), dict(nci_strength=0.1, nci_eps=2.0),
               dict(nci_strength=0.1, nci_reach=0), dict(nci_strength=0.1, nci_reach=9)):
        assert lb.lb_validate(lb.lb_params_default(**kw, **two)) == lb.LB_EINVAL, kw
    # off: eps and reach are not looked at
    assert lb.lb_validate(lb.lb_params_default(nci_strength=0.0, nci_reach=0, **two)) == lb.LB_OK
    # the flag array: one byte per padded node, 256-byte aligned
    p_off = lb.lb_params_default(nx=40, ny=24, nz=20, **two)
    p_on = lb.lb_params_default(nx=40, ny=24, nz=20, nci_strength=0.1, **two)
    extra = lb.lb_required_bytes(p_on) - lb.lb_required_bytes(p_off)
    assert extra >= 40 * 24 * 20 and extra % 256 == 0 and extra < 2 * 40 * 24 * 20 + 8192
