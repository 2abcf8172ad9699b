"""Storage codec pin: the shifted 16-bit modes store the round-to-nearest-even
image of the FP32 link value.

lb_init evaluates the equilibrium links of the same fields with the same FP32
arithmetic whatever the storage type; only the final store differs.  So the
raw FP16 population region must equal numpy's float16 conversion of the raw
FP32 region, and the raw BF16 region the round-to-nearest-even truncation of
the FP32 bits, bit for bit.  The paper proposes 16-bit population storage
with 32-bit arithmetic (Sections 6.1, 6.3 and 7) without fixing a rounding
rule; round-to-nearest-even is the reading taken.
"""
import numpy as np
import pytest

from paper_2304_06437_amd import lb
from paper_2304_06437_amd.sim import Simulation, make_params

pytestmark = pytest.mark.gpu

Q = {9: 9, 19: 19, 27: 27}


def _fields(shape, D, seed):
    """Half the nodes with O(1e-2) deviations, half with O(1e-6) ones, so the
    16-bit stores see normal, subnormal (FP16) and tie-rounding cases."""
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    amp = np.where(np.arange(N) % 2 == 0, 1.0, 1e-4)
    rho = 1.0 + 0.05 * amp * rng.uniform(-1, 1, N)
    u = 0.1 * amp * rng.uniform(-1, 1, (D, N))
    return rho, u


def _raw_populations(lattice, shape, storage, order, rho, u):
    p = make_params(lattice=lattice, shape=shape, storage=storage, order=order)
    with Simulation(p) as sim:
        sim.init(rho, u)
        sim.synchronize()
        pop_off, _, B, npad, px = lb.lb_layout(sim.handle)
        ssize = {"f32": 4, "f16s": 2, "bf16s": 2}[storage]
        q = Q[lattice]
        raw = sim.buffer[pop_off:pop_off + q * npad * ssize].cpu().numpy()
    dt = np.uint32 if ssize == 4 else np.uint16
    region = raw.view(dt).reshape(npad // B, q, B)
    # storage node of every lattice node: x + px (y + ny z)
    nx, ny, nz = shape
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    n = (x + px * (y + ny * z)).reshape(-1)
    return region[n // B, :, n % B]  # (N, Q) raw bits


def _bf16_rne(bits32):
    """Round-to-nearest-even of FP32 bit patterns to BF16 (finite values)."""
    b = bits32.astype(np.uint64)
    lsb = (b >> 16) & 1
    return ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)


CASES = [
    (9, (384, 320, 1), 2),
    (19, (72, 64, 48), 2),
    (27, (48, 40, 36), 2),
    (27, (48, 40, 36), 3),
]


@pytest.mark.parametrize("lattice,shape,order", CASES)
def test_16bit_stores_are_rne_images_of_fp32(lattice, shape, order):
    D = 2 if lattice == 9 else 3
    rho, u = _fields(shape, D, seed=lattice * 10 + order)
    f32 = _raw_populations(lattice, shape, "f32", order, rho, u)
    f16 = _raw_populations(lattice, shape, "f16s", order, rho, u)
    bf16 = _raw_populations(lattice, shape, "bf16s", order, rho, u)
    vals = f32.view(np.float32)
    assert np.isfinite(vals).all()
    want16 = vals.astype(np.float16).view(np.uint16)
    bad16 = int((f16 != want16).sum())
    wantb = _bf16_rne(f32)
    badb = int((bf16 != wantb).sum())
    # how many stores were exact ties (the case round-to-nearest-even decides)
    low = f32 & 0xFFFF
    ties_b = int((low == 0x8000).sum())
    e = (f32 >> 23) & 0xFF
    sub16 = int(((np.abs(vals) < 2.0 ** -14) & (vals != 0)).sum())
    normal16 = (e >= 113) & (e <= 142)  # FP16 normal range: drop 13 mantissa bits
    ties_16 = int((normal16 & ((f32 & 0x1FFF) == 0x1000)).sum())
    print(f"D{D}Q{lattice} order {order}: {vals.size} stores, fp16 ties {ties_16}, "
          f"fp16 subnormal results {sub16}, bf16 ties {ties_b}; mismatches fp16 {bad16}, "
          f"bf16 {badb}")
    assert bad16 == 0 and badb == 0
    assert ties_16 > 0 and ties_b > 0 and sub16 > 0
