"""The short division of the post-collision coefficients equals the IEEE one.

The coefficient prescaling divides by the odd parts 3, 9, 27 of the lattice
weight denominators.  The instruction-bound kernels (the fused step, D3Q27
with 16-bit storage) use a rounded reciprocal plus one correction with the
exact FMA residual instead of the IEEE division; the fused step's results
are compared byte for byte with the two sweeps', which use the IEEE
division, so the two must agree on every input.  lb_check_division runs both
on all 2^32 FP32 bit patterns (finite ones) for each divisor.
"""
import pytest

from paper_2304_06437_amd import lb

pytestmark = pytest.mark.gpu


def test_short_division_equals_ieee_on_every_fp32_input():
    import torch

    mism = lb.lb_check_division(torch.cuda.current_stream().cuda_stream)
    print("mismatches for divisors 3, 9, 27:", mism)
    assert mism == (0, 0, 0)
