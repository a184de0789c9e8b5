"""The integration kernel's reciprocal-based projection quotient against the compiler's
correctly rounded division, on the device, bit for bit: 2^28 random operand pairs over the
admitted range, and every dividend significand (64 times, at random exponents) against
divisors with an all-ones significand (the case where one Newton step from an estimate one
ulp off falls short), so the hardware reciprocal is covered where the host check cannot
model it."""
import pytest
import torch

from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("all_ones,n", [(0, 1 << 28), (1, 1 << 29)])
def test_projection_quotient_matches_division(all_ones, n):
    vbh = require_gpu()
    say(f"[fastdiv] all_ones={all_ones} n={n}")
    bad = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    vbh.binding.vbh_check_division(n, 1805 + all_ones, all_ones, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0


def test_check_division_rejects_bad_arguments():
    vbh = require_gpu()
    bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    for args in ((-1, 0, 0), (10, 0, 2)):
        with pytest.raises(vbh.binding.VbhError):
            vbh.binding.vbh_check_division(*args, bad)
