"""The host rounding rule that the device BF16 split is checked against (test_gpu_bf16_split):
torch's CPU float32 -> bfloat16 conversion rounds to nearest, ties to even.  Pinned against
bit patterns worked out by hand from the formats (bf16 keeps the sign, the 8 exponent bits
and the top 7 fraction bits of a float32)."""
import torch


def bits(v):
    return int(torch.tensor([v], dtype=torch.float32).to(torch.bfloat16).view(torch.int16).item()) & 0xFFFF


def test_round_to_nearest_even_fixtures():
    assert bits(1.0) == 0x3F80
    assert bits(1.0 + 2.0 ** -7) == 0x3F81            # representable: 1 + one bf16 ulp
    assert bits(1.0 + 2.0 ** -8) == 0x3F80            # tie between 0x3F80 and 0x3F81 -> even
    assert bits(1.0 + 3 * 2.0 ** -8) == 0x3F82        # tie between 0x3F81 and 0x3F82 -> even
    assert bits(1.0 + 2.0 ** -8 + 2.0 ** -20) == 0x3F81  # just above the tie -> up
    assert bits(-1.0 - 3 * 2.0 ** -8) == 0xBF82
    assert bits(0.0) == 0x0000
    assert bits(3.0) == 0x4040


def test_split_residual_is_exact_in_fp32():
    x = torch.tensor([1.0 + 2.0 ** -8 + 2.0 ** -20, 3.14159265, -2.0e-30, 6.0e30])
    hi = x.to(torch.bfloat16).to(torch.float32)
    assert torch.equal((x - hi).double(), x.double() - hi.double())
