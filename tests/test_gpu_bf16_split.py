"""BF16 split of the BF16-split products, value by value (the split itself, not its effect).

The device split hi = bf16(a), lo = bf16(a - hi) (round to nearest even) of every variant
(the hardware converts of the plane kernels, the GEMM operand split, the core split) must
equal, bit for bit, the host rule: torch's CPU float32 -> bfloat16 conversion, which rounds
to nearest even (pinned against hand-derived bit patterns in test_bf16_rule.py); a - hi is
exact in FP32.  And hi + lo represents a to <= 2^-16 relative (the bound of the split: the
residual of two 8-bit-significand roundings, at most 2^-9 * 2^-9 of |a|, well inside it).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def host_split(x: torch.Tensor):
    hi = x.to(torch.bfloat16)
    lo = (x - hi.to(torch.float32)).to(torch.bfloat16)
    return hi.view(torch.int16), lo.view(torch.int16)


def values():
    rng = np.random.default_rng(2008)
    n = 1 << 16
    mag = 10.0 ** rng.uniform(-30, 30, size=n)
    x = (rng.standard_normal(n) * mag).astype(np.float32)
    # round-half-even ties and their neighbours at several binades, signed
    base = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -9,
                     1.9999999, 0.75 + 2.0 ** -10, 3.0, 0.0], dtype=np.float64)
    ties = np.concatenate([s * base * 2.0 ** e for e in (-40, -3, 0, 7, 60) for s in (1.0, -1.0)])
    x = np.concatenate([x, ties.astype(np.float32)])
    x = x[: (x.size // 8) * 8 + 6]  # a ragged tail for the 8-wide split (even: complex pairs)
    return torch.from_numpy(x)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_device_split_matches_round_to_nearest_even(variant):
    from paper_2008_09042_amd.encoding import bf16_split
    print(f"[case] bf16 split variant {variant}", flush=True)
    x = values()
    hi, lo = bf16_split(x.to(DEV), variant)
    torch.cuda.synchronize()
    hi, lo = hi.cpu(), lo.cpu()
    rhi, rlo = host_split(x)
    assert torch.equal(hi, rhi), int((hi != rhi).sum())
    assert torch.equal(lo, rlo), int((lo != rlo).sum())
    a = x.double()
    rep = hi.view(torch.bfloat16).double() + lo.view(torch.bfloat16).double()
    nz = a != 0
    err = ((rep - a).abs()[nz] / a.abs()[nz]).max().item()
    assert err <= 2.0 ** -16, err
    assert torch.all(rep[~nz] == 0)


def test_split_empty_and_refusals():
    from paper_2008_09042_amd import _lib as L
    from paper_2008_09042_amd.encoding import bf16_split
    hi, lo = bf16_split(torch.zeros(0, device=DEV), 0)
    assert hi.numel() == 0
    with pytest.raises(L.MaxwellError):
        bf16_split(torch.zeros(7, device=DEV), 1)  # complex pairs: n must be even
    with pytest.raises(L.MaxwellError):
        bf16_split(torch.zeros(8, device=DEV), 3)
