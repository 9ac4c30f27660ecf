"""maxwell_grad_static (the entry point that allocates nothing: its workspace is a
library-held device buffer) against maxwell_grad with a caller workspace, through the C ABI:
two calls in a row on one device, the second with a smaller plan, each bit for bit equal to
maxwell_grad on the same inputs (same kernels, fixed-order reductions) and within the parity
bar of the FP64 oracle; plans whose workspace exceeds the buffer, and plans with per-kernel
timing on, are refused."""
import ctypes

import numpy as np
import pytest
import torch

from _common import TOL, Case, assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def T(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(DEV)


def H(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def p(t):
    return ctypes.c_void_p(t.data_ptr())


def grad_static(plan, x, c, y):
    from paper_2008_09042_amd import _lib as L
    lib = L.load()
    gx = torch.empty_like(x)
    gc = torch.empty_like(c)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)
    L.check(lib.maxwell_grad_static(plan.handle, p(x), p(c), p(y), p(gx), p(gc), p(loss),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return loss, gx, gc


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
def test_static_workspace_matches_caller_workspace(prec):
    print(f"[case] grad_static two calls {prec}", flush=True)
    cases = [Case(seed=401, dims=(64, 64), J=8, K=32, weights=True),        # first call
             Case(seed=402, dims=(30, 20), J=3, K=9, mask="radial", spokes=7, weights=True)]  # smaller
    plans = [cs.plan(prec) for cs in cases]
    assert plans[1].ws_bytes < plans[0].ws_bytes
    outs = []
    for cs, plan in zip(cases, plans):
        x, c, y = T(cs.x0), T(cs.c0), T(cs.y)
        outs.append((grad_static(plan, x, c, y), plan.grad(x, c, y), cs))
    torch.cuda.synchronize()
    for (ls, gxs, gcs), (l1, gx1, gc1), cs in outs:
        assert torch.equal(ls, l1.reshape(1)) and torch.equal(gxs, gx1) and torch.equal(gcs, gc1)
        f_ref, gx_ref, gc_ref = cs.op.loss_and_grad(cs.x0, cs.c0, cs.y, cs.w)
        assert abs(float(ls.item()) - f_ref) / f_ref <= TOL[prec]
        assert_close(H(gxs), gx_ref, TOL[prec], what="gx")
        assert_close(H(gcs), gc_ref, TOL[prec], coils=True, what="gc")


def test_static_workspace_refusals():
    from paper_2008_09042_amd import _lib as L
    from paper_2008_09042_amd.encoding import MaxwellPlan
    print("[case] grad_static refusals", flush=True)
    dims, J, K = (128, 128, 128), 16, 2
    N = int(np.prod(dims))
    rng = np.random.default_rng(3)
    B = torch.zeros((N, K), dtype=torch.complex64, device=DEV)
    B[:, 0] = 1.0 / np.sqrt(N)
    mask = np.sort(rng.choice(N, size=N // 8, replace=False))
    big = MaxwellPlan(dims, J, B=B, mask_idx=mask, precision="fp32", device=DEV)
    assert big.ws_bytes > L.MAXWELL_STATIC_WS_BYTES
    x = torch.zeros(dims, dtype=torch.complex64, device=DEV)
    c = torch.zeros((J, K), dtype=torch.complex64, device=DEV)
    y = torch.zeros((J, mask.size), dtype=torch.complex64, device=DEV)
    with pytest.raises(L.MaxwellError) as ei:
        grad_static(big, x, c, y)
    assert ei.value.status == L.MAXWELL_ERR_WORKSPACE_TOO_SMALL
    cs = Case(seed=403, dims=(32, 24), J=2, K=5)
    small = cs.plan("fp32")
    small.set_timing(True)
    with pytest.raises(L.MaxwellError) as ei:
        grad_static(small, T(cs.x0), T(cs.c0), T(cs.y))
    assert ei.value.status == L.MAXWELL_ERR_UNSUPPORTED
    small.set_timing(False)
    torch.cuda.synchronize()
