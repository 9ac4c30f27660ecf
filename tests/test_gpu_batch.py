"""GPU tests of the batched-slices form (maxwell_batch_*): several independent 2D problems of
uneven sizes, Cartesian (variable-density random masks) and radial, with their own dense
bases, coils and sizes, through one call and through one captured graph.

* every slice's loss and gradient against the FP64 oracle (FP32 <= 1e-5, BF16-split <= 1e-4);
* the batch result equal, bit for bit, to the slices' own maxwell_grad calls (same kernels,
  no atomics);
* graph replays: each replay, with eager work between them, equal bit for bit to the eager
  batch call; a replay after the inputs are rewritten in place equals the eager call on the
  new inputs.
"""
import numpy as np
import pytest
import torch

from _common import TOL, assert_close, c64, maxrel, rel
from oracle import Oracle
from synth import slice_problems

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_cache = {}


def T(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(DEV)


def H(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def slices():
    """Six small slices (seeded): sizes 32..64, J 2..4, K 5..12, both sampling kinds."""
    if "p" not in _cache:
        ps = slice_problems(seed=55, n_slices=6, sizes=(32, 48, 64), Js=(2, 3, 4), Ks=(5, 9, 12), spokes=(6, 12))
        data = []
        for p in ps:
            kw = dict(mask_idx=p.mask_idx) if p.sampling == "cartesian" else dict(traj=p.traj.astype(np.float32).astype(np.float64))
            w = None if p.weights is None else p.weights.astype(np.float32).astype(np.float64)
            op = Oracle(p.dims, B=c64(p.B), **kw)
            y = op.encode(c64(p.x_true), c64(p.c_true))
            y = c64(y + 0.05 * np.linalg.norm(y) / np.linalg.norm(p.noise) * p.noise)
            data.append((p, kw, w, op, y))
        _cache["p"] = data
    return _cache["p"]


def plans(prec):
    from paper_2008_09042_amd.encoding import MaxwellPlan
    key = ("plans", prec)
    if key not in _cache:
        _cache[key] = [MaxwellPlan(p.dims, p.J, B=T(p.B), **kw, weights=w, precision=prec, device=DEV)
                       for p, kw, w, op, y in slices()]
    return _cache[key]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
def test_batch_grad_against_oracle_and_single_calls(prec):
    from paper_2008_09042_amd.encoding import MaxwellBatch
    print(f"[case] batch of 6 slices {prec}", flush=True)
    data = slices()
    pl = plans(prec)
    batch = MaxwellBatch(pl, branches=3)
    xs = [T(p.x0) for p, *_ in data]
    cs = [T(p.c0) for p, *_ in data]
    ys = [T(d[4]) for d in data]
    loss, gx, gc = batch.grad(xs, cs, ys)
    torch.cuda.synchronize()
    for i, ((p, kw, w, op, y), plan) in enumerate(zip(data, pl)):
        f_ref, gx_ref, gc_ref = op.loss_and_grad(c64(p.x0), c64(p.c0), y, w)
        errs = (abs(float(loss[i]) - f_ref) / f_ref, rel(H(gx[i]), gx_ref), rel(H(gc[i]), gc_ref),
                maxrel(H(gx[i]), gx_ref), maxrel(H(gc[i]), gc_ref, coils=True))
        print(f"[case] slice {i} {p.dims} J={p.J} K={p.K} {p.sampling}: {errs}", flush=True)
        assert max(errs) <= TOL[prec], (i, errs)
        l1, gx1, gc1 = plan.grad(xs[i], cs[i], ys[i])
        assert torch.equal(l1, loss[i]) and torch.equal(gx1, gx[i]) and torch.equal(gc1, gc[i]), i


def test_batch_graph_replays():
    from paper_2008_09042_amd.encoding import MaxwellBatch
    print("[case] batch graph capture and replays", flush=True)
    data = slices()
    batch = MaxwellBatch(plans("bf16_split"), branches=4)
    xs = [T(p.x0) for p, *_ in data]
    cs = [T(p.c0) for p, *_ in data]
    ys = [T(d[4]) for d in data]
    ref = batch.grad(xs, cs, ys)
    out = batch.capture(xs, cs, ys)
    for k in range(3):
        batch.replay()
        torch.cuda.synchronize()
        for a, b in zip([ref[0]] + ref[1] + ref[2], [out[0]] + out[1] + out[2]):
            assert torch.equal(a, b), f"replay {k}"
        # eager work between replays (the same call outside the graph, and torch's own kernels)
        again = batch.grad(xs, cs, ys)
        assert torch.equal(again[0], ref[0])
        _ = (xs[0] * 2).sum()
    # new input contents, written in place: the replay reads them
    for x, p in zip(xs, (d[0] for d in data)):
        x.copy_(T(p.x_true))
    new_ref = batch.grad(xs, cs, ys)
    batch.replay()
    torch.cuda.synchronize()
    for a, b in zip([new_ref[0]] + new_ref[1] + new_ref[2], [out[0]] + out[1] + out[2]):
        assert torch.equal(a, b)
    assert not torch.equal(new_ref[0], ref[0])


def test_frames_with_shared_coefficients():
    """Dynamic / multi-contrast frames: one plan per frame (own mask), own images, one shared
    coefficient set.  Summed loss, per-frame gx and summed gc against the oracle, and equal
    bit for bit to the frames' own maxwell_grad calls summed in frame order."""
    from paper_2008_09042_amd.encoding import MaxwellBatch, MaxwellPlan
    from _common import Case
    print("[case] 3 frames sharing coefficients", flush=True)
    frames = [Case(seed=61 + t, dims=(48, 40), J=4, K=9, basis="dense", frac=0.3, weights=True) for t in range(3)]
    B = frames[0].B
    for f in frames[1:]:  # one basis for all frames; each frame keeps its own mask, image, data
        f.B = B
        f.op = Oracle(f.dims, B=B, mask_idx=f.mask)
    c = frames[0].c0
    plans = [MaxwellPlan(f.dims, f.J, B=T(B), mask_idx=f.mask, weights=f.w, precision="fp32", device=DEV)
             for f in frames]
    batch = MaxwellBatch(plans, branches=2)
    xs = [T(f.x0) for f in frames]
    ys = [T(f.y) for f in frames]
    loss, gx, gc = batch.grad_shared(xs, T(c), ys)
    torch.cuda.synchronize()
    f_ref, gc_ref, gx_ref = 0.0, 0.0, []
    for f in frames:
        fr, gxr, gcr = f.op.loss_and_grad(f.x0, c, f.y, f.w)
        f_ref += fr
        gc_ref = gc_ref + gcr
        gx_ref.append(gxr)
    assert abs(float(loss.item()) - f_ref) / f_ref <= TOL["fp32"]
    assert_close(H(gc), gc_ref, TOL["fp32"], coils=True, what="gc")
    for t in range(3):
        assert_close(H(gx[t]), gx_ref[t], TOL["fp32"], what=f"gx[{t}]")
    singles = [p.grad(x, T(c), y) for p, x, y in zip(plans, xs, ys)]
    s = singles[0][2] + singles[1][2] + singles[2][2]
    assert torch.equal(gc, s)
    assert float(loss.item()) == float(singles[0][0].item()) + float(singles[1][0].item()) + float(singles[2][0].item())



@pytest.mark.parametrize("staged", [True, False])
def test_batch_modes_and_device_stamps(staged):
    """Both issue orders (rounds with the FFT passes of several slices per launch, and whole
    chains per branch) give every slice's own maxwell_grad bit for bit; the device stamps of
    each slice (first step start, last step end) are written by eager calls and by graph
    replays."""
    from paper_2008_09042_amd.encoding import MaxwellBatch
    print(f"[case] batch staged={staged} with stamps", flush=True)
    data = slices()
    pl = plans("fp32")
    batch = MaxwellBatch(pl, branches=2, staged=staged, stamps=True)
    assert batch.ticks_per_second > 0
    xs = [T(p.x0) for p, *_ in data]
    cs = [T(p.c0) for p, *_ in data]
    ys = [T(d[4]) for d in data]
    loss, gx, gc = batch.grad(xs, cs, ys)
    torch.cuda.synchronize()
    lat = batch.latencies_ms()
    assert np.all(np.isfinite(lat)) and np.all(lat > 0) and np.all(lat < 1e4), lat
    for i, plan in enumerate(pl):
        l1, gx1, gc1 = plan.grad(xs[i], cs[i], ys[i])
        assert torch.equal(l1, loss[i]) and torch.equal(gx1, gx[i]) and torch.equal(gc1, gc[i]), i
    out = batch.capture(xs, cs, ys)
    batch.stamps.zero_()
    torch.cuda.synchronize()
    batch.replay()
    torch.cuda.synchronize()
    lat = batch.latencies_ms()
    assert np.all(lat > 0), lat
    for a, b in zip([loss] + gx + gc, [out[0]] + out[1] + out[2]):
        assert torch.equal(a, b)
