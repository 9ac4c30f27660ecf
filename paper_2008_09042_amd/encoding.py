"""Python binding of libmaxwell: a plan object and two autograd Functions.

PyTorch supplies device memory and the current stream; every step of the
operator runs in the library's HIP kernels.  There is no fallback: if
libmaxwell.so is missing or no GPU is present, construction raises.

    plan = MaxwellPlan(dims, J, B=B, mask_idx=mask, precision="bf16_split")
    y = MaxwellEncode.apply(x, c, plan)                 # E(x, c), backward = J^H
    f = MaxwellDataFidelity.apply(x, c, y_meas, plan)   # sum w |E - y|^2, backward = 2 J^H (w r)

Paper: Sec. II-B, Eq. (5) (operator), the J_G^H expression (adjoint) and
Eq. (6) (data term).
"""
import ctypes
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_PRECISIONS = {"fp32": L.MAXWELL_FP32, "bf16_split": L.MAXWELL_BF16_SPLIT}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class MaxwellPlan:
    """One operator geometry on one GPU.

    dims      image shape (2 or 3 axes, C-order)
    J         number of coils
    B         dense basis (N, K) (numpy or torch, converted to complex64 on the device)
    U, core   Tucker factors [(n_m, r_m)] and core (r0, r1, r2, K) instead of B
    mask_idx  sorted unique int64 linear indices into the centred k-space grid (Cartesian)
    traj      (M, 2) trajectory in cycles/FOV (non-Cartesian, 2D)
    weights   optional (M,) data weights for the loss and its gradient
    precision "fp32" or "bf16_split" for the basis contractions
    """

    def __init__(self, dims: Sequence[int], J: int, *, B=None, U=None, core=None, mask_idx=None, traj=None,
                 weights=None, precision: str = "fp32", kb_width: int = 6, oversamp: float = 2.0,
                 kb_beta: float = 0.0, device="cuda:0"):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("MaxwellPlan needs a ROCm GPU; none is visible")
        self.device = torch.device(device)
        self.dims = tuple(int(n) for n in dims)
        self.ndim = len(self.dims)
        self.N = int(np.prod(self.dims))
        self.J = int(J)
        self.precision = precision
        dev = self.device

        def dtensor(a):
            t = torch.as_tensor(a)
            return t.to(device=dev, dtype=torch.complex64).contiguous()

        bd = L.BasisDesc()
        if B is not None:
            self.B = dtensor(B)
            if self.B.ndim != 2 or self.B.shape[0] != self.N:
                raise ValueError("B must be (N, K)")
            self.K = int(self.B.shape[1])
            bd.kind = L.MAXWELL_BASIS_DENSE
            bd.dense = self.B.data_ptr()
            self._basis_refs = [self.B]
        else:
            self.U = [dtensor(u) for u in U]
            self.core = dtensor(core)
            self.K = int(self.core.shape[-1])
            bd.kind = L.MAXWELL_BASIS_TUCKER
            for m in range(3):
                bd.r[m] = int(self.U[m].shape[1])
                bd.U[m] = self.U[m].data_ptr()
            bd.core = self.core.data_ptr()
            self._basis_refs = self.U + [self.core]
        bd.K = self.K

        pd = L.PlanDesc()
        pd.ndim = self.ndim
        for d in range(self.ndim):
            pd.n[d] = self.dims[d]
        pd.J = self.J
        pd.precision = _PRECISIONS[precision]
        keep = []
        if traj is None:
            mask = np.ascontiguousarray(np.asarray(mask_idx, dtype=np.int64))
            keep.append(mask)
            pd.sampling = L.MAXWELL_CARTESIAN
            pd.M = mask.size
            pd.mask_idx = mask.ctypes.data
        else:
            tr = np.ascontiguousarray(np.asarray(traj, dtype=np.float32))
            keep.append(tr)
            pd.sampling = L.MAXWELL_NONCARTESIAN
            pd.M = tr.shape[0]
            pd.traj = tr.ctypes.data
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
            keep.append(w)
            pd.weights = w.ctypes.data
        pd.kb_width = kb_width
        pd.oversamp = oversamp
        pd.kb_beta = kb_beta
        self.M = int(pd.M)
        self.has_weights = weights is not None

        handle = ctypes.c_void_p()
        with torch.cuda.device(dev):
            L.check(self.lib.maxwell_plan_create(ctypes.byref(pd), ctypes.byref(bd), ctypes.byref(handle)))
        self.handle = handle
        nbytes = ctypes.c_size_t()
        L.check(self.lib.maxwell_plan_workspace_size(self.handle, ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.path = self.lib.maxwell_plan_path(self.handle).decode()
        raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + self.ws_bytes] if self.ws_bytes else raw[:0]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.lib.maxwell_plan_destroy(h)
            self.handle = None

    # ---- per-kernel timing (HIP events on the launch stream)
    def set_timing(self, enable: bool):
        L.check(self.lib.maxwell_plan_set_timing(self.handle, 1 if enable else 0))

    def timing(self):
        """{kernel name: (launches, total ms)} recorded since set_timing(True)."""
        n = ctypes.c_int()
        L.check(self.lib.maxwell_plan_timing(self.handle, 0, ctypes.byref(n), None, None, None))
        out = {}
        for i in range(n.value):
            name = ctypes.c_char_p()
            cnt = ctypes.c_int64()
            ms = ctypes.c_double()
            L.check(self.lib.maxwell_plan_timing(self.handle, i, None, ctypes.byref(name), ctypes.byref(cnt),
                                                 ctypes.byref(ms)))
            out[name.value.decode()] = (int(cnt.value), float(ms.value))
        return out

    # ---- argument checks (shape / dtype / device / contiguity)
    def _in(self, t: torch.Tensor, shape, name):
        """A complex64 input on the plan's device of exactly `shape`, or a flat view of it
        (1-D with the same number of elements); any other shape is refused (a transposed
        image would otherwise be read in the wrong order)."""
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.complex64 or t.device != self.device:
            raise ValueError(f"{name} must be complex64 on {self.device}")
        shape = tuple(int(v) for v in shape)
        if tuple(t.shape) != shape and not (t.dim() == 1 and t.numel() == int(np.prod(shape))):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape} (or a flat view)")
        return t.contiguous()

    def bf16_split(self, x: torch.Tensor, variant: int = 0):
        """Diagnostic: the device BF16 split of float32 values x -> (hi, lo) as int16 bit
        patterns (maxwell_bf16_split)."""
        return bf16_split(x, variant)

    def _new(self, shape):
        return torch.empty(shape, dtype=torch.complex64, device=self.device)

    def _wsargs(self):
        return ctypes.c_void_p(self.ws.data_ptr()) if self.ws_bytes else None, self.ws_bytes

    # ---- the C-ABI calls
    def basis_apply(self, c):
        c = self._in(c, (self.J, self.K), "c")
        S = self._new((self.J, self.N))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_basis_apply(self.handle, _ptr(c), _ptr(S), ws, nb, _stream()))
        return S

    def basis_adjoint(self, S):
        S = self._in(S, (self.J, self.N), "S")
        c = self._new((self.J, self.K))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_basis_apply_adjoint(self.handle, _ptr(S), _ptr(c), ws, nb, _stream()))
        return c

    def encode(self, x, c):
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        y = self._new((self.J, self.M))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_encode(self.handle, _ptr(x), _ptr(c), _ptr(y), ws, nb, _stream()))
        return y

    def adjoint(self, x, c, y, alpha: float = 1.0, scale: Optional[torch.Tensor] = None,
                want_gx: bool = True, want_gc: bool = True):
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        y = self._in(y, (self.J, self.M), "y")
        if scale is not None:
            if scale.dtype != torch.float32 or scale.device != self.device or scale.numel() != 1:
                raise ValueError("scale must be one float32 on the plan device")
            scale = scale.contiguous()
        gx = self._new(self.dims) if want_gx else None
        gc = self._new((self.J, self.K)) if want_gc else None
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_adjoint(self.handle, _ptr(x), _ptr(c), _ptr(y), ctypes.c_float(alpha),
                                         _ptr(scale), _ptr(gx), _ptr(gc), ws, nb, _stream()))
        return gx, gc

    def forward_loss(self, x, c, y, want_r: bool = True):
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        y = self._in(y, (self.J, self.M), "y")
        r = self._new((self.J, self.M)) if want_r else None
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_forward_loss(self.handle, _ptr(x), _ptr(c), _ptr(y), _ptr(r), _ptr(loss),
                                              ws, nb, _stream()))
        return r, loss

    def forward_transfer(self, x, c, y):
        """Loss and the weighted residual in the plan's transfer layout (maxwell_forward_transfer)."""
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        y = self._in(y, (self.J, self.M), "y")
        t = self._new((self.J, self.M))
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_forward_transfer(self.handle, _ptr(x), _ptr(c), _ptr(y), _ptr(t), _ptr(loss),
                                                  ws, nb, _stream()))
        return t, loss

    def adjoint_transfer(self, x, c, t, alpha: float = 1.0, scale: Optional[torch.Tensor] = None,
                         want_gx: bool = True, want_gc: bool = True):
        """maxwell_adjoint_transfer: the adjoint on a residual from forward_transfer."""
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        t = self._in(t, (self.J, self.M), "t")
        if scale is not None:
            if scale.dtype != torch.float32 or scale.device != self.device or scale.numel() != 1:
                raise ValueError("scale must be one float32 on the plan device")
            scale = scale.contiguous()
        gx = self._new(self.dims) if want_gx else None
        gc = self._new((self.J, self.K)) if want_gc else None
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_adjoint_transfer(self.handle, _ptr(x), _ptr(c), _ptr(t), ctypes.c_float(alpha),
                                                  _ptr(scale), _ptr(gx), _ptr(gc), ws, nb, _stream()))
        return gx, gc

    def grad(self, x, c, y):
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        y = self._in(y, (self.J, self.M), "y")
        gx = self._new(self.dims)
        gc = self._new((self.J, self.K))
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_grad(self.handle, _ptr(x), _ptr(c), _ptr(y), _ptr(gx), _ptr(gc), _ptr(loss),
                                      ws, nb, _stream()))
        return loss, gx, gc

    # ---- Gauss-Newton step (Sec. II-B, Eq. (6) and Eq. (7))
    def jvp(self, x, c, dx, dc):
        """J[dx, dc] at (x, c): F_s((B c_j) dx + x (B dc_j)) -> [J][M]."""
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        dx = self._in(dx, self.dims, "dx")
        dc = self._in(dc, (self.J, self.K), "dc")
        y = self._new((self.J, self.M))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_jvp(self.handle, _ptr(x), _ptr(c), _ptr(dx), _ptr(dc), _ptr(y), ws, nb, _stream()))
        return y

    def normal(self, x, c, dx, dc, lambda_x: float, lambda_c: float):
        """J^H (w J[dx, dc]) + (lambda_x dx, lambda_c dc) at (x, c)."""
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        dx = self._in(dx, self.dims, "dx")
        dc = self._in(dc, (self.J, self.K), "dc")
        ox = self._new(self.dims)
        oc = self._new((self.J, self.K))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_normal(self.handle, _ptr(x), _ptr(c), _ptr(dx), _ptr(dc), float(lambda_x),
                                        float(lambda_c), _ptr(ox), _ptr(oc), ws, nb, _stream()))
        return ox, oc

    def cg(self, x, c, bx, bc, lambda_x: float, lambda_c: float, iters: int):
        """iters CG steps from zero on normal(dv) = b -> (dx, dc, rr) with rr[k] = <r_k, r_k> (FP64)."""
        x = self._in(x, self.dims, "x")
        c = self._in(c, (self.J, self.K), "c")
        bx = self._in(bx, self.dims, "bx")
        bc = self._in(bc, (self.J, self.K), "bc")
        dx = self._new(self.dims)
        dc = self._new((self.J, self.K))
        rr = torch.empty(int(iters) + 1, dtype=torch.float64, device=self.device)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_cg(self.handle, _ptr(x), _ptr(c), _ptr(bx), _ptr(bc), float(lambda_x),
                                    float(lambda_c), int(iters), _ptr(dx), _ptr(dc), _ptr(rr), ws, nb, _stream()))
        return dx, dc, rr

    # ---- extra bilinear terms (multi-map)
    def multi_encode(self, xs, cs):
        """sum_i E(x_i, c_i); xs: [n, *dims], cs: [n, J, K]."""
        n = int(xs.shape[0])
        xs = self._in(xs, (n,) + tuple(self.dims), "xs")
        cs = self._in(cs, (n, self.J, self.K), "cs")
        y = self._new((self.J, self.M))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_multi_encode(self.handle, n, _ptr(xs), _ptr(cs), _ptr(y), ws, nb, _stream()))
        return y

    def multi_grad(self, xs, cs, y):
        """(loss, gxs [n, *dims], gcs [n, J, K]) of sum w |sum_i E(x_i, c_i) - y|^2."""
        n = int(xs.shape[0])
        xs = self._in(xs, (n,) + tuple(self.dims), "xs")
        cs = self._in(cs, (n, self.J, self.K), "cs")
        y = self._in(y, (self.J, self.M), "y")
        gx = self._new((n,) + tuple(self.dims))
        gc = self._new((n, self.J, self.K))
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_multi_grad(self.handle, n, _ptr(xs), _ptr(cs), _ptr(y), _ptr(gx), _ptr(gc),
                                            _ptr(loss), ws, nb, _stream()))
        return loss, gx, gc

    # ---- SENSE with fixed maps and the constrained reconstruction (Sec. II-C; general path)
    def sense_encode(self, S, x):
        S = self._in(S, (self.J, self.N), "S")
        x = self._in(x, self.dims, "x")
        y = self._new((self.J, self.M))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_sense_encode(self.handle, _ptr(S), _ptr(x), _ptr(y), ws, nb, _stream()))
        return y

    def sense_adjoint(self, S, y):
        S = self._in(S, (self.J, self.N), "S")
        y = self._in(y, (self.J, self.M), "y")
        gx = self._new(self.dims)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_sense_adjoint(self.handle, _ptr(S), _ptr(y), _ptr(gx), ws, nb, _stream()))
        return gx

    def sense_normal(self, S, x):
        S = self._in(S, (self.J, self.N), "S")
        x = self._in(x, self.dims, "x")
        out = self._new(self.dims)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_sense_normal(self.handle, _ptr(S), _ptr(x), _ptr(out), ws, nb, _stream()))
        return out

    def tv_prox(self, z, lam: float, iters: int):
        z = self._in(z, self.dims, "z")
        x = self._new(self.dims)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_tv_prox(self.handle, _ptr(z), float(lam), int(iters), _ptr(x), ws, nb, _stream()))
        return x

    def ball_project(self, w, y, eps):
        w = self._in(w, (self.J, self.M), "w")
        y = self._in(y, (self.J, self.M), "y")
        eps = torch.as_tensor(eps, dtype=torch.float32, device=self.device).contiguous()
        z = self._new((self.J, self.M))
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_ball_project(self.handle, _ptr(w), _ptr(y), _ptr(eps), _ptr(z), ws, nb, _stream()))
        return z

    def sense_admm(self, S, y, eps, rho0: float, iters: int, cg_iters: int, tv_iters: int):
        """-> (p, hist) with hist[k] = (rho, primal residual, dual residual) (FP64)."""
        S = self._in(S, (self.J, self.N), "S")
        y = self._in(y, (self.J, self.M), "y")
        eps = torch.as_tensor(eps, dtype=torch.float32, device=self.device).contiguous()
        p = self._new(self.dims)
        hist = torch.empty((int(iters), 3), dtype=torch.float64, device=self.device)
        ws, nb = self._wsargs()
        L.check(self.lib.maxwell_sense_admm(self.handle, _ptr(S), _ptr(y), _ptr(eps), float(rho0), int(iters),
                                            int(cg_iters), int(tv_iters), _ptr(p), _ptr(hist), ws, nb, _stream()))
        return p, hist


class MaxwellBatch:
    """Gradients of many independent slices (each a MaxwellPlan) in one call.

    grad(xs, cs, ys) runs maxwell_batch_grad eagerly.  capture(xs, cs, ys) records that
    call into one CUDA/HIP graph on fixed buffers (the tensors passed in, whose contents the
    caller may update in place, and outputs owned here); replay() launches the graph and
    returns the same output tensors each time.  staged=True issues the slices' steps in
    phases (each phase's FFT passes of all slices launched together); staged=False runs
    each slice's whole chain on one of `branches` concurrent branches.  stamps=True makes
    every call write each slice's device timestamps (first step start, last step end);
    latencies_ms() reads them after the call (or replay) has completed."""

    def __init__(self, plans, branches: int = 4, staged: bool = True, stamps: bool = False):
        self.plans = list(plans)
        if not self.plans:
            raise ValueError("a batch needs at least one plan")
        self.device = self.plans[0].device
        if any(p.device != self.device for p in self.plans):
            raise ValueError("all plans of a batch must be on one device")
        self.lib = self.plans[0].lib
        n = len(self.plans)
        arr = (ctypes.c_void_p * n)(*[p.handle.value for p in self.plans])
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.maxwell_batch_create(arr, n, branches, ctypes.byref(handle)))
        self.handle = handle
        nbytes = ctypes.c_size_t()
        L.check(self.lib.maxwell_batch_workspace_size(self.handle, ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + self.ws_bytes]
        self.graph = None
        self.stamps = torch.zeros(2 * n, dtype=torch.int64, device=self.device) if stamps else None
        rate = ctypes.c_double()
        with torch.cuda.device(self.device):
            L.check(self.lib.maxwell_batch_set_options(self.handle, int(bool(staged)),
                                                       _ptr(self.stamps) if stamps else None, ctypes.byref(rate)))
        self.ticks_per_second = float(rate.value)

    def latencies_ms(self):
        """Per-slice latency inside the last completed batch call (device timestamps), ms."""
        if self.stamps is None:
            raise RuntimeError("the batch was created without stamps")
        t = self.stamps.cpu().numpy().reshape(-1, 2)
        return (t[:, 1] - t[:, 0]).astype(np.float64) * 1e3 / self.ticks_per_second

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.lib.maxwell_batch_destroy(h)
            self.handle = None

    def _outputs(self):
        gx = [p._new(p.dims) for p in self.plans]
        gc = [p._new((p.J, p.K)) for p in self.plans]
        loss = torch.zeros(len(self.plans), dtype=torch.float64, device=self.device)
        return loss, gx, gc

    def _call(self, xs, cs, ys, loss, gx, gc):
        n = len(self.plans)
        P = ctypes.c_void_p * n
        ptrs = lambda ts: P(*[t.data_ptr() for t in ts])  # noqa: E731
        lp = P(*[loss.data_ptr() + 8 * i for i in range(n)])
        L.check(self.lib.maxwell_batch_grad(self.handle, ptrs(xs), ptrs(cs), ptrs(ys), ptrs(gx), ptrs(gc), lp,
                                            ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, _stream()))

    def _inputs(self, xs, cs, ys):
        if not (len(xs) == len(cs) == len(ys) == len(self.plans)):
            raise ValueError("xs, cs and ys need one tensor per slice")
        xs = [p._in(x, p.dims, "x") for p, x in zip(self.plans, xs)]
        cs = [p._in(c, (p.J, p.K), "c") for p, c in zip(self.plans, cs)]
        ys = [p._in(y, (p.J, p.M), "y") for p, y in zip(self.plans, ys)]
        return xs, cs, ys

    def grad(self, xs, cs, ys):
        """(loss [n] FP64, [gx_i], [gc_i]) for every slice, as MaxwellPlan.grad."""
        xs, cs, ys = self._inputs(xs, cs, ys)
        loss, gx, gc = self._outputs()
        self._call(xs, cs, ys, loss, gx, gc)
        return loss, gx, gc

    def grad_shared(self, xs, c, ys):
        """Frames sharing one coefficient set c: (summed loss FP64, [gx_t], gc summed over the
        frames in frame order) via maxwell_batch_grad_shared."""
        xs, cs, ys = self._inputs(xs, [c] * len(self.plans), ys)
        c = cs[0]
        p0 = self.plans[0]
        gx = [p._new(p.dims) for p in self.plans]
        gc = p0._new((p0.J, p0.K))
        loss = torch.zeros((), dtype=torch.float64, device=self.device)
        n = len(self.plans)
        P = ctypes.c_void_p * n
        ptrs = lambda ts: P(*[t.data_ptr() for t in ts])  # noqa: E731
        L.check(self.lib.maxwell_batch_grad_shared(self.handle, ptrs(xs), _ptr(c), ptrs(ys), ptrs(gx), _ptr(gc),
                                                   _ptr(loss), ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                                   _stream()))
        return loss, gx, gc

    def capture(self, xs, cs, ys):
        """Record the batch gradient on these buffers into one graph."""
        given = list(xs) + list(cs) + list(ys)
        xs, cs, ys = self._inputs(xs, cs, ys)
        if any(t.data_ptr() != g.data_ptr() for t, g in zip(xs + cs + ys, given)):
            raise ValueError("capture needs contiguous complex64 inputs (the graph reads them in place)")
        self._bound = (xs, cs, ys)
        self._out = self._outputs()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):  # warm-up outside the capture
            self._call(xs, cs, ys, *self._out)
        torch.cuda.current_stream(self.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._call(xs, cs, ys, *self._out)
        return self._out

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        return self._out


def _like(g: Optional[torch.Tensor], t: torch.Tensor):
    """A gradient in the shape of its input (the input may be a flat view)."""
    return None if g is None else g.reshape(t.shape)


def tune_counts():
    """(choices timed, choices reused) by plan creation in this process (maxwell_tune_counts)."""
    lib = L.load()
    m, r = ctypes.c_int64(), ctypes.c_int64()
    L.check(lib.maxwell_tune_counts(ctypes.byref(m), ctypes.byref(r)))
    return int(m.value), int(r.value)


def bf16_split(x: torch.Tensor, variant: int = 0):
    """The device BF16 split (maxwell_bf16_split) of a float32 tensor on a GPU:
    hi = bf16(x), lo = bf16(x - hi) as int16 tensors holding the bit patterns."""
    lib = L.load()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float32 or x.device.type != "cuda":
        raise ValueError("x must be a float32 tensor on a GPU")
    x = x.contiguous().reshape(-1)
    hi = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    lo = torch.empty_like(hi)
    with torch.cuda.device(x.device):
        L.check(lib.maxwell_bf16_split(_ptr(x), x.numel(), int(variant), _ptr(hi), _ptr(lo), _stream()))
    return hi, lo


class MaxwellEncode(torch.autograd.Function):
    """y = E(x, c); backward applies the Jacobian adjoint J^H to the incoming gradient.

    E is complex-linear in each argument, so in PyTorch's convention the
    vector-Jacobian product is exactly (J_x^H gy, J_c^H gy).  B c is
    recomputed inside the adjoint call; no per-coil maps are stored."""

    @staticmethod
    def forward(ctx, x, c, plan):
        ctx.plan = plan
        ctx.save_for_backward(x, c)
        return plan.encode(x, c)

    @staticmethod
    def backward(ctx, gy):
        x, c = ctx.saved_tensors
        gx, gc = ctx.plan.adjoint(x, c, gy.contiguous(), want_gx=ctx.needs_input_grad[0],
                                  want_gc=ctx.needs_input_grad[1])
        return _like(gx, x), _like(gc, c), None


class MaxwellDataFidelity(torch.autograd.Function):
    """f = sum_j sum_m w_m |E(x, c)_jm - y_jm|^2 (FP64 scalar).

    When a gradient is wanted, forward keeps the weighted residual r = w (.) (E - y)
    ([J][M]) in the plan's transfer layout (on the fused 3D path already taken back
    along the readout, the adjoint's first step); backward runs the adjoint at (x, c)
    on it with scale 2 * grad_output (read on the device), recomputing B c.  Without
    a wanted gradient, forward computes the loss alone."""

    @staticmethod
    def forward(ctx, x, c, y, plan):
        ctx.plan = plan
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            t, loss = plan.forward_transfer(x, c, y)
            ctx.save_for_backward(x, c, t)
        else:
            _, loss = plan.forward_loss(x, c, y, want_r=False)
        return loss

    @staticmethod
    def backward(ctx, gloss):
        x, c, t = ctx.saved_tensors
        scale = gloss.detach().to(torch.float32).reshape(1)
        gx, gc = ctx.plan.adjoint_transfer(x, c, t, alpha=2.0, scale=scale, want_gx=ctx.needs_input_grad[0],
                                           want_gc=ctx.needs_input_grad[1])
        return _like(gx, x), _like(gc, c), None, None


def tucker_compress(B: torch.Tensor, dims, eps: float):
    """Accuracy-controlled Tucker form of a dense basis B [N, K] (complex64, on a GPU):
    -> ([U0, U1, U2] with U_m [n_m, r_m], core [r0, r1, r2, K], ranks, dropped squared norms)."""
    lib = L.load()
    if not isinstance(B, torch.Tensor) or B.dtype != torch.complex64 or B.dim() != 2:
        raise ValueError("B must be a complex64 [N, K] tensor")
    dims = [int(d) for d in dims]
    N, K = int(B.shape[0]), int(B.shape[1])
    if int(np.prod(dims)) != N:
        raise ValueError("prod(dims) must equal B.shape[0]")
    B = B.contiguous()
    dev = B.device
    U = [torch.empty((d, d), dtype=torch.complex64, device=dev) for d in dims]
    core = torch.empty((N * K,), dtype=torch.complex64, device=dev)
    d64 = (ctypes.c_int64 * 3)(*dims)
    ranks = (ctypes.c_int64 * 3)()
    dropped = (ctypes.c_double * 3)()
    with torch.cuda.device(dev):
        L.check(lib.maxwell_tucker_compress(d64, K, _ptr(B), float(eps), _ptr(U[0]), _ptr(U[1]), _ptr(U[2]),
                                            _ptr(core), ranks, dropped, _stream()))
    r = [int(v) for v in ranks]
    Us = [U[m].reshape(-1)[: dims[m] * r[m]].reshape(dims[m], r[m]).clone() for m in range(3)]
    core = core[: r[0] * r[1] * r[2] * K].reshape(r[0], r[1], r[2], K).clone()
    return Us, core, r, [float(v) for v in dropped]
