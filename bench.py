"""Benchmark: gradient evaluations of the autograd encoding operator on one MI355X.

Workload: 3D Cartesian 128^3 image, 32 coils, K = 300 basis stored Tucker-factored
(factors 128x40, core 40x40x40x300), Poisson-disc mask R = 8 over (k0, k1) with a
20x20 centre and full readouts along k2 (2,048 lines x 128 = 262,144 samples per coil).
All inputs are seeded synthetic data (synth/), resident on the GPU before timing.

One step = one gradient evaluation of the autograd operator: forward
maxwell_forward_loss (B c, x (.) s_j, centred DFT, mask gather, weighted residual,
FP64 loss), then backward maxwell_adjoint on the residual (B c recomputed,
scatter, inverse DFT, coil combination, B^H).  Throughput is coil-images/s
= J x steps / s.  The headline precision is BF16-split; FP32 on the same GPU
is reported beside it.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]
    python bench.py --workload batch      # 64 uneven 2D slices through one captured graph
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "E/E^H/grad evals/sec (coil-images/s), BF16-split vs FP32 at ≤1e-4 rel err"
HBM_PEAK_GBS = 8000.0
PEAKS_TFLOPS = {"fp32": 157.3, "bf16": 2516.6}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16_split", choices=["bf16_split", "fp32"])
    ap.add_argument("--workload", default="cart3d",
                    choices=["cart3d", "batch", "gn", "admm", "compress", "kernels2d", "kernels2d_big"],
                    help="cart3d: the headline 128^3 Tucker workload; batch: 64 uneven 2D slices with "
                         "dense bases through one captured graph; gn: conjugate-gradient steps of the "
                         "Gauss-Newton normal equations on the 128^3 Tucker workload; admm: constrained "
                         "TV-SENSE reconstruction steps on the 2D 256^2 workload; compress: Tucker "
                         "compression of a smooth dense 3D basis; kernels2d: per-kernel roofline "
                         "figures of the general path on the 2D Cartesian and radial workloads; "
                         "kernels2d_big: the same with 128-coil stacks of 268 MB (above the "
                         "last-level cache)")
    ap.add_argument("--cg-iters", type=int, default=10, help="gn workload: CG steps per timed call")
    ap.add_argument("--branches", type=int, default=4, help="batch workload: concurrent branches")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the second-precision run")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (calibrates rocprofv3 byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) made with --copy-probe "
                         "into the per-launch HBM traffic file under profiles/, then exit")
    return ap.parse_args()


def make_inputs():
    from synth import problem
    t0 = time.time()
    p = problem("cart3d_128_tucker40x300_j32")
    log(f"[bench] inputs generated in {time.time() - t0:.1f}s: dims {p.dims} J {p.J} K {p.K} M {p.M}")
    return p


def time_steps(step, steps, warmup, torch):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        step()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


WORKLOAD = "cart3d_128_tucker40x300_j32"
KERNEL_SOURCES = {  # sources whose change invalidates a recorded traffic figure
    "plane_adj": ["tucker_fused.hip", "fused.h", "fft_device.h", "mfma_frag.h"],
    "plane_fwd": ["tucker_fused.hip", "fused.h", "fft_device.h", "mfma_frag.h"],
}
KERNEL_SYMBOLS = {"plane_adj": "plane_adj_kernel<1, 128, 128, 3, true>", "plane_fwd": "plane_fwd_kernel<1, 128, 128, 3, false>"}


def source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, "paper_2008_09042_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_{WORKLOAD}.txt")


def recorded_traffic(kernel):
    """HBM bytes per launch from the recorded counter runs, or None if absent or stale."""
    path = traffic_file(kernel)
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    if kv.get("source_sha256_16") != source_hash(kernel):
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


def traffic_from(fetch_dir, write_dir, probe_mib):
    """Per-launch FETCH_SIZE / WRITE_SIZE of the dominant kernels, scaled by the copy probe."""
    import csv
    import glob

    def per_kernel(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        acc = {}
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    known = probe_mib * 2**20
    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        acc = per_kernel(d, counter)
        copies = [v for k, v in acc.items() if "MulFunctor" in k]
        probe = max(max(v) for v in copies) * 1024.0  # KiB -> bytes; the probe is the largest multiply
        factor = known / probe
        for kernel, sym in KERNEL_SYMBOLS.items():
            vals = [v for k, vs in acc.items() if sym in k for v in vs]
            if vals:
                out.setdefault(kernel, {})[counter] = (sum(vals) / len(vals) * 1024.0 * factor, factor, len(vals))
    for kernel, c in out.items():
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        with open(traffic_file(kernel), "w") as fh:
            fh.write(f"# HBM traffic per launch of {KERNEL_SYMBOLS[kernel]}, workload {WORKLOAD}\n")
            fh.write(f"# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch), averaged over "
                     f"{c['FETCH_SIZE'][2]} dispatches, scaled so that a {probe_mib} MiB streaming kernel (x 2) reads and "
                     f"writes {probe_mib} MiB\n")
            fh.write(f"fetch_scale={c['FETCH_SIZE'][1]:.4f}\nwrite_scale={c['WRITE_SIZE'][1]:.4f}\n")
            fh.write(f"fetch_bytes_per_launch={c['FETCH_SIZE'][0]:.0f}\nwrite_bytes_per_launch={c['WRITE_SIZE'][0]:.0f}\n")
            fh.write(f"source_sha256_16={source_hash(kernel)}\n")
        log(f"[bench] wrote {traffic_file(kernel)}")


def kernel_work(name, p, prec):
    """Algorithmic work of one launch of a kernel of the fused 3D Tucker path.

    Returns (bound, unit, amount, peak).  Contractions count 8 real flops per complex
    multiply-accumulate (CMAC) over the mode products the kernel performs; memory-bound
    kernels count the bytes they must move (complex64 = 8 B, FP32 weights = 4 B)."""
    n0, n1, n2 = p.dims
    r0, r1, r2 = (u.shape[1] for u in p.U)
    J, K, M = p.J, p.K, p.M
    planes = J * n2
    # FP32 plans issue 16x16x4 FP32 MFMAs; BF16-split plans issue 16x16x32 BF16 MFMAs,
    # three per algorithmic product (hi*hi + hi*lo + lo*hi), so their fraction of the
    # published BF16 peak is at most 1/3 when counted in algorithmic flops as here.
    mfma_peak = PEAKS_TFLOPS["bf16" if prec == "bf16_split" else "fp32"]
    R = r0 * r1 * r2
    core_bytes = 8.0 * (R * K + J * K + J * R)
    v_p = r0 * r1 * n1 + n0 * r0 * n1          # V = W U1^T, P = U0 V  per coil-plane
    y_w = n0 * n1 * r1 + r0 * n0 * r1          # Y = h conj(U1), Wb = U0^H Y
    table = {
        "plane_fwd": ("mfma", "TFLOP/s", 8.0 * planes * v_p, mfma_peak),
        "plane_adj": ("mfma", "TFLOP/s", 8.0 * planes * (v_p + y_w), mfma_peak),
        "line_fwd": ("hbm", "GB/s", 8.0 * J * M * 3 + 4.0 * M, HBM_PEAK_GBS),
        "line_adj": ("hbm", "GB/s", 8.0 * J * M * 2, HBM_PEAK_GBS),
        "core_fwd": ("hbm", "GB/s", core_bytes, HBM_PEAK_GBS),
        "core_adj": ("hbm", "GB/s", core_bytes, HBM_PEAK_GBS),
        "gemm_core_coef": ("hbm", "GB/s", core_bytes, HBM_PEAK_GBS),
        "gemm_core_adjoint": ("hbm", "GB/s", core_bytes, HBM_PEAK_GBS),
        "mode3_fwd": ("hbm", "GB/s", 8.0 * (J * R + J * n2 * r0 * r1 + n2 * r2), HBM_PEAK_GBS),
        "mode3_adj": ("hbm", "GB/s", 8.0 * (J * R + J * n2 * r0 * r1 + n2 * r2), HBM_PEAK_GBS),
        "gemm_mode3": ("hbm", "GB/s", 8.0 * (J * R + J * n2 * r0 * r1 + n2 * r2), HBM_PEAK_GBS),
        "gemm_mode3_adjoint": ("hbm", "GB/s", 8.0 * (J * R + J * n2 * r0 * r1 + n2 * r2), HBM_PEAK_GBS),
    }
    return table.get(name)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, coils=32, repeats=2):
    """The FP64 oracle on host cores: `repeats` gradient evaluations over `coils` coils, with BLAS
    threads and scipy.fft workers both set to the cores in the process affinity mask."""
    import scipy.fft
    import threadpoolctl
    from oracle import Oracle
    ncores = len(os.sched_getaffinity(0))
    with threadpoolctl.threadpool_limits(limits=ncores), scipy.fft.set_workers(ncores):
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
        op = Oracle(p.dims, U=p.U, core=p.core, mask_idx=p.mask_idx)
        rng = np.random.default_rng(0)
        y = rng.normal(size=(coils, p.M)) + 1j * rng.normal(size=(coils, p.M))
        t0 = time.perf_counter()
        for _ in range(repeats):
            op.loss_and_grad(p.x0, p.c0[:coils], y)
        dt = time.perf_counter() - t0
    return {"value": repeats * coils / dt, "unit": "coil-images/s", "cores": int(max(threads, ncores)),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{repeats} FP64 gradient evaluations over {coils} of the 32 coils at 128^3 "
                      f"(Tucker 40^3 x 300, 262,144 samples/coil): {dt:.1f} s; scipy.fft workers = {ncores}, "
                      f"BLAS threads = {threads}"}


# The paper's only timed operator (Supporting Table S1): one Tucker-basis matrix-vector product
# (q = 75 / 200 / 500 columns, FOV 192 x 192 x 170, eps_t = 1e-4), with its hardware.  Context,
# not a target: a different operator (the basis product alone, one coil) on other machines.
PAPER_CONTEXT = {
    "source": "Supporting Table S1, Tucker basis MVP time (s) at q = 75 / 200 / 500, FOV 192x192x170",
    "tucker_mvp_s_gpu": {"q75": 0.6, "q200": 1.1, "q500": 2.9, "hardware": "Tesla V100, PyTorch, CUDA 10.1"},
    "tucker_mvp_s_cpu": {"q75": 18.9, "q200": 50.4, "q500": 127.1, "hardware": "Intel Xeon"},
    "dense_mvp_s_gpu": {"q75": 0.1, "hardware": "Tesla V100 (q = 200, 500 do not fit)"},
}


def device_smooth_basis(torch, dims, params, dev):
    """The slice recipe's basis (smooth columns poly_q(2r) exp(2 pi i k_q . r), QR-orthonormalised)
    evaluated on the device in FP64 from the parameters drawn on the host (synth.smooth_params):
    64 host QRs of up to 102,400 x 256 would take minutes.  Input synthesis only."""
    exps, coef, kvec = params
    r = [(torch.arange(n, device=dev, dtype=torch.float64) - n // 2) / n for n in dims]
    g = torch.meshgrid(*r, indexing="ij")
    g = [t.reshape(-1) for t in g]
    mono = torch.stack([torch.prod(torch.stack([(2.0 * g[d]) ** e[d] for d in range(len(dims))]), dim=0)
                        for e in exps], dim=1)
    kv = torch.from_numpy(np.asarray(kvec)).to(dev)
    phase = sum(torch.outer(g[d], kv[:, d]) for d in range(len(dims)))
    cols = (mono.to(torch.complex128) @ torch.from_numpy(np.asarray(coef)).to(dev)) * torch.exp(2j * np.pi * phase)
    q = torch.linalg.qr(cols, mode="reduced").Q
    return q.to(torch.complex64).contiguous()


def bench_batch(args, torch):
    """The batched-slices workload: 64 seeded 2D problems of uneven sizes (dense bases, 3.9 GB
    in all), each one gradient evaluation per step, all slices in one replay of a captured
    graph (maxwell_batch_grad on `branches` concurrent branches).  Prints one JSON line."""
    from paper_2008_09042_amd.encoding import MaxwellBatch, MaxwellPlan
    from synth import BATCH, slice_problems
    dev = torch.device("cuda:0")
    t0 = time.time()
    ps = slice_problems(seed=5, n_slices=BATCH["n_slices"], materialise_basis=False)
    log(f"[bench] {len(ps)} slices generated in {time.time() - t0:.1f}s")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(dev)  # noqa: E731
    plans, xs, cs, ys = [], [], [], []
    other = [q for q in ("bf16_split", "fp32") if q != args.precision][0]
    other_plans = []
    t0 = time.time()
    for p in ps:
        kw = dict(mask_idx=p.mask_idx) if p.sampling == "cartesian" else dict(traj=p.traj)
        Bd = device_smooth_basis(torch, p.dims, p.basis_params, dev)
        plans.append(MaxwellPlan(p.dims, p.J, B=Bd, **kw, weights=p.weights, precision=args.precision,
                                 device=dev))
        if not args.no_compare:  # the same slices at the other precision, on the same device bases
            other_plans.append(MaxwellPlan(p.dims, p.J, B=Bd, **kw, weights=p.weights, precision=other,
                                           device=dev))
        xs.append(T(p.x0))
        cs.append(T(p.c0))
        ys.append(T(p.noise))
    torch.cuda.synchronize()
    from paper_2008_09042_amd.encoding import tune_counts
    tuned = tune_counts()
    log(f"[bench] plans ready in {time.time() - t0:.1f}s (dense products: {tuned[0]} shapes timed, "
        f"{tuned[1]} reused from the tuning cache)")
    batch = MaxwellBatch(plans, branches=args.branches, staged=True)
    coils = sum(p.J for p in ps)
    basis_bytes = sum(8 * p.N * p.K for p in ps)
    eager_ms, _ = time_steps(lambda: batch.grad(xs, cs, ys), args.steps, args.warmup, torch)
    batch.capture(xs, cs, ys)
    ms, wall = time_steps(batch.replay, args.steps, args.warmup, torch)
    log(f"[bench] batch: {ms:.3f} ms/step graph ({coils * 1000.0 / ms:.0f} coil-images/s), eager {eager_ms:.3f} ms")
    del batch
    # per-slice latency inside a captured replay: the same batch with each slice's device
    # timestamps (start of its first step, end of its last) written by the graph itself (two
    # small kernels per slice, so its step is timed on its own); median over replays
    sb = MaxwellBatch(plans, branches=args.branches, staged=True, stamps=True)
    sb.capture(xs, cs, ys)
    stamped_ms, _ = time_steps(sb.replay, args.steps, args.warmup, torch)
    lat_runs = []
    for _ in range(5):
        sb.replay()
        torch.cuda.synchronize()
        lat_runs.append(sb.latencies_ms())
    lat = np.median(np.array(lat_runs), axis=0)
    log(f"[bench] batch with per-slice timestamps: {stamped_ms:.3f} ms/step graph; slice latency p50 "
        f"{np.percentile(lat, 50):.3f} ms, p99 {np.percentile(lat, 99):.3f} ms")
    del sb
    # the same batch with each slice's whole chain on a branch (no phases), for comparison
    cb = MaxwellBatch(plans, branches=args.branches, staged=False)
    cb.capture(xs, cs, ys)
    chain_ms, _ = time_steps(cb.replay, args.steps, args.warmup, torch)
    log(f"[bench] batch, whole chains per branch: {chain_ms:.3f} ms/step graph")
    del cb
    compare = None
    if other_plans:
        ob = MaxwellBatch(other_plans, branches=args.branches, staged=True)
        ob.capture(xs, cs, ys)
        oms, _ = time_steps(ob.replay, args.steps, args.warmup, torch)
        compare = {"precision": other, "ms_per_step": oms, "value": coils * 1000.0 / oms}
        log(f"[bench] batch {other}: {oms:.3f} ms/step graph ({coils * 1000.0 / oms:.0f} coil-images/s)")
        del ob
    out = {
        "metric": METRIC,
        "value": coils * 1000.0 / ms,
        "unit": "coil-images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split" if args.precision == "bf16_split" else "f32",
        "data": "synthetic (seeded phantoms, smooth QR-orthonormalised dense bases, variable-density "
                "Poisson-disc / golden-angle radial sampling)",
        "config": {"workload": BATCH["name"], "slices": len(ps), "coils_total": coils,
                   "basis_gb": round(basis_bytes / 1e9, 2), "branches": args.branches,
                   "cartesian_slices": sum(p.sampling == "cartesian" for p in ps),
                   "step": "one graph replay: loss + gradient of every slice (maxwell_grad per slice: "
                           "B c once, kept for the adjoint; B^H once), the slices' steps issued in phases "
                           "with each phase's FFT passes of all slices launched together"},
        "eager_ms_per_step": eager_ms,
        "chains_per_branch_ms_per_step": chain_ms,
        "stamped_ms_per_step": stamped_ms,
        "plan_tuning": {"timed": tuned[0], "reused_from_cache": tuned[1]},
        "other_precision": compare,
        "basis_stream_gbs": 2.0 * basis_bytes / (ms * 1e-3) / 1e9,
        "slice_latency_ms": {"source": "device timestamps inside replays of the same batch captured with "
                                       "them (median of 5 replays)",
                             "p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "min": float(lat.min()), "max": float(lat.max())},
    }
    print(json.dumps(out), flush=True)


def bench_gn(args, torch):
    """Gauss-Newton step of the joint solve on the 128^3 Tucker workload: maxwell_cg with
    cg-iters steps per call, each step one normal-operator application (two encodes for the
    JVP, one adjoint with B c recomputed, the shift) plus the FP64 inner products.  Prints
    one JSON line (coil-images/s = J x normal-operator applications per second)."""
    from paper_2008_09042_amd.encoding import MaxwellPlan
    dev = torch.device("cuda:0")
    p = make_inputs()
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(dev)  # noqa: E731
    U = [T(u) for u in p.U]
    core = T(p.core)
    res = {}
    for prec in ([args.precision] if args.no_compare else [args.precision] +
                 [q for q in ("bf16_split", "fp32") if q != args.precision]):
        plan = MaxwellPlan(p.dims, p.J, U=U, core=core, mask_idx=p.mask_idx, precision=prec, device=dev)
        x0, c0 = T(p.x0), T(p.c0)
        y = plan.encode(T(p.x_true), T(p.c_true)).contiguous()
        _, bx, bc = plan.grad(x0, c0, y)  # right-hand side of the shape of a Gauss-Newton step
        bx, bc = -0.5 * bx, -0.5 * bc
        ox, oc = plan.normal(x0, c0, bx, bc, 0.0, 0.0)
        q = (torch.vdot(bx.reshape(-1), ox.reshape(-1)).real + torch.vdot(bc.reshape(-1), oc.reshape(-1)).real) / (
            torch.linalg.vector_norm(bx) ** 2 + torch.linalg.vector_norm(bc) ** 2)
        lam = float(0.2 * q)
        it = args.cg_iters
        ms, wall = time_steps(lambda: plan.cg(x0, c0, bx, bc, lam, lam, it), args.steps, args.warmup, torch)
        res[prec] = ms / it
        log(f"[bench] gn {prec}: {ms:.3f} ms per {it} CG steps ({ms / it:.3f} ms per normal-operator "
            f"application, {p.J * it * 1000.0 / ms:.0f} coil-images/s)")
        if prec == args.precision:
            plan.set_timing(True)
            plan.cg(x0, c0, bx, bc, lam, lam, it)
            torch.cuda.synchronize()
            kt = plan.timing()
            plan.set_timing(False)
            log("[bench] gn kernel timing (us per launch): " +
                ", ".join(f"{k} {1000 * t / n:.1f}x{n // it}" for k, (n, t) in kt.items() if n))
        del plan
    ms_it = res[args.precision]
    out = {
        "metric": "Gauss-Newton normal-operator applications/sec x coils (coil-images/s)",
        "value": p.J * 1000.0 / ms_it,
        "unit": "coil-images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_it * args.cg_iters,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split" if args.precision == "bf16_split" else "f32",
        "data": "synthetic (seeded phantom, Tucker basis, Poisson-disc mask; no datasets)",
        "config": {"workload": "gn_" + WORKLOAD, "cg_iters_per_step": args.cg_iters,
                   "step": "maxwell_cg: CG steps on (J^H J + lambda) dv = b, FP64 inner products on the device"},
        "ms_per_cg_iteration": {k: v for k, v in res.items()},
    }
    print(json.dumps(out), flush=True)


def bench_admm(args, torch):
    """Constrained TV-SENSE reconstruction (Sec. II-C) on the 2D Cartesian 256^2 workload
    (32 coils, variable-density mask): maxwell_sense_admm with 10 outer steps per call, each
    20 TV steps and 5 CG steps.  Coil maps: the workload's basis times its coefficients,
    scaled to order-one sensitivities.  Prints one JSON line."""
    from paper_2008_09042_amd.encoding import MaxwellPlan
    from synth import problem
    dev = torch.device("cuda:0")
    t0 = time.time()
    p = problem("cart2d_256_dense200_j32")
    log(f"[bench] inputs generated in {time.time() - t0:.1f}s: dims {p.dims} J {p.J} K {p.K} M {p.M}")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(dev)  # noqa: E731
    plan = MaxwellPlan(p.dims, p.J, B=T(p.B), mask_idx=p.mask_idx, precision="fp32", device=dev)
    S = plan.basis_apply(T(p.c_true))
    S = (S / torch.sqrt(torch.mean(torch.sum(S.abs() ** 2, dim=0)))).contiguous()
    y = plan.sense_encode(S, T(p.x_true))
    noise = T(p.noise)
    y = (y + noise * (0.01 * torch.linalg.vector_norm(y) / torch.linalg.vector_norm(noise))).contiguous()
    eps = (1.05 * 0.01 * torch.linalg.vector_norm(y, dim=1)).float()
    outer, cg_it, tv_it = 10, 5, 20
    ms, wall = time_steps(lambda: plan.sense_admm(S, y, eps, 1.0, outer, cg_it, tv_it), args.steps, args.warmup,
                          torch)
    plan.set_timing(True)
    plan.sense_admm(S, y, eps, 1.0, outer, cg_it, tv_it)
    torch.cuda.synchronize()
    kt = plan.timing()
    plan.set_timing(False)
    log(f"[bench] admm: {ms:.3f} ms per {outer} ADMM steps ({ms / outer:.3f} ms per step)")
    log("[bench] admm kernel timing (us per launch, launches per ADMM step): " +
        ", ".join(f"{k} {1000 * t / n:.1f}x{n / outer:g}" for k, (n, t) in kt.items() if n))
    # every ADMM step applies F_s S (and its adjoint) cg_it + 4 times per coil
    applies = outer * (cg_it + 4) * p.J
    out = {
        "metric": "constrained TV-SENSE ADMM steps/sec (Sec. II-C), x coils",
        "value": outer * p.J * 1000.0 / ms,
        "unit": "coil-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantom, smooth dense basis maps, variable-density mask; no datasets)",
        "config": {"workload": "admm_cart2d_256_j32", "admm_steps_per_call": outer, "cg_steps": cg_it,
                   "tv_steps": tv_it, "step": "maxwell_sense_admm call"},
        "coil_operator_applications_per_s": applies * 1000.0 / ms,
    }
    print(json.dumps(out), flush=True)


def bench_compress(args, torch):
    """Accuracy-controlled Tucker compression (ST-HOSVD, eps = 1e-4) of a smooth dense 3D basis
    of 64^3 voxels x 100 columns (210 MB): the compression step that produces the Tucker
    form from dense inputs.  Prints one JSON line."""
    from paper_2008_09042_amd.encoding import tucker_compress
    from synth import rng_for, smooth_dense_basis
    dev = torch.device("cuda:0")
    dims, K, eps = (64, 64, 64), 100, 1e-4
    t0 = time.time()
    B = smooth_dense_basis(rng_for(61, 2), dims, K, 6, 3.0)
    log(f"[bench] basis {dims} x {K} generated in {time.time() - t0:.1f}s")
    Bt = torch.from_numpy(B.astype(np.complex64)).to(dev)
    del B
    ms, wall = time_steps(lambda: tucker_compress(Bt, dims, eps), args.steps, args.warmup, torch)
    Us, core, r, dropped = tucker_compress(Bt, dims, eps)
    torch.cuda.synchronize()
    dense_bytes = 8 * int(np.prod(dims)) * K
    tucker_bytes = 8 * (sum(int(n) * int(q) for n, q in zip(dims, r)) + int(np.prod(r)) * K)
    err = float(np.sqrt(sum(dropped)) / torch.linalg.vector_norm(Bt).item())
    log(f"[bench] compress: {ms:.1f} ms, ranks {r}, {dense_bytes / 1e6:.0f} MB -> {tucker_bytes / 1e6:.2f} MB, "
        f"relative error {err:.2e}")
    out = {
        "metric": "Tucker compressions/sec (ST-HOSVD, eps 1e-4)",
        "value": 1000.0 / ms,
        "unit": "compressions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64-gram/f32-products",
        "data": "synthetic (smooth dense basis: polynomial x plane-wave fields, QR-orthonormalised)",
        "config": {"workload": "compress_dense_64cube_k100", "eps": eps, "ranks": r,
                   "dense_mb": dense_bytes / 1e6, "tucker_mb": tucker_bytes / 1e6},
        "relative_error": err,
    }
    print(json.dumps(out), flush=True)


def bench_kernels2d(args, torch, names=("cart2d_256_dense200_j32", "radial2d_256_dense128_j16")):
    """Per-kernel roofline figures of the general path (dense basis GEMMs on the matrix cores,
    axis FFTs, Cartesian sampling, KB gridding) on the 2D Cartesian 256^2 (32 coils, K 200)
    and radial 256^2 (16 coils, K 128, 64 spokes x 512) workloads, from the in-library HIP
    events over `steps` gradient evaluations.  Achieved = algorithmic work / average launch
    time; algorithmic bytes count each array once (complex64 8 B, FP32 4 B, index 4 B).
    Prints one JSON line."""
    from paper_2008_09042_amd.encoding import MaxwellPlan
    from synth import problem
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(dev)  # noqa: E731
    res = {}
    for name in names:
        t0 = time.time()
        p = problem(name)
        log(f"[bench] {name}: inputs ready in {time.time() - t0:.1f}s")
        kw = dict(mask_idx=p.mask_idx) if p.traj is None else dict(traj=p.traj, weights=p.weights)
        N, J, K, M = int(np.prod(p.dims)), p.J, p.K, p.M
        for prec in ("bf16_split", "fp32"):
            plan = MaxwellPlan(p.dims, J, B=T(p.B), **kw, precision=prec, device=dev)
            x, c, y = T(p.x0), T(p.c0), T(p.noise)
            for _ in range(args.warmup):
                plan.grad(x, c, y)
            torch.cuda.synchronize()
            plan.set_timing(True)
            for _ in range(args.steps):
                plan.grad(x, c, y)
            torch.cuda.synchronize()
            kt = plan.timing()
            plan.set_timing(False)
            G = (2 * p.dims[0]) * (2 * p.dims[1]) if p.traj is not None else 0
            gemm_flops = 8.0 * J * N * K
            gemm_bytes = 8.0 * (N * K + J * K + J * N)
            work = {
                "gemm_dense_apply": ("mfma", gemm_flops, PEAKS_TFLOPS["bf16" if prec == "bf16_split" else "fp32"],
                                     gemm_bytes),
                "gemm_dense_adjoint": ("mfma", gemm_flops, PEAKS_TFLOPS["bf16" if prec == "bf16_split" else "fp32"],
                                       gemm_bytes),
                # Cartesian: the mask is applied in the last forward and the first inverse
                # pass (8 B per element in, 8 B per sample and 4 B of inverse mask per point
                # out, and the reverse), so the four passes move 48 J N + 16 J M + 8 N bytes
                # gridding (g0 x g1 grid, n0 x n1 window): the first forward pass reads the
                # window (8 B per image element and coil, and the image) and writes its n0 rows,
                # the second reads them and writes the grid; the first inverse pass reads the
                # grid and writes the window's n1 columns, the last reads them and writes the
                # window: 8 J (2 N + 2 n0 g1 + 2 G + 2 g0 n1) + 8 N bytes in four passes
                "fft_axis": ("hbm", (16.0 * J * (N + G + 2 * p.dims[0] * p.dims[1] * 2) + 8.0 * N) / 4 if G
                             else (48.0 * J * N + 16.0 * J * M + 8.0 * N) / 4, None, None),
                "gather": ("hbm", 8.0 * J * M * 2 + 4.0 * M, None, None),
                "scatter": ("hbm", 8.0 * J * (M + N) + 4.0 * N, None, None),
                "nufft_degrid": ("hbm", 8.0 * J * (G + M) + M * (8.0 + 48.0), None, None),
                "nufft_spread": ("hbm", 8.0 * J * (G + 2 * M) + M * (64.0 + 8.0) + 4.0 * G, None, None),
                "adjoint_combine": ("hbm", 8.0 * (3 * J * N + 2 * N), None, None),
                "residual": ("hbm", 8.0 * J * M * 3 + 4.0 * M, None, None),
            }
            out = {}
            for k, (n_launch, ms) in kt.items():
                if not n_launch or k not in work:
                    continue
                us = 1000.0 * ms / n_launch
                bound, amount, peak, byts = work[k]
                if bound == "mfma":
                    tf = amount / (us * 1e-6) / 1e12
                    out[k] = {"us": round(us, 1), "bound": "mfma", "achieved_tflops": round(tf, 2),
                              "peak_tflops": peak, "frac": round(tf / peak, 4),
                              "hbm_gbs": round(byts / (us * 1e-6) / 1e9, 1),
                              "hbm_frac": round(byts / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 3)}
                else:
                    gbs = amount / (us * 1e-6) / 1e9
                    out[k] = {"us": round(us, 1), "bound": "hbm", "achieved_gbs": round(gbs, 1),
                              "peak_gbs": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 3)}
            res[f"{name}/{prec}"] = out
            log(f"[bench] {name} {prec}: " + ", ".join(
                f"{k} {v['us']}us {v.get('achieved_gbs', v.get('achieved_tflops'))}"
                f"{'GB/s' if v['bound'] == 'hbm' else 'TF/s'} ({100 * v['frac']:.1f}%)" for k, v in out.items()))
            del plan
    print(json.dumps({"metric": "per-kernel roofline fractions, general path", "workload": "+".join(names),
                      "steps": args.steps, "kernels": res}), flush=True)


def main():
    args = parse()
    if args.traffic_from:
        traffic_from(args.traffic_from[0], args.traffic_from[1], args.copy_probe or 256)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1 "
                                   "(the coil-sharded multi-GPU design is documented but not built)"}))
        sys.exit(2)
    import torch
    from paper_2008_09042_amd.encoding import MaxwellDataFidelity, MaxwellPlan
    if args.copy_probe:
        # one streaming kernel that reads and writes exactly MIB MiB (float32 scale by 2), the
        # calibration of the byte counters
        n = args.copy_probe * 2**20 // 4
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "batch":
        bench_batch(args, torch)
        return
    if args.workload == "gn":
        bench_gn(args, torch)
        return
    if args.workload == "admm":
        bench_admm(args, torch)
        return
    if args.workload == "compress":
        bench_compress(args, torch)
        return
    if args.workload == "kernels2d":
        bench_kernels2d(args, torch)
        return
    if args.workload == "kernels2d_big":
        bench_kernels2d(args, torch, ("cart2d_512_dense16_j128", "radial2d_256_dense32_j128"))
        return

    dev = torch.device("cuda:0")
    p = make_inputs()
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(dev)  # noqa: E731
    U = [T(u) for u in p.U]
    core = T(p.core)
    plans = {}
    for prec in ("bf16_split", "fp32"):
        plans[prec] = MaxwellPlan(p.dims, p.J, U=U, core=core, mask_idx=p.mask_idx, precision=prec, device=dev)
    log(f"[bench] plans ready; workspace {plans['fp32'].ws_bytes / 2**30:.2f} GiB")
    # measured data y = E(x_true, c_true) + noise at 40 dB (synthesised on the GPU)
    y = plans["fp32"].encode(T(p.x_true), T(p.c_true))
    noise = T(p.noise)
    y = y + noise * (0.01 * torch.linalg.vector_norm(y) / torch.linalg.vector_norm(noise))
    y = y.contiguous()
    x0 = T(p.x0)
    c0 = T(p.c0)

    results = {}
    grads = {}
    kernels_by_prec = {}
    order = [args.precision] + ([] if args.no_compare else [q for q in ("bf16_split", "fp32") if q != args.precision])
    for prec in order:
        plan = plans[prec]
        x = x0.clone().requires_grad_(True)
        c = c0.clone().requires_grad_(True)

        def step():
            x.grad = None
            c.grad = None
            f = MaxwellDataFidelity.apply(x, c, y, plan)
            f.backward()
            return f

        ms, wall = time_steps(step, args.steps, args.warmup, torch)
        results[prec] = ms
        grads[prec] = (x.grad.clone(), c.grad.clone())
        log(f"[bench] {prec}: {ms:.3f} ms/step ({p.J * 1000.0 / ms:.0f} coil-images/s), wall {wall:.2f}s")
        # same K steps again with per-kernel HIP events recorded by the library on the launch stream
        plan.set_timing(True)
        ms_t, _ = time_steps(step, args.steps, 0, torch)
        kt = plan.timing()
        plan.set_timing(False)
        kernels_by_prec[prec] = {k: {"launches": n, "avg_us": 1000.0 * t / n} for k, (n, t) in kt.items() if n}
        log(f"[bench] {prec} kernel timing pass: {ms_t:.3f} ms/step; " +
            ", ".join(f"{k} {v['avg_us']:.1f}us x{v['launches']}" for k, v in
                      sorted(kernels_by_prec[prec].items(), key=lambda kv: -kv[1]["avg_us"] * kv[1]["launches"])))

    prec = args.precision
    ms = results[prec]
    out = {
        "metric": METRIC,
        "value": p.J * 1000.0 / ms,
        "unit": "coil-images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split" if prec == "bf16_split" else "f32",
        "data": "synthetic (seeded phantom, Tucker basis, Poisson-disc mask; no datasets)",
        "config": {"workload": "cart3d_128_tucker40x300_j32", "image": list(p.dims), "coils": p.J, "K": p.K,
                   "tucker_ranks": [40, 40, 40], "samples_per_coil": p.M, "precision": prec,
                   "step": "autograd grad eval: forward loss + backward adjoint, B c recomputed"},
    }
    if "fp32" in results and prec != "fp32":
        out["fp32"] = {"ms_per_step": results["fp32"], "value": p.J * 1000.0 / results["fp32"]}
        gx32, gc32 = grads["fp32"]
        gxs, gcs = grads[prec]
        out["bf16_split_vs_fp32_rel_diff"] = {
            "gx": float(torch.linalg.vector_norm(gxs - gx32) / torch.linalg.vector_norm(gx32)),
            "gc": float(torch.linalg.vector_norm(gcs - gc32) / torch.linalg.vector_norm(gc32))}
    kernels = kernels_by_prec[prec]
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    work = kernel_work(dom, p, prec)
    if work is not None:
        bound, unit, amount, peak = work
        avg_s = kernels[dom]["avg_us"] * 1e-6
        achieved = amount / avg_s / (1e12 if unit == "TFLOP/s" else 1e9)
        out["roofline"] = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                           "frac": achieved / peak, "traffic": recorded_traffic(dom),
                           "per_launch": amount, "avg_launch_us": kernels[dom]["avg_us"]}
    if "fp32" in kernels_by_prec:
        # the basis-apply kernels of the FP32 plan against the FP32 matrix-core peak (algorithmic
        # flops: 8 per complex multiply-accumulate of the mode products each kernel performs)
        k32 = kernels_by_prec["fp32"]
        out["roofline_fp32"] = {}
        for name in ("plane_fwd", "plane_adj"):
            if name in k32:
                bound, unit, amount, peak = kernel_work(name, p, "fp32")
                achieved = amount / (k32[name]["avg_us"] * 1e-6) / 1e12
                out["roofline_fp32"][name] = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                                              "frac": achieved / peak, "per_launch": amount,
                                              "avg_launch_us": k32[name]["avg_us"]}
        out["kernels_fp32"] = k32
    out["kernels"] = kernels
    out["paper_context"] = PAPER_CONTEXT
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host (bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
