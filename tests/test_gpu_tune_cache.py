"""The plan-time tuning cache across processes: a first process creating dense-basis plans
times the candidates (streaming kernel, tiled GEMM at each split-K factor) and writes its
choices to the tuning file; a second process with the same file times nothing, reuses every
choice, and so runs the same kernels (its gradient is equal bit for bit)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
from _common import Case
from paper_2008_09042_amd.encoding import tune_counts
out = {}
for name, kw in (("j8", dict(seed=501, dims=(64, 48), J=8, K=32)), ("j32", dict(seed=502, dims=(48, 40), J=32, K=20))):
    cs = Case(**kw)
    plan = cs.plan("bf16_split")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to("cuda:0")
    loss, gx, gc = plan.grad(T(cs.x0), T(cs.c0), T(cs.y))
    torch.cuda.synchronize()
    out[name] = [float(loss.item()), float(gx.abs().sum().item()), float(gc.abs().sum().item())]
out["counts"] = tune_counts()
print("RESULT " + json.dumps(out), flush=True)
"""


def run_child(cache):
    env = dict(os.environ, MAXWELL_TUNE_CACHE=cache)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_tuning_file_reused_by_a_second_process(tmp_path):
    cache = str(tmp_path / "tune.txt")
    print("[case] tuning cache, first process", flush=True)
    first = run_child(cache)
    assert first["counts"][0] == 4 and first["counts"][1] == 0, first["counts"]
    lines = open(cache).read().splitlines()
    assert len(lines) == 4 and all(" = " in l and "N=" in l for l in lines), lines
    print("[case] tuning cache, second process", flush=True)
    second = run_child(cache)
    assert second["counts"] == [0, 4], second["counts"]
    assert first["j8"] == second["j8"] and first["j32"] == second["j32"]
    assert len(open(cache).read().splitlines()) == 4
