"""LBM_TRACE=1: per-launch timing printed when a lattice is destroyed.

A child process (the variable is read when a handle is created) steps a
small jet lattice and a two-level refined slab, then destroys them; its
stderr must list every step-kernel launch with the right call counts (three
even and three odd steps; each level-1 tile class twice as often as level
0's), and nothing at all without the variable.
"""
import os
import re
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import gc
import numpy as np
import torch
import paper_1206_0389_amd as P
import synth
torch.cuda.set_device(0)
nx, ny, nz = 64, 16, 12
lat = P.Lattice(model="fclb", storage="f32", shape=(nx, ny, nz), nu=0.02)
iu, im = synth.jet_inlet(nx, ny, 4.0, 0.05, 0.002)
lat.set_boundaries([P.WALL] * 4 + [P.INLET, P.OUTFLOW],
                   face_u=[[0.0, 0.0, 0.002]] * 4 + [[0.0, 0.0, 0.0]] * 2,
                   inlet_u=torch.from_numpy(iu), inlet_mask=torch.from_numpy(im))
lat.set_populations(torch.from_numpy(synth.random_populations(27, (nz, ny, nx), 1e-3, seed=1)))
lat.step(6)
lat.reduce()
del lat
gc.collect()
m = np.zeros((16, 1, 1), dtype=np.uint8)
m[6:10] = 1
g = P.RefinedLattice(model="fclb", storage="f32", shape=(4, 4, 64), nu=0.02, block=4,
                     level_map=m, nlevels=2, faces=[P.PERIODIC] * 6)
for level in range(2):
    sh = g.shape3(level)
    g.init_equilibrium(level, torch.zeros(sh, dtype=torch.float64, device="cuda"),
                       torch.zeros((3,) + tuple(sh), dtype=torch.float64, device="cuda"))
g.step(2)
torch.cuda.synchronize()
del g
gc.collect()
print("child done", flush=True)
"""

LINE = re.compile(r"lbm trace:\s+(\d+) calls\s+([\d.]+) ms total\s+([\d.]+) us mean\s+([\d.]+) "
                  r"us min\s+([\d.]+) us max\s+(.*)$")


def _run(trace):
    env = dict(os.environ)
    env.pop("LBM_TRACE", None)
    if trace:
        env["LBM_TRACE"] = "1"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    print("case trace child, LBM_TRACE", trace, flush=True)
    p = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-3000:]
    assert "child done" in p.stdout
    return p.stderr


def test_trace_lists_every_launch():
    err = _run(True)
    print(err, flush=True)
    assert "lbm trace (lattice)" in err and "lbm trace (refined lattice)" in err
    lattice, refined = err.split("lbm trace (refined lattice)")
    rows = []
    for block, name in ((lattice, "lattice"), (refined, "refined")):
        for line in block.splitlines():
            m = LINE.search(line)
            if m:
                n, tot, mean, mn, mx = (float(v) for v in m.groups()[:5])
                assert n >= 1 and tot > 0 and 0 < mn <= mean <= mx, line
                rows.append((name, int(n), m.group(6)))
    even = sum(n for w, n, lab in rows if w == "lattice" and "step_kernel" in lab and
               "ODD = false" in lab)
    odd = [n for w, n, lab in rows if w == "lattice" and "step_kernel" in lab and
           "ODD = true" in lab]
    assert even == 3
    assert odd and all(n == 3 for n in odd)
    assert sum(n for w, n, lab in rows if w == "lattice" and "reduce" in lab) == 1
    levels = {}
    for w, n, lab in rows:
        m = re.match(r"(level_step_kernel \(\w+ tiles\)) \[level (\d)\]", lab)
        if w == "refined" and m:
            levels[(m.group(1), int(m.group(2)))] = n
    assert levels, refined
    for (lab, lev), n in levels.items():
        if lev == 0 and (lab, 1) in levels:
            assert levels[(lab, 1)] == 2 * n, (lab, n, levels[(lab, 1)])
    assert any("ghost_patch_kernel [level 1]" in lab for _, _, lab in rows)


def test_no_trace_without_the_variable():
    err = _run(False)
    assert "lbm trace" not in err
