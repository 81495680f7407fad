"""Throughput benchmark: MLUPS and fraction of the MI355X HBM roofline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-others] [--workload NAME]

Default workload (one step = one fused collide-and-stream update of every
node, boundary rules included): the round jet, D3Q27 FCLB on a uniform
256 x 256 x 512 lattice, FP32 deviation storage, D = 32 top-hat inlet at
u = 0.05 with a seeded 1 % per-step perturbation, co-flow 0.002 on moving
side walls, zero-gradient outflow, nu = 1e-4. Inputs are synthetic and
resident in HBM before timing starts; K steps are timed with HIP events on
the stream the kernels run on, bracketed by device synchronisation.

Prints one JSON line. ``roofline`` prices the step kernel's algorithmic
traffic, 2 Q b bytes per node update (Q populations of b bytes read and
written once), against the 8 TB/s HBM peak; its ``traffic`` is the HBM
traffic per step measured in the same run by two rocprofv3 counter passes
over a short child run (``--traffic off`` skips them); the adjoint legs'
traffic comes from two more passes over a child run of those legs alone. ``others`` holds the same
measurement for the other model/storage combinations. ``adjoint`` times the
inlet-sensitivity gradient (128 x 128 x 256 jet, 400 steps, checkpoints
every 20; FCLB adjoint in FP32 and FP64, MRT-LES adjoint in FP32) and the
adjoint step kernel alone, priced at 3 Q b
bytes per node (state and adjoint read, adjoint written). ``statistics``
times the velocity time-average accumulation on the default workload.
``cpu_baseline``
is the FP64 oracle timed on the host cores on a cut-down of the same
workload.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import shutil
import signal
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LLC_BYTES = 256 << 20  # MI355X last-level (Infinity) cache
METRIC = "MLUPS and % of HBM roofline, D3Q19-MRT and D3Q27-FCLB, FP32/FP16 vs FP64"
BYTES = {"f64": 8, "f32": 4, "f16": 2}
# HBM bytes per step of the default workload measured with rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (scaled by a copy kernel of known size), valid only
# for the step kernel's sources whose hash is recorded with it.
STEP_SOURCES = ("stencil.h", "mrt.h", "fclb.h", "kernels.h", "trace.h", "lbm_api.hip")
MEASURED_TRAFFIC = {"bytes_per_step": 7.385e9, "sources_sha256_16": "bb6d12c17aa84cc6",
                    "workload": "jet256-fclb-f32"}
# The same for one adjoint step of the 128 x 128 x 256 jet (FP32), per model.
ADJOINT_SOURCES = ("stencil.h", "mrt.h", "fclb.h", "kernels.h", "adjoint.h", "trace.h",
                   "lbm_api.hip")
MEASURED_ADJOINT_TRAFFIC = {"sources_sha256_16": "53cad682a266f8d5", "storage": "f32",
                            "bytes_per_step": {"fclb": 1.386e9, "mrt": 0.966e9}}


def sources_hash(names=STEP_SOURCES):
    import hashlib
    m = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1206_0389_amd", "csrc", n), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="jet256-fclb-f32")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-others", action="store_true")
    p.add_argument("--other-steps", type=int, default=50)
    p.add_argument("--no-adjoint", action="store_true")
    p.add_argument("--traffic", choices=["auto", "off"], default="auto",
                   help="measure the step kernels' HBM traffic with rocprofv3 counter passes "
                        "over a short child run (auto: when rocprofv3 is available)")
    p.add_argument("--only-adjoint", action="store_true",
                   help="run only the adjoint legs and the copy probe (the adjoint counter "
                        "passes' child run)")
    return p.parse_args()


COPY_BYTES = 4 << 30  # the copy probe's size (copy_bandwidth)


def _run_counter_pass(exe, counter, workload, outdir, timeout, adjoint=False):
    """One rocprofv3 --pmc pass over a short child run of this script (the
    workload's steps, or with adjoint the adjoint legs alone); returns the
    rows of its counter csv (or raises RuntimeError)."""
    what = (["--only-adjoint"] if adjoint else
            ["--workload", workload, "--steps", "3", "--warmup", "1", "--no-adjoint"])
    cmd = [exe, "--pmc", counter, "--output-format", "csv", "-d", outdir, "-o",
           counter.lower() + ("_adj" if adjoint else ""), "--", sys.executable,
           os.path.abspath(__file__)] + what + ["--no-others", "--no-cpu-baseline",
                                               "--traffic", "off"]
    env = dict(os.environ, TMPDIR=os.environ.get("TMPDIR", "/tmp"))
    proc = subprocess.Popen(cmd, cwd="/tmp", env=env, stdout=subprocess.PIPE,
                            stderr=subprocess.STDOUT, text=True, start_new_session=True)
    try:
        out, _ = proc.communicate(timeout=timeout)
    except subprocess.TimeoutExpired:
        os.killpg(proc.pid, signal.SIGKILL)
        proc.communicate()
        raise RuntimeError("%s pass timed out" % counter)
    files = glob.glob(os.path.join(outdir, "**", "%s%s_counter_collection.csv"
                                   % (counter.lower(), "_adj" if adjoint else "")),
                      recursive=True)
    # the profiler may end with a non-zero status after the program's
    # results are complete: accept the run when the child printed its line
    if not files or '"metric"' not in out:
        raise RuntimeError("%s pass failed (status %s)" % (counter, proc.returncode))
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _step_kernel_kib(rows):
    """Sum of the counter over the step-kernel dispatches, the number of
    steps they make (even launches plus odd steps, counted by the widest odd
    launch) and the copy probe's mean value per dispatch."""
    total, even, odd, copies = 0.0, 0, {}, []
    for r in rows:
        name, v = r["Kernel_Name"], float(r["Counter_Value"])
        grid = r.get("Grid_Size", r.get("Grid_Size_X", "0"))
        if "copy_kernel" in name:
            copies.append(v)
            continue
        m = re.search(r"step_kernel<[^,]+, [^,]+, (true|false)", name)
        if "step_even_pair_kernel<" in name:
            even += 1
        elif m and "level_step" not in name:
            if m.group(1) == "false":
                even += 1
            else:
                odd[int(grid)] = odd.get(int(grid), 0) + 1
        elif "link_kernel" not in name:
            continue
        total += v
    steps = even + (odd[max(odd)] if odd else 0)
    return total, steps, (sum(copies) / len(copies) if copies else None)


def _adjoint_kernel_kib(rows):
    """Per (collision, storage) of the adjoint kernel: the counter summed
    over its dispatches and the adjoint steps they make (the dispatches of
    the widest launch); and the copy probe's mean value per dispatch."""
    acc, copies = {}, []
    for r in rows:
        name, v = r["Kernel_Name"], float(r["Counter_Value"])
        if "copy_kernel" in name:
            copies.append(v)
            continue
        m = re.search(r"adjoint_kernel<(\d+), (float|double),", name)
        if not m:
            continue
        key = ("fclb" if m.group(1) == "2" else "mrt", "f32" if m.group(2) == "float" else "f64")
        grid = int(r.get("Grid_Size", r.get("Grid_Size_X", "0")))
        tot, grids = acc.setdefault(key, [0.0, {}])
        acc[key][0] = tot + v
        grids[grid] = grids.get(grid, 0) + 1
    out = {k: (t, g[max(g)]) for k, (t, g) in acc.items()}
    return out, (sum(copies) / len(copies) if copies else None)


def live_adjoint_traffic(timeout=120):
    """HBM bytes per adjoint step of each adjoint leg, from two counter
    passes over a child run of the adjoint legs alone, scaled like
    live_traffic. Returns ({(collision, storage): bytes}, description) or
    (None, reason)."""
    exe = shutil.which("rocprofv3")
    if exe is None:
        return None, "rocprofv3 not available"
    outdir = tempfile.mkdtemp(prefix="lbm_traffic_adj_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        per = {}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            print("bench: adjoint traffic pass", counter, flush=True)
            legs, copy_kib = _adjoint_kernel_kib(
                _run_counter_pass(exe, counter, None, outdir, timeout, adjoint=True))
            if not legs or not copy_kib:
                return None, "no adjoint or copy dispatches in the %s pass" % counter
            scale = (COPY_BYTES / 1024.0) / copy_kib
            for k, (tot, steps) in legs.items():
                per[k] = per.get(k, 0.0) + tot * scale * 1024.0 / steps
        return per, ("measured in this run: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE over a "
                     "child run of the adjoint legs, scaled by the copy kernel's ratios")
    except (RuntimeError, OSError, KeyError, ValueError) as e:
        return None, str(e)
    finally:
        shutil.rmtree(outdir, ignore_errors=True)


def live_traffic(workload, timeout=120):
    """HBM bytes per step of the workload's step kernels (and link kernel),
    from two counter passes (FETCH_SIZE, then WRITE_SIZE) over a short child
    run, each scaled by what the counter reads for the copy kernel of known
    size in the same run. Runs before this process touches the GPU. Returns
    (bytes per step, description) or (None, reason)."""
    exe = shutil.which("rocprofv3")
    if exe is None:
        return None, "rocprofv3 not available"
    outdir = tempfile.mkdtemp(prefix="lbm_traffic_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        parts = {}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            print("bench: traffic pass", counter, flush=True)
            total, steps, copy_kib = _step_kernel_kib(
                _run_counter_pass(exe, counter, workload, outdir, timeout))
            if steps == 0 or not copy_kib:
                return None, "no step or copy dispatches in the %s pass" % counter
            scale = (COPY_BYTES / 1024.0) / copy_kib
            parts[counter] = (total * scale * 1024.0 / steps, scale, steps)
        f, w = parts["FETCH_SIZE"], parts["WRITE_SIZE"]
        return f[0] + w[0], ("measured in this run: rocprofv3 --pmc FETCH_SIZE (x%.3f) and "
                             "WRITE_SIZE (x%.3f, the copy kernel's ratios) over %d steps of "
                             "a child run" % (f[1], w[1], f[2]))
    except (RuntimeError, OSError, KeyError, ValueError) as e:
        return None, str(e)
    finally:
        shutil.rmtree(outdir, ignore_errors=True)


def kind_refined(name):
    return name.split("-")[0].startswith("ref")


def workload(name):
    """(model, storage, shape, kind) from a name like jet256-fclb-f32."""
    kind, model, storage = name.split("-")
    shapes = {"jet256": (256, 256, 512), "tgv256": (256, 256, 512), "tgv128": (128, 128, 128),
              "jet128": (128, 128, 256), "ref128": (128, 128, 256), "ref3l128": (128, 128, 256),
              "nozzle256": (256, 256, 512), "nozzlecurved256": (256, 256, 512)}
    return model, storage, shapes[kind], kind


def refined_jet_mask(nx, ny, nz, B=16, layers=8, radius=62.0):
    """Blocks of the first `layers` streamwise block layers whose centre lies
    within `radius` coarse nodes of the jet axis."""
    import numpy as np
    m = np.zeros((nz // B, ny // B, nx // B), dtype=np.uint8)
    for bz in range(layers):
        for by in range(ny // B):
            for bx in range(nx // B):
                cx, cy = (bx + 0.5) * B - nx / 2, (by + 0.5) * B - ny / 2
                if cx * cx + cy * cy <= radius * radius:
                    m[bz, by, bx] = 1
    return m


def jet_setup(nx, ny, synth):
    """Boundary data of the round-jet workloads (side walls moving with the
    co-flow, velocity inlet at z-, zero-gradient outflow at z+)."""
    diam = 32.0 if nx >= 256 else 16.0
    iu, im = synth.jet_inlet(nx, ny, diam, 0.05, 0.002)
    return {"nu": 1e-4, "cs": 0.1, "diameter": diam, "inlet_u": iu, "inlet_mask": im,
            "face_u": [[0.0, 0.0, 0.002]] * 4 + [[0.0, 0.0, 0.0]] * 2,
            "inlet_amp": 0.01 * 0.05, "seed": 12060389}


def nozzle_mask(nx, ny, nz, diameter, wall=2, length=16):
    """Solid tube around the inlet disk: nodes whose distance from the jet
    axis lies in [D/2, D/2 + wall) on the first `length` planes."""
    import numpy as np
    y, x = np.mgrid[0:ny, 0:nx]
    r = np.hypot(x + 0.5 - nx / 2.0, y + 0.5 - ny / 2.0)
    ring = (r >= diameter / 2.0) & (r < diameter / 2.0 + wall)
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:length] = ring
    return m


def make_lattice(name, P, torch, synth):
    import numpy as np
    model, storage, shape, kind = workload(name)
    nx, ny, nz = shape
    if kind in ("ref128", "ref3l128"):
        nu, cs, B = 1e-4, 0.1, 16
        levels = 2 if kind == "ref128" else 3
        lmap = refined_jet_mask(nx, ny, nz, B)
        if levels == 3:
            lmap = lmap + refined_jet_mask(nx, ny, nz, B, layers=4, radius=34.0)
        iu, im = synth.jet_inlet(nx, ny, 16.0, 0.05, 0.002)
        lius, lims = [None], [None]
        for l in range(1, levels):
            a, b = synth.jet_inlet(nx << l, ny << l, 16.0 * 2 ** l, 0.05, 0.002)
            lius.append(torch.from_numpy(a))
            lims.append(torch.from_numpy(b))
        fu = [[0.0, 0.0, 0.002]] * 4 + [[0.0, 0.0, 0.0]] * 2
        lat = P.RefinedLattice(model=model, storage=storage, shape=shape, nu=nu, cs_smag=cs,
                               block=B, level_map=lmap, nlevels=levels,
                               faces=[P.WALL] * 4 + [P.INLET, P.OUTFLOW], face_u=fu,
                               inlet_u=torch.from_numpy(iu), inlet_mask=torch.from_numpy(im),
                               level_inlet_u=lius, level_inlet_mask=lims, inlet_amp=5e-4,
                               seed=12060389)
        for level in range(levels):
            d, u = synth.uniform_fields(*lat.shape3(level)[::-1], u=(0.0, 0.0, 0.002),
                                        dtype=np.float32)
            lat.init_equilibrium(level, torch.from_numpy(d), torch.from_numpy(u))
        # node updates per level-0 step: level l updates its fluid and band
        # nodes 2^l times
        per = [v["counts"]["fluid"] + v["counts"]["band"] for v in lat.levels]
        ups = sum(n_l << l for l, n_l in enumerate(per))
        desc = {"workload": "%d-level refined round jet, level 0 %dx%dx%d, 16^3 blocks, level map "
                            "%s blocks at levels 1..%d (level 1: layers 0-7, centre radius <= 62%s), "
                            "D=16 at level 0 inlet u=0.05 +1%% perturbation, co-flow 0.002, "
                            "nu_0=1e-4"
                            % (levels, nx, ny, nz,
                               "/".join(str(int((lmap >= l).sum())) for l in range(1, levels)),
                               levels - 1, "; level 2: layers 0-3, radius <= 34"
                               if levels == 3 else ""),
                "collision": model, "storage": storage, "nx": nx, "ny": ny, "nz": nz,
                "updated_nodes_per_level": per, "ghost_nodes_per_level":
                    [v["counts"]["ghost"] for v in lat.levels],
                "covered_per_level": [v["counts"]["covered"] for v in lat.levels],
                "updates_per_level0_step": ups,
                "cs_smag": cs if model == "mrt" else None}
        lat.updates_per_step = ups
        return lat, desc
    if kind.startswith("jet") or kind.startswith("nozzle"):
        js = jet_setup(nx, ny, synth)
        nu, cs, diam = js["nu"], js["cs"], js["diameter"]
        lat = P.Lattice(model=model, storage=storage, shape=shape, nu=nu, cs_smag=cs)
        faces = [P.WALL, P.WALL, P.WALL, P.WALL, P.INLET, P.OUTFLOW]
        lat.set_boundaries(faces, face_u=js["face_u"], inlet_u=torch.from_numpy(js["inlet_u"]),
                           inlet_mask=torch.from_numpy(js["inlet_mask"]),
                           inlet_amp=js["inlet_amp"], seed=js["seed"])
        d, u = synth.uniform_fields(nx, ny, nz, u=(0.0, 0.0, 0.002), dtype=np.float32)
        extra = ""
        if kind.startswith("nozzle"):
            sm = nozzle_mask(nx, ny, nz, diam)
            lat.set_solids(torch.from_numpy(sm))
            extra = ", solid nozzle tube (wall 2, length 16, %d solid nodes)" % int(sm.sum())
        if kind == "nozzlecurved256":
            # the tube's round surfaces as curved walls: wall distances of
            # every fluid-solid link, found in a box around the tube
            m = int(diam) // 2 + 4
            box = (18, 2 * m, 2 * m)
            org = (nx // 2 - m, ny // 2 - m, 0)
            _, nodes, q = synth.link_distances(synth.nozzle_tube(nx, ny, diam, 2.0, 16.0), box,
                                               P.VELOCITIES[:lat.Q], origin=org,
                                               full_shape=(nz, ny, nx))
            lat.set_links(torch.from_numpy(nodes), torch.from_numpy(q))
            extra += ", interpolated bounce-back on %d nodes" % len(nodes)
        desc = {"workload": "round jet %dx%dx%d, D=%d inlet u=0.05 +1%% seeded perturbation, "
                            "co-flow 0.002 moving side walls, zero-gradient outflow, nu=1e-4%s"
                            % (nx, ny, nz, int(diam), extra),
                "collision": model, "storage": storage, "nx": nx, "ny": ny, "nz": nz,
                "cs_smag": cs if model == "mrt" else None}
    else:
        nu, cs = (4.0e-3 if nx == 128 else 1e-3), 0.1
        lat = P.Lattice(model=model, storage=storage, shape=shape, nu=nu, cs_smag=cs)
        d, u = synth.taylor_green((nx, ny, nz), 0.05)
        d, u = d.astype(np.float32), u.astype(np.float32)
        desc = {"workload": "periodic Taylor-Green %dx%dx%d, u0=0.05, nu=%g" % (nx, ny, nz, nu),
                "collision": model, "storage": storage, "nx": nx, "ny": ny, "nz": nz,
                "cs_smag": cs if model == "mrt" else None}
    lat.init_equilibrium(torch.from_numpy(d), torch.from_numpy(u))
    del d, u
    return lat, desc


def time_steps(lat, torch, steps, warmup, windows=5):
    """ms per step: the median over `windows` consecutive windows that split
    the K timed steps (HIP events on the kernels' stream at each window
    boundary; one synchronisation before and after the K steps)."""
    stream = torch.cuda.current_stream()
    lat.step(warmup)
    torch.cuda.synchronize()
    windows = max(1, min(windows, steps))
    sizes = [steps // windows + (1 if k < steps % windows else 0) for k in range(windows)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(windows + 1)]
    ev[0].record(stream)
    for k, n in enumerate(sizes):
        lat.step(n)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) / sizes[k] for k in range(windows))
    total = ev[0].elapsed_time(ev[windows]) / steps
    return per[len(per) // 2], {"windows": windows, "ms_per_step_windows": per,
                                "ms_per_step_mean": total}


def measure(name, P, torch, synth, steps, warmup):
    lat, desc = make_lattice(name, P, torch, synth)
    ms, spread = time_steps(lat, torch, steps, warmup)
    red = lat.reduce(check=False)
    model, storage, shape, _ = workload(name)
    q = 19 if model == "mrt" else 27
    n = getattr(lat, "updates_per_step", shape[0] * shape[1] * shape[2])
    alg_bytes = 2 * q * BYTES[storage] * n
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    out = {"name": name, "mlups": n / (ms * 1e-3) / 1e6, "ms_per_step": ms,
           "achieved_GBs": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS,
           "bytes_per_lup": 2 * q * BYTES[storage], "finite": all(map(lambda v: v == v, red)),
           "timing": spread, "config": desc}
    # populations that fit the 256 MB last-level cache are not an HBM figure
    pop_bytes = q * BYTES[storage] * shape[0] * shape[1] * shape[2]
    if not kind_refined(name) and pop_bytes < LLC_BYTES:
        out["note"] = ("populations (%.0f MB) fit the %d MB last-level cache: the rate is "
                       "not bound by HBM" % (pop_bytes / 1e6, LLC_BYTES // (1 << 20)))
    del lat
    torch.cuda.empty_cache()
    return out


def measure_adjoint(P, torch, synth, storage="f32", steps=50, model="fclb"):
    """Inlet-sensitivity gradient of the 128 x 128 x 256 jet (D = 16, u =
    0.05, nu = 2e-4, co-flow 0.002), 400 steps from rest with checkpoints
    every 20, u_z perturbed on the 16 x 16 nozzle square (N(0, 0.005^2), seed
    389), J = mean kinetic energy of the 32^3 probe at z in [80, 112).
    model: "fclb" (D3Q27 FCLB) or "mrt" (D3Q19 MRT-LES, Table 1 basis, C_S =
    0.1)."""
    from paper_1206_0389_amd.adjoint import InletProbeObjective
    n, nz, d, nsteps = 128, 256, 16, 400
    c = synth.jet_adjoint_case(n, nz, d, u_jet=0.05, u_coflow=0.002, sigma=0.005, seed=389)
    fu = [[0.0, 0.0, 0.002]] * 4 + [[0.0, 0.0, 0.0]] * 2
    cs = 0.1 if model == "mrt" else 0.0
    lat = P.Lattice(model=model, storage=storage, shape=(n, n, nz), nu=2e-4, cs_smag=cs)
    Q = lat.Q
    obj = InletProbeObjective(lat, [P.WALL] * 4 + [P.INLET, P.OUTFLOW], fu,
                              torch.from_numpy(c["base_u"]), c["square"], c["probe_lo"],
                              c["probe_hi"], nsteps, every=20)
    delta = torch.from_numpy(c["delta"]).cuda()
    obj.forward(delta)
    obj.backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = obj.forward(delta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grad, _ = obj.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    b0, b1, a0, a1 = c["square"]
    gnorm = float(grad[2, b0:b1, a0:a1].norm())
    # the adjoint step kernel alone, on recorded states
    f = obj._rec[0]
    lam = obj._rec[1].clone()
    lam2 = torch.empty_like(lam)
    g = torch.zeros_like(grad)
    stream = torch.cuda.current_stream()
    for _ in range(5):
        lat.adjoint_step(f, lam, lam2, g)
        lam, lam2 = lam2, lam
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        lat.adjoint_step(f, lam, lam2, g)
        lam, lam2 = lam2, lam
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nodes = n * n * nz
    bpn = 3 * Q * (8 if storage == "f64" else 4)
    gbs = bpn * nodes / (ms * 1e-3) / 1e9
    name = "FCLB" if model == "fclb" else "MRT-LES (C_S 0.1)"
    out = {"workload": "inlet-sensitivity jet 128x128x256 %s, D=16 u=0.05 nu=2e-4, 400 "
                       "steps, checkpoints every 20, 16x16 u_z perturbation (sigma 0.005, seed "
                       "389), probe 32^3 at z in [80,112)" % name,
           "collision": model, "storage": storage, "J": J, "grad_l2": gnorm, "gradient_s": t2 - t0,
           "forward_s": t1 - t0, "backward_s": t2 - t1, "adjoint_step_ms": ms,
           "adjoint_mlups": nodes / (ms * 1e-3) / 1e6, "adjoint_bytes_per_node": bpn,
           "adjoint_GBs": gbs, "adjoint_frac_of_8TBs": gbs / HBM_PEAK_GBS,
           "kernel": "adjoint_kernel<%s>" % ("double" if storage == "f64" else "float"),
           "traffic": (MEASURED_ADJOINT_TRAFFIC["bytes_per_step"][model]
                       if (MEASURED_ADJOINT_TRAFFIC["storage"] == storage and
                           MEASURED_ADJOINT_TRAFFIC["sources_sha256_16"] ==
                           sources_hash(ADJOINT_SOURCES)) else None)}
    del obj, lat, f, lam, lam2, g
    torch.cuda.empty_cache()
    return out


def measure_stats(P, torch, synth, name="jet256-fclb-f32", reps=50):
    """Velocity time-average accumulation on the default workload: per call
    Q b bytes of populations read and 6 FP64 running sums read and written."""
    lat, desc = make_lattice(name, P, torch, synth)
    sums = lat.stats_buffer()
    lat.stats_accumulate(sums)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lat.stats_accumulate(sums)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    model, storage, shape, _ = workload(name)
    n = shape[0] * shape[1] * shape[2]
    per_node = (27 if model == "fclb" else 19) * BYTES[storage] + 2 * 6 * 8
    gbs = per_node * n / (ms * 1e-3) / 1e9
    # the jet's spreading (Eqs. (23)-(24)) from the mean: 32 rays x 64 radii
    # on each of the 512 cross-sections
    mean, rms, _ = lat.stats_finalize(sums, reps + 1)
    del rms
    lat.jet_profile(mean, ndir=32, dr=0.5, nr=64)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        _, re, _ = lat.jet_profile(mean, ndir=32, dr=0.5, nr=64)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_prof = e0.elapsed_time(e1) / 10
    del lat, sums, mean
    torch.cuda.empty_cache()
    return {"name": name + "-stats", "kernel": "stats_accumulate_kernel", "ms_per_call": ms,
            "bytes_per_node": per_node, "achieved_GBs": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS,
            "jet_profile_ms": ms_prof, "jet_profile": "32 rays x 64 radii (dr 0.5) on 512 sections"}


def copy_bandwidth(P, torch, nbytes=4 << 30, reps=10):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    P.stream_copy(b, a, nbytes)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.stream_copy(b, a, nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def cpu_baseline(model_name, target_s=10.0):
    """The FP64 oracle on the host, on a 64^3 cut-down of the jet: all the
    cores this process may use, then a single core (OpenMP team size)."""
    import oracle
    import synth
    cores = len(os.sched_getaffinity(0))
    model = oracle.FCLB27 if model_name == "fclb" else oracle.MRT19
    n = 64
    iu, im = synth.jet_inlet(n, n, 8.0, 0.05, 0.002)
    fu = [[0.0, 0.0, 0.002]] * 4 + [[0.0, 0.0, 0.0]] * 2
    lat = oracle.Lattice(model, n, n, n, nu=1e-4, cs_smag=0.1,
                         faces=[oracle.WALL] * 4 + [oracle.INLET, oracle.OUTFLOW], face_u=fu,
                         inlet_u=iu, inlet_mask=im, inlet_amp=5e-4, seed=12060389)
    d, u = synth.uniform_fields(n, n, n, u=(0.0, 0.0, 0.002))
    f0 = lat.init_equilibrium(d, u)
    res = {}
    for label, threads in (("all", cores), ("single", 1)):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        f = lat.run(f0, 0, 1)
        per = time.perf_counter() - t0
        steps = max(1, min(200, int(target_s / max(per, 1e-3))))
        t0 = time.perf_counter()
        lat.run(f, 1, steps)
        dt = time.perf_counter() - t0
        res[label] = (n ** 3 * steps / dt / 1e6, steps, dt, oracle.max_threads())
    oracle.set_threads(cores)
    (v_all, s_all, dt_all, c_all), (v_one, s_one, dt_one, _) = res["all"], res["single"]
    return {"value": v_all, "unit": "MLUPS", "cores": c_all, "kind": "oracle",
            "single_core_value": v_one, "cpu_model": cpu_model(),
            "sample": "FP64 oracle, %s, jet cut-down %d^3 (D=8): %d steps in %.1f s on %d "
                      "threads; %d steps in %.1f s on 1 thread"
                      % (model_name, n, s_all, dt_all, c_all, s_one, dt_one)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    live, live_adj = (None, "off"), (None, "off")
    if args.traffic == "auto" and not args.only_adjoint:
        # child runs, before this process uses the GPU
        if not kind_refined(args.workload):
            live = live_traffic(args.workload)
        # a pass that timed out is not tried again (a normal pass takes seconds)
        if not args.no_adjoint and "timed out" not in str(live[1]):
            live_adj = live_adjoint_traffic()
    import torch
    import paper_1206_0389_amd as P
    import synth

    torch.cuda.set_device(0)
    if args.only_adjoint:
        legs = [measure_adjoint(P, torch, synth, st) for st in ("f32", "f64")]
        legs.append(measure_adjoint(P, torch, synth, "f32", model="mrt"))
        copy_bandwidth(P, torch)
        print(json.dumps({"metric": METRIC, "adjoint": legs}), flush=True)
        return
    print("bench: workload", args.workload, flush=True)
    main_res = measure(args.workload, P, torch, synth, args.steps, args.warmup)
    print("bench: main done %.1f MLUPS" % main_res["mlups"], flush=True)
    others = []
    if not args.no_others:
        for name in ["jet256-fclb-f16", "jet256-fclb-f64", "jet256-clb-f32", "jet256-mrt-f32",
                     "jet256-mrt-f16",
                     "jet256-mrt-f64", "tgv256-fclb-f32", "tgv256-mrt-f32", "tgv256-mrt-f16",
                     "tgv256-mrt-f64", "tgv128-fclb-f32", "tgv128-mrt-f32", "ref128-fclb-f32",
                     "ref128-fclb-f16", "ref128-mrt-f32", "ref128-mrt-f16", "ref3l128-fclb-f32", "nozzle256-fclb-f32", "nozzlecurved256-fclb-f32"]:
            if name == args.workload:
                continue
            r = measure(name, P, torch, synth, args.other_steps, 10)
            print("bench: %s %.1f MLUPS" % (name, r["mlups"]), flush=True)
            others.append(r)
    adjoint = None
    if not args.no_adjoint:
        adjoint = [measure_adjoint(P, torch, synth, st) for st in ("f32", "f64")]
        adjoint.append(measure_adjoint(P, torch, synth, "f32", model="mrt"))
        for a in adjoint:
            key = (a["collision"], a["storage"])
            if live_adj[0] is not None and key in live_adj[0]:
                a["traffic"], a["traffic_source"] = live_adj[0][key], live_adj[1]
            elif a["traffic"] is not None:
                a["traffic_source"] = ("stored counter passes of these sources (live "
                                       "measurement: %s)" % live_adj[1])
        print("bench: adjoint gradient %.2f s (f32)" % adjoint[0]["gradient_s"], flush=True)
    stats = measure_stats(P, torch, synth) if not args.no_others else None
    copy_gbs = copy_bandwidth(P, torch)
    model, storage, shape, kind = workload(args.workload)
    refined = kind.startswith("ref")
    # a refined coarse step is a sequence of launches on several streams: its
    # algorithmic bytes are those of every node update of the step
    alg_per_launch = main_res["bytes_per_lup"] * (
        main_res["config"]["updates_per_level0_step"] if refined else
        shape[0] * shape[1] * shape[2])
    roof = {"bound": "hbm", "achieved": main_res["achieved_GBs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": main_res["achieved_GBs"] / HBM_PEAK_GBS,
            "traffic": None,
            "traffic_unit": "bytes per step (one even launch, or the two odd launches)",
            "kernel": ("refined coarse step (level steps and interface kernels) <%s,%s>"
                       if refined else "step_kernel<%s,%s>") % (model, storage),
            "algorithmic_bytes_per_launch": alg_per_launch,
            "copy_probe_GBs": copy_gbs,
            "frac_of_copy_probe": main_res["achieved_GBs"] / copy_gbs}
    stored_ok = (MEASURED_TRAFFIC["sources_sha256_16"] == sources_hash()
                 and MEASURED_TRAFFIC["workload"] == args.workload)
    if live[0] is not None:
        roof["traffic"], roof["traffic_source"] = live[0], live[1]
    elif stored_ok:
        roof["traffic"] = MEASURED_TRAFFIC["bytes_per_step"]
        roof["traffic_source"] = ("stored counter passes of these sources (hash %s; live "
                                  "measurement: %s)" % (sources_hash(), live[1]))
    else:
        roof["traffic_source"] = "not measured (%s)" % live[1]
    line = {"metric": METRIC, "value": main_res["mlups"], "unit": "MLUPS", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_res["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": storage, "data": "synthetic", "config": main_res["config"],
            "roofline": roof, "timing": main_res["timing"], "others": others,
            "adjoint": adjoint, "statistics": stats}
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", flush=True)
        line["cpu_baseline"] = cpu_baseline(model)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
