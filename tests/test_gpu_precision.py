"""Per-field error of FP32 and FP16 deviation storage.

Against the FP64 oracle directly: 32^3 Taylor-Green vortex, 100 steps, both
models. At the 128^3 size of the Taylor-Green workload (u0 = 0.05, Re = 1600
on the 128 wavelength: nu = 4e-3), 100 and 2000 steps, against FP64 storage
on the GPU, whose steps match the oracle to 1e-12 (test_gpu_parity.py).

Errors are stated per field (density deviation and each velocity component)
as max |error| / max |FP64 field| and as relative L2. Bounds: FP32 stores the
deviation f - w with 2^-24 relative rounding and computes in FP32, so the
fields carry a few units of 1e-7 relative error per step, growing at most
linearly with the step count; FP16 rounds the deviation to 2^-11 relative,
a few 1e-4 per step, partly averaged out over the populations of a node.
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import gpu_lattice, oracle_lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

FIELDS = ("drho", "ux", "uy", "uz")


def _fields(drho, u):
    return {"drho": drho, "ux": u[0], "uy": u[1], "uz": u[2]}


def _errors(got, ref):
    out = {}
    scale_u = max(float(np.abs(ref[k]).max()) for k in ("ux", "uy", "uz"))
    for k in FIELDS:
        scale = float(np.abs(ref[k]).max()) if k == "drho" else scale_u
        d = got[k] - ref[k]
        out[k] = (float(np.abs(d).max()) / scale,
                  float(np.linalg.norm(d) / max(np.linalg.norm(ref[k]), 1e-300)))
    return out


def _gpu_fields(name, storage, n, nu, steps, cs=0.1):
    drho, u = synth.taylor_green(n, 0.05)
    g = gpu_lattice(name, storage, (n, n, n), nu, cs=cs)
    g.init_equilibrium(torch.from_numpy(drho), torch.from_numpy(u))
    out = {}
    done = 0
    for s in steps:
        g.step(s - done)
        done = s
        d, v = g.macroscopic()
        out[s] = _fields(d.cpu().numpy(), v.cpu().numpy())
    return out


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
def test_reduced_storage_vs_oracle_tgv32(name):
    n, nu, steps = 32, 0.005, 100
    print("case precision vs oracle", name, flush=True)
    drho, u = synth.taylor_green(n, 0.05)
    o = oracle_lattice(name, (n, n, n), nu, cs=0.1)
    f = o.run(o.init_equilibrium(drho, u), 0, steps)
    ref = _fields(*o.macroscopic(f))
    bounds = {"f32": 1e-5, "f16": 2e-2}
    for storage, bound in bounds.items():
        got = _gpu_fields(name, storage, n, nu, [steps])[steps]
        err = _errors(got, ref)
        print(name, storage, "32^3 step 100 vs oracle (max rel, L2 rel):",
              {k: ("%.2e" % a, "%.2e" % b) for k, (a, b) in err.items()}, flush=True)
        for k in FIELDS:
            assert err[k][0] <= bound, (storage, k, err[k])


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
def test_reduced_storage_tgv128(name):
    n, nu = 128, 4e-3
    steps = [100, 2000]
    print("case precision 128^3", name, flush=True)
    ref = _gpu_fields(name, "f64", n, nu, steps)
    bounds = {("f32", 100): 2e-5, ("f32", 2000): 2e-4, ("f16", 100): 3e-2, ("f16", 2000): 6e-2}
    for storage in ("f32", "f16"):
        got = _gpu_fields(name, storage, n, nu, steps)
        for s in steps:
            err = _errors(got[s], ref[s])
            print(name, storage, "128^3 step", s, "vs FP64 (max rel, L2 rel):",
                  {k: ("%.2e" % a, "%.2e" % b) for k, (a, b) in err.items()}, flush=True)
            for k in FIELDS:
                assert err[k][0] <= bounds[(storage, s)], (storage, s, k, err[k])
