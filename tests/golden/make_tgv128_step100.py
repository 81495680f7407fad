"""Write the FP64 CPU reference of the 128^3 Taylor-Green case at step 100.

    python tests/golden/make_tgv128_step100.py

Calls only the oracle (and the seeded input generators). The case: 128^3
periodic box, Taylor-Green vortex of amplitude u0 = 0.05 (Re 1600 on the
128-node wavelength: nu = 4e-3), equilibrium start, Smagorinsky constant
0.1 for MRT-LES, 100 steps, for the FCLB and MRT-LES (Table 1 basis)
models. The oracle steps every node; the file keeps, per model, the largest
magnitude of each field over the whole box (the scales of the relative
errors) and the fields at 512 nodes drawn by a seeded generator (numpy
PCG64, seed 1206), which the GPU run is compared with.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import synth  # noqa: E402
from lbm_cases import oracle_lattice  # noqa: E402

N, NU, U0, STEPS, NSAMPLE, SEED = 128, 4e-3, 0.05, 100, 512, 1206


def sample_nodes():
    rng = np.random.default_rng(SEED)
    return rng.integers(0, N, size=(NSAMPLE, 3))  # (x, y, z)


def main():
    out = os.path.join(HERE, "tgv128_step100.txt")
    xyz = sample_nodes()
    lines = ["# FP64 oracle, Taylor-Green 128^3, u0 %.3g, nu %.3g, %d steps" % (U0, NU, STEPS),
             "# per model: 'model <name>', 'scale drho ux uy uz' (max |field| over the box),",
             "# then NSAMPLE lines 'x y z drho ux uy uz'"]
    for name in ("fclb", "mrt_table1"):
        o = oracle_lattice(name, (N, N, N), NU, cs=0.1)
        drho, u = synth.taylor_green(N, U0)
        f = o.run(o.init_equilibrium(drho, u), 0, STEPS)
        d, v = o.macroscopic(f)
        fields = [d, v[0], v[1], v[2]]
        lines.append("model %s" % name)
        lines.append("scale " + " ".join(repr(float(np.abs(a).max())) for a in fields))
        for x, y, z in xyz:
            lines.append("%d %d %d " % (x, y, z) +
                         " ".join(repr(float(a[z, y, x])) for a in fields))
        print(name, "done", flush=True)
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
