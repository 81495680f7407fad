"""Write the stored FP64 CPU adjoint of the cut-down inlet-sensitivity jet.

    python tests/golden/make_adjoint_jet.py [--fd] [--model mrt]

Calls only the oracle (and the seeded input generators). The case is the
128 x 128 x 256 round jet of the inlet-sensitivity study with every length
divided by four: a 32 x 32 x 64 FCLB lattice, nozzle diameter 4 at
u = 0.05 on the z- face, co-flow 0.002 (inlet outside the disk and the side
walls moving with it), zero-gradient outflow at z+, nu = 2e-4, 400 steps from
rest, a static N(0, 0.005^2) perturbation of u_z (seed 389) on the 4 x 4
square around the nozzle, and J = mean |j|^2 / (2 rho) over the 8^3 probe
x, y in [12, 20), z in [20, 28) after the last step.

The file holds J and dJ/du on the 4 x 4 square for each velocity component.
With --fd it also checks the z-components against central differences of J
(h = 1e-6) and records them. --model mrt writes the same case for the D3Q19
MRT-LES model (Table 1 basis, C_S = 0.1) into adjoint_jet_mrt_32x32x64.txt.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = {"fclb": os.path.join(HERE, "adjoint_jet_32x32x64.txt"),
       "mrt": os.path.join(HERE, "adjoint_jet_mrt_32x32x64.txt")}
N, NZ, D, NSTEPS, NU, COFLOW = 32, 64, 4, 400, 2e-4, 0.002
MODEL = "fclb"


def case():
    c = synth.jet_adjoint_case(N, NZ, D, u_jet=0.05, u_coflow=COFLOW, sigma=0.005, seed=389)
    face_u = [[0.0, 0.0, COFLOW] for _ in range(4)] + [[0.0, 0.0, 0.0]] * 2
    return c, face_u


def lattice(inlet_u, face_u):
    W, I, O = oracle.WALL, oracle.INLET, oracle.OUTFLOW
    model, cs = (oracle.FCLB27, 0.0) if MODEL == "fclb" else (oracle.MRT19, 0.1)
    return oracle.Lattice(model, N, N, NZ, nu=NU, cs_smag=cs, basis=oracle.BASIS_TABLE1,
                          faces=[W, W, W, W, I, O], face_u=face_u, inlet_u=inlet_u)


def objective(inlet_u, face_u, c):
    lat = lattice(inlet_u, face_u)
    f = lat.run(np.zeros((lat.Q, NZ, N, N)), 0, NSTEPS)
    return lat.probe_ke(f, c["probe_lo"], c["probe_hi"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fd", action="store_true")
    ap.add_argument("--model", choices=["fclb", "mrt"], default="fclb")
    args = ap.parse_args()
    global MODEL
    MODEL = args.model
    oracle.build(force=False)
    c, face_u = case()
    t0 = time.time()
    lat = lattice(c["inlet_u"], face_u)
    J, grad, _ = lat.inlet_gradient(np.zeros((lat.Q, NZ, N, N)), 0, NSTEPS, c["probe_lo"],
                                    c["probe_hi"], every=20)
    print(f"adjoint done in {time.time() - t0:.0f} s, J = {J:.17e}", flush=True)
    b0, b1, a0, a1 = c["square"]
    g = grad[:, b0:b1, a0:a1]
    name = "FCLB" if MODEL == "fclb" else "MRT-LES (Table 1 basis, C_S = 0.1)"
    lines = [f"# FP64 CPU adjoint (oracle) of the cut-down inlet-sensitivity jet, {name},",
             "# written by tests/golden/make_adjoint_jet.py"
             + ("" if MODEL == "fclb" else " --model mrt")
             + "; see its docstring for the case.",
             f"J {J:.17e}"]
    for comp in range(3):
        for b in range(D):
            lines.append(f"grad {comp} {b} " + " ".join(f"{v:.17e}" for v in g[comp, b]))
    if args.fd:
        h = 1e-6
        fd = np.zeros((D, D))
        for b in range(D):
            for a in range(D):
                up, um = c["inlet_u"].copy(), c["inlet_u"].copy()
                up[2, b0 + b, a0 + a] += h
                um[2, b0 + b, a0 + a] -= h
                fd[b, a] = (objective(up, face_u, c) - objective(um, face_u, c)) / (2 * h)
                print(f"fd {b} {a} {fd[b, a]:.6e} adjoint {g[2, b, a]:.6e}", flush=True)
        rel = float(np.linalg.norm(fd - g[2]) / np.linalg.norm(fd))
        print(f"relative L2 difference adjoint vs FD: {rel:.3e}", flush=True)
        assert rel <= 1e-6, rel
        for b in range(D):
            lines.append(f"fd 2 {b} " + " ".join(f"{v:.17e}" for v in fd[b]))
    with open(OUT[MODEL], "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT[MODEL])


if __name__ == "__main__":
    main()
