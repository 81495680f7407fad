"""Hand-written FCLB and MRT-LES adjoints on the GPU against the oracle's
dual-number adjoint and against finite differences, through the C ABI.

FP64: one adjoint step element by element to 1e-12 relative (rounding order
only), the inlet-gradient terms likewise; the 400-step inlet gradient of the
cut-down jet against the stored oracle gradient to 1e-10 and against central
differences of J (GPU, FP64) to 1e-4. FP32: one step to 2e-5 of the largest
adjoint entry (FP32 rounding of inputs and arithmetic, conditioned like the
forward collision). The MRT-LES adjoint (both bases, C_S = 0.1) to the
same bars, and its multi-step inlet gradient against the oracle's driver.
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC
FACE_U = [[0.0, 0.001, 0.002], [0.0, 0.0, 0.002], [0.001, 0.0, 0.002], [0.0, 0.0, 0.002],
          [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]]
FACE_SETS = {
    "periodic": [P] * 6,
    "jet": [W, W, W, W, I, O],
    "closed": [W] * 6,
    "channel": [P, P, W, W, I, O],
    "walls_z": [P, P, P, P, W, O],
    "x_inlet": [I, W, P, P, W, O],
}
GOLDEN = {m: os.path.join(os.path.dirname(__file__), "golden", f)
          for m, f in (("fclb", "adjoint_jet_32x32x64.txt"),
                       ("mrt", "adjoint_jet_mrt_32x32x64.txt"))}


# name: (library model, oracle model, basis, Smagorinsky constant)
MODELS = {
    "fclb": ("fclb", oracle.FCLB27, oracle.BASIS_TABLE1, 0.0),
    "mrt_table1": ("mrt", oracle.MRT19, oracle.BASIS_TABLE1, 0.1),
    "mrt_dhumieres": ("mrt", oracle.MRT19, oracle.BASIS_DHUMIERES, 0.1),
}


def _pair(faces, shape, storage="f64", nu=0.02, model="fclb"):
    import paper_1206_0389_amd as Pk
    nx, ny, nz = shape
    name, code, basis, cs = MODELS[model]
    print("case adjoint", model, faces, shape, storage, flush=True)
    iu = None
    if I in faces:
        ax = faces.index(I) // 2
        na = ny if ax == 0 else nx
        nb = ny if ax == 2 else nz
        iu = synth.jet_inlet(na, nb, 2.0, 0.05, 0.002)[0]
    g = Pk.Lattice(model=name, storage=storage, shape=shape, nu=nu, cs_smag=cs, mrt_basis=basis)
    if faces != [P] * 6:
        g.set_boundaries(faces, face_u=FACE_U,
                         inlet_u=None if iu is None else torch.from_numpy(iu))
    o = oracle.Lattice(code, nx, ny, nz, nu=nu, faces=faces, face_u=FACE_U, inlet_u=iu,
                       cs_smag=cs, basis=basis)
    return g, o, iu


@pytest.mark.parametrize("model", list(MODELS))
@pytest.mark.parametrize("faces", list(FACE_SETS))
@pytest.mark.parametrize("shape", [(6, 5, 7), (37, 9, 11), (300, 3, 4)])
def test_adjoint_step_parity_fp64(faces, shape, model):
    g, o, iu = _pair(FACE_SETS[faces], shape, model=model)
    nx, ny, nz = shape
    f = synth.random_populations(g.Q, (nz, ny, nx), 1e-2, seed=8)
    ln = synth.random_populations(g.Q, (nz, ny, nx), 1.0, seed=9)
    gshape = (3,) + (iu.shape[1:] if iu is not None else (1, 1))
    go = np.zeros(gshape)
    ref = o.adjoint_step(f, ln, go)
    ft, lt = torch.from_numpy(f).cuda(), torch.from_numpy(ln).cuda()
    out = torch.empty_like(ft)
    gg = torch.zeros(gshape, dtype=torch.float64, device="cuda")
    g.adjoint_step(ft, lt, out, gg if iu is not None else None)
    err = float(np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max())
    assert err <= 1e-12, err
    if iu is not None:
        gerr = float(np.abs(gg.cpu().numpy() - go).max() / np.abs(go).max())
        assert gerr <= 1e-12, gerr
        # accumulates: a second call adds the same terms
        g.adjoint_step(ft, lt, out, gg)
        assert float(np.abs(gg.cpu().numpy() - 2 * go).max()) <= 1e-12 * np.abs(go).max()


@pytest.mark.parametrize("model", list(MODELS))
@pytest.mark.parametrize("faces", ["jet", "periodic"])
def test_adjoint_step_fp32(faces, model):
    shape = (37, 9, 11)
    g, o, iu = _pair(FACE_SETS[faces], shape, storage="f32", model=model)
    nx, ny, nz = shape
    f = synth.random_populations(g.Q, (nz, ny, nx), 1e-2, seed=10).astype(np.float32)
    ln = synth.random_populations(g.Q, (nz, ny, nx), 1.0, seed=11).astype(np.float32)
    gshape = (3,) + (iu.shape[1:] if iu is not None else (1, 1))
    go = np.zeros(gshape)
    ref = o.adjoint_step(f.astype(np.float64), ln.astype(np.float64), go)
    ft, lt = torch.from_numpy(f).cuda(), torch.from_numpy(ln).cuda()
    out = torch.empty_like(ft)
    gg = torch.zeros(gshape, dtype=torch.float64, device="cuda")
    g.adjoint_step(ft, lt, out, gg if iu is not None else None)
    err = float(np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max())
    print("FP32 adjoint relative error", err, flush=True)
    assert err <= 2e-5, err
    if iu is not None:
        assert float(np.abs(gg.cpu().numpy() - go).max() / np.abs(go).max()) <= 2e-5


@pytest.mark.parametrize("model", ["fclb", "mrt_table1"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_probe_ke_and_seed(storage, model):
    shape = (12, 10, 14)
    g, o, _ = _pair(FACE_SETS["jet"], shape, storage=storage, model=model)
    nx, ny, nz = shape
    f = synth.random_populations(g.Q, (nz, ny, nx), 1e-2, seed=12)
    g.set_populations(torch.from_numpy(f))
    g.step(3)  # odd parity: the probe reads the state through the pull rules
    fo = o.run(f, 0, 3)
    lo, hi = (2, 3, 4), (9, 8, 12)
    dt = g.adjoint_dtype
    lam = torch.empty((g.Q, nz, ny, nx), dtype=dt, device="cuda")
    J = g.probe_ke(lo, hi, lam)
    Jo, lamo = o.probe_ke(fo, lo, hi, grad=True)
    tol = 1e-12 if storage == "f64" else 2e-5
    assert abs(J - Jo) <= tol * Jo
    assert float(np.abs(lam.double().cpu().numpy() - lamo).max()) <= tol * np.abs(lamo).max()


def test_adjoint_rejects_unsupported_cases_and_aliasing():
    import paper_1206_0389_amd as Pk
    # no recording step with FP16 storage (the adjoint needs FP32 or FP64)
    g = Pk.Lattice(model="mrt", storage="f16", shape=(4, 4, 4), nu=0.02)
    with pytest.raises(Pk.LbmError):
        g.step_record(torch.empty((19, 4, 4, 4), dtype=torch.float32, device="cuda"))
    h = Pk.Lattice(model="fclb", storage="f64", shape=(4, 4, 4), nu=0.02)
    f = torch.zeros((27, 4, 4, 4), dtype=torch.float64, device="cuda")
    lam = torch.zeros_like(f)
    with pytest.raises(Pk.LbmError):
        h.adjoint_step(f, lam, lam)
    with pytest.raises(Pk.LbmError):
        h.probe_ke((0, 0, 0), (5, 4, 4))
    # no adjoint through free-slip faces
    h.set_boundaries([Pk.FREESLIP] * 2 + [Pk.PERIODIC] * 4)
    with pytest.raises(Pk.LbmError):
        h.adjoint_step(f, lam, torch.empty_like(f))
    with pytest.raises(Pk.LbmError):
        h.step_record(torch.empty_like(f))
    # no adjoint of the CLB variant either
    c = Pk.Lattice(model="clb", storage="f64", shape=(4, 4, 4), nu=0.02)
    with pytest.raises(Pk.LbmError):
        c.adjoint_step(f, lam, torch.empty_like(f))
    with pytest.raises(Pk.LbmError):
        c.step_record(torch.empty_like(f))
    # nor through fixed-pressure faces
    h.set_boundaries([Pk.PRESSURE] * 2 + [Pk.PERIODIC] * 4, face_drho=[0.001] * 6)
    with pytest.raises(Pk.LbmError):
        h.adjoint_step(f, lam, torch.empty_like(f))
    with pytest.raises(Pk.LbmError):
        h.step_record(torch.empty_like(f))


# ------------------------------------------------------------ cut-down jet
N, NZ, D, NSTEPS, NU, COFLOW = 32, 64, 4, 400, 2e-4, 0.002


def _jet_objective(storage, every=20, scale=4, model="fclb"):
    """The inlet-sensitivity jet (128 x 128 x 256, D = 16) with every length
    divided by scale (MRT-LES: Table 1 basis, C_S = 0.1)."""
    import paper_1206_0389_amd as Pk
    from paper_1206_0389_amd.adjoint import InletProbeObjective
    n, nz, d = 4 * N // scale, 4 * NZ // scale, 4 * D // scale
    c = synth.jet_adjoint_case(n, nz, d, u_jet=0.05, u_coflow=COFLOW, sigma=0.005, seed=389)
    face_u = [[0.0, 0.0, COFLOW] for _ in range(4)] + [[0.0, 0.0, 0.0]] * 2
    lat = Pk.Lattice(model=model, storage=storage, shape=(n, n, nz), nu=NU,
                     cs_smag=0.1 if model == "mrt" else 0.0)
    obj = InletProbeObjective(lat, [W, W, W, W, I, O], face_u, torch.from_numpy(c["base_u"]),
                              c["square"], c["probe_lo"], c["probe_hi"], NSTEPS, every=every)
    return obj, c


def _golden(model="fclb"):
    path = GOLDEN[model]
    if not os.path.exists(path):
        pytest.skip("stored oracle gradient not written")
    J, grad, fd = None, np.zeros((3, D, D)), np.zeros((D, D))
    for line in open(path):
        p = line.split()
        if not p or p[0].startswith("#"):
            continue
        if p[0] == "J":
            J = float(p[1])
        elif p[0] == "grad":
            grad[int(p[1]), int(p[2])] = [float(v) for v in p[3:]]
        elif p[0] == "fd":
            fd[int(p[2])] = [float(v) for v in p[3:]]
    return J, grad, fd


@pytest.mark.parametrize("model", ["fclb", "mrt"])
def test_cutdown_gradient_fp64_matches_oracle(model):
    """J and dJ/du_in (every component) of the 400-step cut-down jet against
    the oracle's stored FP64 adjoint (MRT-LES: Table 1 basis, C_S = 0.1)."""
    Jo, go, _ = _golden(model)
    obj, c = _jet_objective("f64", model=model)
    delta = torch.from_numpy(c["delta"]).cuda().requires_grad_(True)
    J = obj(delta)
    assert abs(float(J.detach()) - Jo) <= 1e-10 * abs(Jo)
    J.backward()
    g = delta.grad.cpu().numpy()
    assert np.linalg.norm(g - go[2]) <= 1e-10 * np.linalg.norm(go[2])
    full, _ = obj.backward()
    b0, b1, a0, a1 = c["square"]
    gf = full[:, b0:b1, a0:a1].cpu().numpy()
    assert np.abs(gf - go).max() <= 1e-10 * np.abs(go).max()


@pytest.mark.parametrize("model", ["fclb", "mrt"])
def test_cutdown_gradient_matches_finite_differences(model):
    """Central differences of J (GPU, FP64, h = 1e-6) for all 16 components
    (MRT-LES with the eddy viscosity on: the strain magnitude is zero where
    the flow has not arrived, where the adjoint takes derivative 0 and the
    differences see only second-order changes)."""
    obj, c = _jet_objective("f64", model=model)
    delta = torch.from_numpy(c["delta"]).cuda()
    obj.forward(delta)
    grad, _ = obj.backward()
    b0, b1, a0, a1 = c["square"]
    g = grad[2, b0:b1, a0:a1].cpu().numpy()
    h = 1e-6
    fd = np.zeros((D, D))
    for b in range(D):
        for a in range(D):
            dp, dm = delta.clone(), delta.clone()
            dp[b, a] += h
            dm[b, a] -= h
            fd[b, a] = (obj.value(dp) - obj.value(dm)) / (2 * h)
    rel = float(np.linalg.norm(g - fd) / np.linalg.norm(fd))
    print(model, "adjoint vs FD relative L2", rel, flush=True)
    assert rel <= 1e-4


def test_mrt_cutdown_gradient_fp32_close_to_fp64():
    """MRT-LES: FP32 storage and adjoint against the FP64 gradient (1e-4)."""
    out = {}
    for storage in ("f64", "f32"):
        obj, c = _jet_objective(storage, model="mrt")
        delta = torch.from_numpy(c["delta"]).cuda()
        J = obj.forward(delta)
        grad, _ = obj.backward()
        b0, b1, a0, a1 = c["square"]
        out[storage] = (J, grad[2, b0:b1, a0:a1].cpu().numpy())
    (J64, g64), (J32, g32) = out["f64"], out["f32"]
    rel = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    print("MRT FP32 vs FP64 gradient relative L2", rel, "J", J32, J64, flush=True)
    assert abs(J32 - J64) <= 1e-4 * abs(J64)
    assert rel <= 1e-4


def test_cutdown_gradient_fp32():
    """FP32 storage and FP32 adjoint against the oracle's FP64 gradient."""
    Jo, go, _ = _golden()
    obj, c = _jet_objective("f32")
    delta = torch.from_numpy(c["delta"]).cuda()
    J = obj.forward(delta)
    grad, _ = obj.backward()
    b0, b1, a0, a1 = c["square"]
    g = grad[2, b0:b1, a0:a1].cpu().numpy()
    rel = float(np.linalg.norm(g - go[2]) / np.linalg.norm(go[2]))
    print("FP32 gradient relative L2 vs FP64 oracle", rel, "J", J, Jo, flush=True)
    assert abs(J - Jo) <= 1e-4 * abs(Jo)
    assert rel <= 1e-4


def test_backward_after_value_and_second_forward():
    """A value() call between forward and backward (a finite-difference probe
    at another delta, which changes the lattice's inlet) leaves the gradient
    of the forward pass unchanged; a second forward through the autograd
    function before the first one's backward is refused."""
    obj, c = _jet_objective("f64")
    delta = torch.from_numpy(c["delta"]).cuda()
    obj.forward(delta)
    g1, l1 = obj.backward()
    obj.forward(delta)
    obj.value(delta + 1e-3)
    g2, l2 = obj.backward()
    assert torch.equal(g1, g2) and torch.equal(l1, l2)
    d1 = delta.clone().requires_grad_(True)
    J1 = obj(d1)
    J2 = obj(delta.clone().requires_grad_(True))
    with pytest.raises(RuntimeError):
        J1.backward()
    J2.backward()


def test_checkpoint_spacing_does_not_change_gradient():
    obj1, c = _jet_objective("f64", every=20)
    obj2, _ = _jet_objective("f64", every=7)
    delta = torch.from_numpy(c["delta"]).cuda()
    assert obj1.forward(delta) == obj2.forward(delta)
    g1, l1 = obj1.backward()
    g2, l2 = obj2.backward()
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


# ------------------------------------------------- full-size jet (128^2 x 256)
_FULL = {}


def _full_gradients(model="fclb"):
    """FP64 and FP32 adjoint gradients of the full-size jet, computed once
    per model (the FP64 objective kept for the difference quotients)."""
    if model not in _FULL:
        for other in list(_FULL):  # one model's checkpoints at a time
            del _FULL[other]
        torch.cuda.empty_cache()
        r = {}
        for storage in ("f64", "f32"):
            obj, c = _jet_objective(storage, scale=1, model=model)
            delta = torch.from_numpy(c["delta"]).cuda()
            J = obj.forward(delta)
            grad, _ = obj.backward()
            b0, b1, a0, a1 = c["square"]
            r[storage] = (J, grad[2, b0:b1, a0:a1].cpu().numpy())
            if storage == "f64":
                r["obj"], r["delta"] = obj, delta
            del obj
            torch.cuda.empty_cache()
        _FULL[model] = r
    return _FULL[model]


@pytest.mark.parametrize("model", ["fclb", "mrt"])
def test_full_jet_fp32_gradient_close_to_fp64(model):
    r = _full_gradients(model)
    (J64, g64), (J32, g32) = r["f64"], r["f32"]
    rel = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    print("full jet", model, ": J", J64, J32, "FP32 vs FP64 gradient relative L2", rel,
          flush=True)
    assert abs(J32 - J64) <= 1e-4 * abs(J64)
    assert rel <= 1e-4


@pytest.mark.parametrize("part", range(4))
@pytest.mark.parametrize("model", ["fclb", "mrt"])
def test_full_jet_gradient_matches_finite_differences(part, model):
    """Central differences of J (FP64, h = 1e-6) for all 256 components,
    a quarter per test (MRT-LES: Table 1 basis, C_S = 0.1)."""
    r = _full_gradients(model)
    obj, delta = r["obj"], r["delta"]
    g = r["f64"][1]
    h = 1e-6
    rows = range(4 * part, 4 * part + 4)
    fd = np.zeros((4, g.shape[1]))
    for k, b in enumerate(rows):
        for a in range(g.shape[1]):
            dp, dm = delta.clone(), delta.clone()
            dp[b, a] += h
            dm[b, a] -= h
            fd[k, a] = (obj.value(dp) - obj.value(dm)) / (2 * h)
    ga = g[4 * part:4 * part + 4]
    rel = float(np.linalg.norm(ga - fd) / np.linalg.norm(fd))
    print("full jet", model, "rows", list(rows), "adjoint vs FD relative L2", rel, flush=True)
    assert rel <= 1e-4


@pytest.mark.parametrize("model", ["fclb", "mrt_dhumieres"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("faces", ["jet", "periodic"])
def test_step_record_matches_get_populations(storage, faces, model):
    """lbm_step_record writes the state lbm_get_populations returns before the
    step (FP64: exactly; FP32: the bounce-back term is added in FP32) and
    advances the lattice exactly like lbm_step."""
    shape = (37, 9, 11)
    nx, ny, nz = shape
    g1, _, _ = _pair(FACE_SETS[faces], shape, storage=storage, model=model)
    g2, _, _ = _pair(FACE_SETS[faces], shape, storage=storage, model=model)
    f = synth.random_populations(g1.Q, (nz, ny, nx), 1e-2, seed=14)
    for g in (g1, g2):
        g.set_populations(torch.from_numpy(f))
    dt = g1.adjoint_dtype
    rec = torch.empty((g1.Q, nz, ny, nx), dtype=dt, device="cuda")
    for k in range(3):  # even and odd parities
        want = g1.populations(dt)
        g1.step_record(rec)
        g2.step(1)
        if storage == "f64":
            assert torch.equal(rec, want), k
        else:
            assert float((rec - want).abs().max()) <= 1e-7 * float(want.abs().max()), k
        assert torch.equal(g1.populations(), g2.populations()), k
    import paper_1206_0389_amd as Pk
    with pytest.raises(Pk.LbmError):
        g1.step_record(rec.to(torch.float32 if dt == torch.float64 else torch.float64))


@pytest.mark.parametrize("model", ["fclb", "mrt_dhumieres"])
def test_objective_with_zero_and_one_step(model):
    """nsteps = 0: J is the probe of the initial state and nothing depends on
    the inlet; nsteps = 1: J and dJ/du_in against the oracle's driver."""
    import paper_1206_0389_amd as Pk
    from paper_1206_0389_amd.adjoint import InletProbeObjective
    name, code, basis, cs = MODELS[model]
    n, nz, D = 12, 16, 4
    c = synth.jet_adjoint_case(n, nz, D, u_jet=0.05, u_coflow=COFLOW, sigma=0.005, seed=7)
    lo, hi = (3, 3, 2), (9, 9, 6)
    face_u = [[0.0, 0.0, COFLOW] for _ in range(4)] + [[0.0, 0.0, 0.0]] * 2
    q = 27 if code == oracle.FCLB27 else 19
    f0 = synth.random_populations(q, (nz, n, n), 1e-2, seed=4)
    o = oracle.Lattice(code, n, n, nz, nu=0.02, faces=[W, W, W, W, I, O], face_u=face_u,
                       inlet_u=c["inlet_u"], cs_smag=cs, basis=basis)
    for nsteps in (0, 1):
        lat = Pk.Lattice(model=name, storage="f64", shape=(n, n, nz), nu=0.02, cs_smag=cs,
                         mrt_basis=basis)
        obj = InletProbeObjective(lat, [W, W, W, W, I, O], face_u, torch.from_numpy(c["base_u"]),
                                  c["square"], lo, hi, nsteps, every=1, f0=torch.from_numpy(f0))
        J = obj.forward(torch.from_numpy(c["delta"]).cuda())
        grad, lam0 = obj.backward()
        Jo, go, lo0 = o.inlet_gradient(f0, 0, nsteps, lo, hi, every=1)
        assert abs(J - Jo) <= 1e-12 * abs(Jo)
        if nsteps == 0:
            assert float(grad.abs().max()) == 0.0
        else:
            assert float(np.abs(grad.cpu().numpy() - go).max()) <= 1e-12 * np.abs(go).max()
        assert float(np.abs(lam0.cpu().numpy() - lo0).max()) <= 1e-12 * np.abs(lo0).max()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("model", ["mrt_table1", "mrt_dhumieres"])
def test_mrt_objective_gradient_matches_oracle(model, storage):
    """J and dJ/du_in through 24 MRT-LES steps (C_S = 0.1) of a small jet
    from a random state, checkpoints every 5 steps: FP64 against the
    oracle's driver to 1e-10, FP32 storage and adjoint to 1e-4."""
    import paper_1206_0389_amd as Pk
    from paper_1206_0389_amd.adjoint import InletProbeObjective
    name, code, basis, cs = MODELS[model]
    n, nz, D, nsteps, nu = 12, 16, 4, 24, 0.01
    c = synth.jet_adjoint_case(n, nz, D, u_jet=0.05, u_coflow=COFLOW, sigma=0.005, seed=17)
    lo, hi = (3, 3, 6), (9, 9, 12)
    face_u = [[0.0, 0.0, COFLOW] for _ in range(4)] + [[0.0, 0.0, 0.0]] * 2
    f0 = synth.random_populations(19, (nz, n, n), 1e-3, seed=5)
    print("case mrt objective", model, storage, flush=True)
    lat = Pk.Lattice(model=name, storage=storage, shape=(n, n, nz), nu=nu, cs_smag=cs,
                     mrt_basis=basis)
    obj = InletProbeObjective(lat, [W, W, W, W, I, O], face_u, torch.from_numpy(c["base_u"]),
                              c["square"], lo, hi, nsteps, every=5,
                              f0=torch.from_numpy(f0.astype(np.float32 if storage == "f32"
                                                            else np.float64)))
    J = obj.forward(torch.from_numpy(c["delta"]).cuda())
    grad, lam0 = obj.backward()
    o = oracle.Lattice(code, n, n, nz, nu=nu, faces=[W, W, W, W, I, O], face_u=face_u,
                       inlet_u=c["inlet_u"], cs_smag=cs, basis=basis)
    f0o = f0.astype(np.float32).astype(np.float64) if storage == "f32" else f0
    Jo, go, lo0 = o.inlet_gradient(f0o, 0, nsteps, lo, hi, every=5)
    gerr = float(np.linalg.norm(grad.cpu().numpy() - go) / np.linalg.norm(go))
    lerr = float(np.abs(lam0.double().cpu().numpy() - lo0).max() / np.abs(lo0).max())
    print("J", J, Jo, "gradient", gerr, "lambda_0", lerr, flush=True)
    tol = 1e-10 if storage == "f64" else 1e-4
    assert abs(J - Jo) <= tol * abs(Jo)
    assert gerr <= tol and lerr <= tol
