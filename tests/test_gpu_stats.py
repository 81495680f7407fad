"""Time averages on the GPU (lbm_stats_accumulate, lbm_stats_finalize)
against the oracle's statistics of its own states (the jet statistics of
Section 3: mean velocity, rms fluctuation, turbulent intensity Eq. (25)).

Both sides start from the same seeded far-from-equilibrium state of a small
jet and average the velocity after each of K steps. The GPU keeps FP64
running sums and forms var = <u^2> - <u>^2; the oracle averages its states
in two passes. Bounds, derived from the per-step state error e (FP64 1e-12,
FP32 4e-6 relative, test_gpu_parity.py) accumulated over K steps:
  mean:  |d mean| <= K e max|u|
  var:   |d var|  <= 4 K e max<u^2>   (2 u du, plus the one-pass rounding,
                                       a few K 1e-16 <u^2>)
  ti:    relative K e / (var / max<u^2>) on nodes whose variance is at least
         1e-3 max<u^2> (the bound of d var over 2 var, doubled).
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import JET_FACES, MODELS, face_velocities, gpu_lattice, oracle_lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

ERR = {"f64": 1e-12, "f32": 4e-6}
ROUND = {"f64": np.float64, "f32": np.float32}


def _compare(mean, rms, ti, ref, K, storage):
    m_o, r_o, t_o = ref
    e = ERR[storage]
    u2max = float((m_o ** 2 + r_o ** 2).max())
    umax = float(np.abs(m_o).max())
    dm = float(np.abs(mean - m_o).max())
    dv = float(np.abs(rms ** 2 - r_o ** 2).max())
    assert dm <= K * e * umax, (dm, K * e * umax)
    assert dv <= 4 * K * e * u2max, (dv, 4 * K * e * u2max)
    mask = r_o[2] ** 2 >= 1e-3 * u2max
    assert mask.sum() > 0
    rel = float((np.abs(ti - t_o) / np.abs(t_o))[mask].max())
    assert rel <= 2 * K * e / 1e-3, rel
    return dm / umax, dv / u2max, rel


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_jet_statistics_against_oracle(name, storage):
    shape, K, t0 = (16, 12, 10), 8, 4
    nx, ny, nz = shape
    Q = 19 if MODELS[name][0] == oracle.MRT19 else 27
    print("case statistics", name, storage, shape, "K", K, flush=True)
    inlet = synth.jet_inlet(nx, ny, 6.0, 0.05, 0.002)
    kw = dict(faces=JET_FACES, face_u=face_velocities(0.002), inlet=inlet, amp=5e-4, seed=7)
    f0 = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=21)
    f0 = f0.astype(ROUND[storage]).astype(np.float64)
    g = gpu_lattice(name, storage, shape, 0.02, cs=0.1, **kw)
    g.set_populations(torch.from_numpy(f0), t0)
    sums = g.stats_buffer()
    for _ in range(K):
        g.step(1)
        g.stats_accumulate(sums)
    point = (nx // 2, ny // 2)
    mean, rms, ti = (t.cpu().numpy() for t in g.stats_finalize(sums, K, axis=2, point=point))
    o = oracle_lattice(name, shape, 0.02, cs=0.1, **kw)
    f, us = f0.copy(), []
    for k in range(K):
        f = o.run(f, t0 + k, 1)
        us.append(o.macroscopic(f)[1])
    ref = oracle.velocity_statistics(us, axis=2, point=point)
    print(name, storage, "mean, var, ti errors", _compare(mean, rms, ti, ref, K, storage),
          flush=True)


def test_statistics_axis_choice_and_errors():
    """Streamwise axis x on a periodic lattice: ti is the x rms over the mean
    x velocity at the axis point of each x cross-section; invalid calls raise
    before any launch."""
    import paper_1206_0389_amd as P
    shape, K = (12, 10, 8), 5
    nx, ny, nz = shape
    print("case statistics axis x", shape, flush=True)
    g = gpu_lattice("fclb", "f64", shape, 0.02)
    f0 = synth.random_populations(27, (nz, ny, nx), amp=1e-2, seed=5)
    f0[1] += 0.01  # mean flow along +x
    g.set_populations(torch.from_numpy(f0), 0)
    sums = g.stats_buffer()
    for _ in range(K):
        g.step(1)
        g.stats_accumulate(sums)
    point = (3, 6)  # (y, z) of the jet axis
    mean, rms, ti = g.stats_finalize(sums, K, axis=0, point=point)
    want = rms[0] / mean[0][point[1], point[0], :].reshape(1, 1, nx)
    assert float((ti - want).abs().max()) <= 1e-15 * float(want.abs().max())
    mean2, rms2, ti2 = g.stats_finalize(sums, K, dtype=torch.float32)
    assert ti2 is None and mean2.dtype == torch.float32
    assert float((mean2.double() - mean).abs().max()) <= 1e-7 * float(mean.abs().max())
    with pytest.raises(P.LbmError):
        g.stats_finalize(sums, 0)
    with pytest.raises(P.LbmError):
        g.stats_finalize(sums, K, axis=0, point=(ny, 0))
    with pytest.raises(ValueError):
        g.stats_accumulate(sums[:3])
