"""The health check inside lbm_step (lbm_set_check), through the C ABI.

A NaN written into one population of one node on the host stops the steps
at the first check with LBM_ENONFINITE (the steps before it stand); a
periodic lattice conserves mass, so a tight mass bound passes there, while
an inflow/outflow jet changes its mass and trips the same bound with
LBM_EMASS. Checked steps leave the state exactly as unchecked steps do.
"""
import numpy as np
import pytest

import synth
from lbm_cases import JET_FACES, face_velocities, gpu_lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("name,storage", [("fclb", "f32"), ("mrt_table1", "f64"),
                                          ("fclb", "f16")])
def test_nan_injected_on_the_host_stops_at_the_first_check(name, storage):
    import paper_1206_0389_amd as Pk
    _say("case check nan", name, storage)
    g = gpu_lattice(name, storage, (20, 12, 16), 0.02, cs=0.1)
    f = synth.random_populations(g.Q, (16, 12, 20), 1e-3, seed=4)
    g.set_populations(torch.from_numpy(f))
    g.set_check(3)  # checks the clean state at once
    f[5, 7, 3, 11] = np.nan
    g.set_populations(torch.from_numpy(f))
    with pytest.raises(Pk.LbmError) as e:
        g.step(10)
    assert e.value.status == Pk.ENONFINITE
    assert g.time == 3
    # a state that already holds the NaN is refused when the check is set
    with pytest.raises(Pk.LbmError) as e:
        g.set_check(1)
    assert e.value.status == Pk.ENONFINITE


def test_mass_check_passes_on_a_periodic_lattice_and_changes_nothing():
    _say("case check periodic mass")
    f = synth.random_populations(27, (16, 12, 20), 1e-3, seed=8)
    a = gpu_lattice("fclb", "f64", (20, 12, 16), 0.02)
    b = gpu_lattice("fclb", "f64", (20, 12, 16), 0.02)
    a.set_populations(torch.from_numpy(f))
    b.set_populations(torch.from_numpy(f))
    m0 = a.reduce()[0]
    # FP64 rounding of the mass over 3840 nodes: far below 1e-10
    a.set_check(2, mass_tol=1e-10)
    a.step(9)
    b.step(9)
    assert a.time == 9
    assert torch.equal(a.populations(), b.populations())
    assert abs(a.reduce()[0] - m0) <= 1e-10


def test_mass_check_trips_on_an_open_jet():
    import paper_1206_0389_amd as Pk
    _say("case check open jet mass")
    nx, ny, nz = 16, 16, 24
    g = gpu_lattice("fclb", "f32", (nx, ny, nz), 0.02, faces=JET_FACES,
                    face_u=face_velocities(), inlet=synth.jet_inlet(nx, ny, 4.0, 0.05, 0.002))
    d, u = synth.uniform_fields(nx, ny, nz)
    g.init_equilibrium(torch.from_numpy(d), torch.from_numpy(u))
    g.set_check(4, mass_tol=1e-9)
    with pytest.raises(Pk.LbmError) as e:
        g.step(40)
    assert e.value.status == Pk.EMASS
    assert g.time % 4 == 0 and 0 < g.time <= 40
    # finiteness only: the open jet steps on
    g.set_check(4)
    g.step(8)
