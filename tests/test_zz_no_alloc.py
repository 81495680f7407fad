"""lbm_reduce_static (static partial-sum buffer, device output, nothing
allocated) against lbm_reduce on the same lattice, through the C ABI.

The two differ only in summation order (the static variant folds z planes
into the blocks of one x-y plane once a lattice has more blocks than the
buffer's 16384 rows), so each sum agrees to 1e-13 of the sum of the
magnitudes of its terms (the FP64 error bound of either order is below
1e-14 of it at these sizes). Two calls in a row, the second on a smaller
lattice, check that nothing of the first call's partial sums leaks into the
second.
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


def _lattice(name, storage, shape, seed, faces=None):
    nx, ny, nz = shape
    g = gpu_lattice(name, storage, shape, 0.02, cs=0.1, faces=faces,
                    face_u=None if faces is None else face_velocities(),
                    inlet=None if faces is None else synth.jet_inlet(nx, ny, 4.0, 0.05, 0.002),
                    amp=5e-4, seed=seed)
    Q = g.Q
    f = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=seed)
    g.set_populations(torch.from_numpy(f).to(torch.float32 if storage == "f32" else
                                             torch.float64))
    g.step(3)
    return g


def _magnitudes(g):
    """Sum over nodes of |rho - 1|, |j_a| and the kinetic energy term."""
    rho, u = g.macroscopic()
    r = 1.0 + rho if g.Q == 27 else torch.ones_like(rho)
    j = u * r
    ke = 0.5 * (j * j).sum(0) / r
    return np.array([rho.abs().sum().item()] + [j[a].abs().sum().item() for a in range(3)] +
                    [ke.abs().sum().item()])


def _compare(g, out):
    want = np.array(g.reduce())
    g.reduce_static(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    tol = 1e-13 * _magnitudes(g) + 1e-300
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - want) <= tol), (got, want, tol)
    return got


def test_static_reduce_matches_reduce_on_two_calls():
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    # 128 x 128 x 320: 64 blocks a plane, 320 planes -> 256 rows fold z
    _say("case reduce_static fclb f32 (128, 128, 320) jet faces")
    big = _lattice("fclb", "f32", (128, 128, 320), 3, faces=JET_FACES)
    first = _compare(big, out)
    del big
    _say("case reduce_static mrt_table1 f64 (40, 24, 16) periodic")
    small = _lattice("mrt_table1", "f64", (40, 24, 16), 5)
    second = _compare(small, out)
    assert not np.array_equal(first, second)


def test_static_reduce_without_folding_is_reduce_exactly():
    """Lattices whose blocks all fit take lbm_reduce's order: equal sums."""
    out = torch.empty((5,), dtype=torch.float64, device="cuda")
    _say("case reduce_static fclb f64 (48, 32, 24) exact")
    g = _lattice("fclb", "f64", (48, 32, 24), 9)
    g.reduce_static(out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.array(g.reduce()))


def test_static_reduce_rejects_planes_beyond_the_buffer():
    import paper_1206_0389_amd as Pk
    out = torch.empty((5,), dtype=torch.float64, device="cuda")
    # 4096 x 1040: 16 x 1040 = 16640 blocks of 256 nodes in one plane
    _say("case reduce_static refusal (4096, 1040, 2)")
    g = gpu_lattice("fclb", "f32", (4096, 1040, 2), 0.02)
    with pytest.raises(Pk.LbmError):
        g.reduce_static(out)
    with pytest.raises(ValueError):
        g.reduce_static(torch.empty((5,), dtype=torch.float32, device="cuda"))
