"""The jet spreading profile on the GPU (lbm_jet_profile: the width of
Eq. (23) and the profile of Eq. (24)) against the oracle.

Seeded synthetic mean fields shaped like a spreading jet (a Gaussian whose
width grows along the axis, with seeded random perturbations) along each of
the three axes, read as FP64 and FP32 (the oracle reads the same FP32
values): u_m, the three radii and the profile agree to 1e-12 (the ray sums
differ only in order); sections where no ray reaches the radius give NaN on
both sides. End to end: the mean of lbm_stats_finalize on a small jet.
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import gpu_lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _jet_mean(shape, axis, seed):
    nx, ny, nz = shape
    n3 = (nx, ny, nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = [(n - 1) / 2.0 + 0.3 for n in n3]
    crd = (x, y, z)
    other = [d for d in range(3) if d != axis]
    b = 3.0 + 0.15 * crd[axis]
    r2 = sum(((crd[d] - c[d]) / b) ** 2 for d in other)
    noise = synth.gaussian_field((nz, ny, nx), 1.5, seed)
    mean = np.zeros((3, nz, ny, nx))
    mean[axis] = 0.05 * np.exp(-r2) * (1.0 + 0.05 * noise)
    for d in other:
        mean[d] = 0.002 * synth.gaussian_field((nz, ny, nx), 2.0, seed + 1 + d)
    return mean, (c[other[0]], c[other[1]])


def _cmp(got, ref, tol):
    got, ref = np.asarray(got), np.asarray(ref)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    err = np.abs(got[ok] - ref[ok]).max() / max(np.abs(ref[ok]).max(), 1e-300)
    assert err <= tol, err


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_jet_profile_against_oracle(axis, dtype):
    shape = (20, 18, 24) if axis == 2 else (24, 20, 18) if axis == 0 else (20, 24, 18)
    print("case jet_profile axis", axis, dtype, shape, flush=True)
    mean, center = _jet_mean(shape, axis, 41 + axis)
    if dtype == "f32":
        mean = mean.astype(np.float32).astype(np.float64)
    g = gpu_lattice("fclb", "f32", shape, 0.01)
    tmean = torch.from_numpy(mean.astype(np.float32 if dtype == "f32" else np.float64)).cuda()
    um, re, prof = g.jet_profile(tmean, axis=axis, center=center, ndir=24, dr=0.35, nr=40)
    rum, rre, rprof = oracle.jet_profile(mean, axis, center, 24, 0.35, 40)
    _cmp(um.cpu().numpy(), rum, 1e-14)
    _cmp(re.cpu().numpy(), rre, 1e-12)
    _cmp(prof.cpu().numpy(), rprof, 1e-12)
    print("radii", np.nanmin(rre), np.nanmax(rre), flush=True)


def test_jet_profile_of_time_averages():
    import paper_1206_0389_amd as Pk
    from lbm_cases import JET_FACES, face_velocities
    shape = (24, 24, 20)
    nx, ny, nz = shape
    g = gpu_lattice("fclb", "f64", shape, 0.002, faces=JET_FACES, face_u=face_velocities(0.002),
                    inlet=synth.jet_inlet(nx, ny, 8.0, 0.05, 0.002), amp=5e-3, seed=5)
    d, u = synth.uniform_fields(nx, ny, nz, u=(0.0, 0.0, 0.002))
    g.init_equilibrium(torch.from_numpy(d), torch.from_numpy(u))
    g.step(40)
    sums = g.stats_buffer()
    for _ in range(10):
        g.step(2)
        g.stats_accumulate(sums)
    mean, rms, _ = g.stats_finalize(sums, 10)
    um, re, prof = g.jet_profile(mean, axis=2, ndir=16, dr=0.5, nr=24)
    m = mean.cpu().numpy()
    c = ((nx - 1) / 2.0, (ny - 1) / 2.0)
    rum, rre, rprof = oracle.jet_profile(m, 2, c, 16, 0.5, 24)
    _cmp(um.cpu().numpy(), rum, 1e-14)
    _cmp(re.cpu().numpy(), rre, 1e-12)
    _cmp(prof.cpu().numpy(), rprof, 1e-12)
    # the jet leaves the inlet disk: near it the radius is about the disk's
    assert 2.0 < np.nanmean(rre[2, 1:6]) < 6.0
    with pytest.raises(Pk.LbmError):  # centre outside the section
        g.jet_profile(mean, axis=2, center=(nx, 0.0))
    with pytest.raises(Pk.LbmError):
        g.jet_profile(mean, axis=2, nr=1)


@pytest.mark.parametrize("axis", [2, 0])
def test_jet_fit_against_oracle(axis):
    """The jet-law fits (lbm_jet_fit, Eqs. (22)-(24)) of each side's own
    spreading profile of the same synthetic jet, and of seeded arrays that
    follow the laws exactly."""
    shape = (20, 18, 24) if axis == 2 else (24, 20, 18)
    print("case jet_fit axis", axis, flush=True)
    mean, center = _jet_mean(shape, axis, 51 + axis)
    g = gpu_lattice("fclb", "f32", shape, 0.01)
    um, re, prof = g.jet_profile(torch.from_numpy(mean).cuda(), axis=axis, center=center,
                                 ndir=24, dr=0.35, nr=40)
    got = g.jet_fit(um, re, prof, 0.35, -2.5, 0.05, 6.0, 1, um.numel() - 1).cpu().numpy()
    rum, rre, rprof = oracle.jet_profile(mean, axis, center, 24, 0.35, 40)
    ref = np.array(oracle.jet_fit(rum, rre, rprof, 0.35, -2.5, 0.05, 6.0, 1, rum.size - 1))
    assert got[3] == ref[3]
    np.testing.assert_allclose(got[:3], ref[:3], rtol=1e-11)
    # arrays that follow the laws exactly
    npl, nr, dr = 40, 30, 0.5
    x = np.arange(npl) - 3.0
    um2 = np.where(x > 0, 0.05 * 6.104 * 8.0 / np.where(x > 0, x, 1.0), 0.3)
    re2 = np.full((3, npl), np.nan)
    re2[2] = np.where(x > 0, 0.109 * np.maximum(x, 1.0), np.nan)
    r = dr * np.arange(nr)
    prof2 = 0.938 * np.exp(-0.944 * (r[None, :] / np.where(x > 0, re2[2], 1.0)[:, None]) ** 2)
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (um2, re2, prof2)]
    got2 = g.jet_fit(*t, dr, 3.0, 0.05, 8.0).cpu().numpy()
    ref2 = np.array(oracle.jet_fit(um2, re2, prof2, dr, 3.0, 0.05, 8.0, 0, npl))
    np.testing.assert_allclose(got2[:2], [6.104, 0.109], rtol=1e-12)
    assert got2[2] <= 1e-15 and got2[3] == ref2[3]
    import paper_1206_0389_amd as Pk
    with pytest.raises(Pk.LbmError):
        g.jet_fit(*t, dr, 3.0, 0.05, 8.0, p0=5, p1=5)
