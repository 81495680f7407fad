"""Host logic of the refined lattice, on the CPU: the library's level boxes
and node types (built on the host at create / set_boundaries / set_solids,
no device call) against the oracle's geometry, written separately from the
same definitions; invalid nestings and interface solids are refused."""
import ctypes
import types

import numpy as np
import pytest

import oracle
import synth
from lbm_cases import (REFINED_CASES as CASES, REFINED_FACE_U as FACE_U, jet_map,
                       refined_jet_geometry, slab_map)

P_ = pytest.importorskip("paper_1206_0389_amd")

W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC


def _lib():
    try:
        return P_.lib()
    except RuntimeError:  # pragma: no cover
        pytest.skip("liblbm.so not built")


def _library_levels(model, basis, shape, B, m, L, faces, drho=None, solids=None):
    lib = _lib()
    cfg = P_.make_config({oracle.FCLB27: "fclb", oracle.MRT19: "mrt", oracle.CLB27: "clb"}[model],
                         "f64", shape, 0.02, 0.1, basis, None,
                         types.SimpleNamespace(cuda_stream=0))  # no stream is used here
    h = ctypes.c_void_p()
    rc = lib.lbm_refined_create(ctypes.byref(cfg), B, L,
                                m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(h))
    if rc:
        return rc, None
    try:
        bc = P_.Boundaries()
        for k in range(6):
            bc.face_type[k] = int(faces[k])
            for c in range(3):
                bc.face_u[k][c] = FACE_U[k][c]
            if drho is not None:
                bc.face_drho[k] = drho[k]
        fake = (ctypes.c_void_p * L)(*([0] + [0x1000] * (L - 1)))  # stored, never read here
        nulls = (ctypes.c_void_p * L)()
        if I in faces:
            bc.inlet_u = 0x1000
            bc.inlet_dtype = 1
        rc = lib.lbm_refined_set_boundaries(h, ctypes.byref(bc), fake, nulls)
        if rc:
            return rc, None
        out = []
        for l in range(L):
            lo = (ctypes.c_int32 * 3)()
            dims = (ctypes.c_int32 * 3)()
            cnt = (ctypes.c_int64 * 5)()
            assert lib.lbm_refined_geometry(h, l, lo, dims, cnt) == 0
            if solids is not None and solids[l] is not None:
                box = _box(tuple(lo), tuple(dims), solids[l], (shape[0] << l))
                rc = lib.lbm_refined_set_solids(h, l, box.ctypes.data_as(
                    ctypes.POINTER(ctypes.c_uint8)))
                if rc:
                    return rc, None
            t = np.zeros((dims[2], dims[1], dims[0]), dtype=np.uint8)
            assert lib.lbm_refined_types(h, l, t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))) == 0
            out.append((tuple(lo), tuple(dims), t))
        return 0, out
    finally:
        lib.lbm_refined_destroy(h)


def _box(lo, dims, full, nx):
    (ox, oy, oz), (mx, my, mz) = lo, dims
    wx = min(mx, nx - ox)
    out = np.zeros((mz, my, mx), dtype=full.dtype)
    out[..., :wx] = full[oz:oz + mz, oy:oy + my, ox:ox + wx]
    return out


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("model", [oracle.FCLB27, oracle.MRT19])
def test_library_geometry_matches_oracle(case, model):
    levels, jet, faces, drho = CASES[case]
    if jet:
        n, nz, B, m = refined_jet_geometry(case)
        shape = (n, n, nz)
    else:
        shape, B = (4, 4, 64), 4
        m = slab_map(levels)
    rc, lv = _library_levels(model, oracle.BASIS_TABLE1, shape, B, m, levels, faces, drho)
    assert rc == 0
    iu = [None] + [np.zeros((3, shape[1] << l, shape[0] << l)) for l in range(1, levels)]
    c = oracle.Lattice(model, *shape, nu=0.02, faces=faces, face_u=FACE_U, face_drho=drho,
                       inlet_u=np.zeros((3, shape[1], shape[0])) if I in faces else None)
    R = oracle.Refined(c, B, m, levels, inlet_u=iu if I in faces else None)
    for l, (lo, dims, t) in enumerate(lv):
        assert dims[0] % 64 == 0 and lo[0] % 64 == 0
        want = _box(lo, dims, R.types(l), shape[0] << l)
        assert np.array_equal(t, want), l
        # every used node of the oracle lies in the library's box
        assert int((R.types(l) > 0).sum()) == int((want > 0).sum())


def test_library_refuses_what_the_oracle_refuses():
    shape, B = (16, 16, 32), 4
    m = np.zeros((8, 4, 4), dtype=np.uint8)
    m[3, 1, 1] = 2  # a level-2 block next to level-0 blocks
    assert _library_levels(oracle.FCLB27, 0, shape, B, m, 3, [W] * 6)[0] != 0
    with pytest.raises(ValueError):
        oracle.Refined(oracle.Lattice(oracle.FCLB27, *shape, nu=0.02, faces=[W] * 6), B, m, 3)
    # a solid bar through the level-1 ghost layer of the two-level jet
    m2 = jet_map(16, 32, 4, 2)
    sm = np.zeros((64, 32, 32), dtype=np.uint8)
    sm[4:6, 6:8, :] = 1
    rc, _ = _library_levels(oracle.FCLB27, 0, shape, B, m2, 2, [W, W, W, W, I, O],
                            solids=[None, sm])
    assert rc != 0
    iu = [None, np.zeros((3, 32, 32))]
    with pytest.raises(ValueError):
        oracle.Refined(oracle.Lattice(oracle.FCLB27, *shape, nu=0.02, faces=[W, W, W, W, I, O],
                                      inlet_u=np.zeros((3, 16, 16))), B, m2, 2, inlet_u=iu,
                       solid=[None, sm])
