"""Host-side checks of the C ABI (no GPU needed: nothing here launches).

The library must load and export every function declared in include/lbm.h;
argument validation happens on the host before any launch.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:int|const char\*)\s+(lbm_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def P():
    import paper_1206_0389_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("liblbm.so not built")
    return P


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["lbm_create_lattice", "lbm_set_boundaries", "lbm_step", "lbm_get_macroscopic"]:
        assert n in names


def test_library_exports_every_declared_symbol(P):
    lib = P.lib()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) <= set(P.exported_symbols()) | {"lbm_strerror"}


def _cfg(P, **kw):
    c = P.Config()
    c.model = {"fclb": P.D3Q27_FCLB, "mrt": P.D3Q19_MRT_LES}[kw.get("model", "fclb")]
    c.storage = kw.get("storage", P.F32)
    c.nx, c.ny, c.nz = kw.get("shape", (16, 8, 4))
    c.nu = kw.get("nu", 0.01)
    c.cs_smag = kw.get("cs", 0.0)
    c.mrt_basis = kw.get("basis", 0)
    c.use_default_rates = 1
    return c


def _create(P, c):
    h = ctypes.c_void_p()
    rc = P.lib().lbm_create_lattice(ctypes.byref(c), ctypes.byref(h))
    return rc, h


def test_create_validates_configuration(P):
    ok, h = _create(P, _cfg(P))
    assert ok == P.OK
    P.lib().lbm_destroy(h)
    bad = [dict(nu=0.0), dict(nu=-1.0), dict(cs=-0.1), dict(shape=(0, 4, 4)),
           dict(shape=(2048, 2048, 1024)), dict(storage=7)]
    for kw in bad:
        rc, _ = _create(P, _cfg(P, **kw))
        assert rc == P.EINVAL, kw
    c = _cfg(P, model="mrt")
    c.mrt_basis = 5
    assert _create(P, c)[0] == P.EINVAL
    c = _cfg(P, model="mrt")
    c.use_default_rates = 0
    c.rates[0] = 2.5
    assert _create(P, c)[0] == P.EINVAL
    assert P.lib().lbm_create_lattice(None, None) == P.EINVAL


def test_create_enforces_the_population_slab_limit(P):
    """One population (nodes x element size) must stay below 4 GiB: the
    kernels address it with 32-bit byte offsets."""
    # 1024 x 1024 x 512 nodes: 4 GiB per population in FP64, 2 GiB in FP32
    big = (1024, 1024, 512)
    assert _create(P, _cfg(P, shape=big, storage=P.F64))[0] == P.EINVAL
    rc, h = _create(P, _cfg(P, shape=big, storage=P.F32))
    assert rc == P.OK
    P.lib().lbm_destroy(h)
    rc, h = _create(P, _cfg(P, shape=(1024, 1024, 511), storage=P.F64))
    assert rc == P.OK
    P.lib().lbm_destroy(h)


def test_required_bytes_and_binding_checks(P):
    _, h = _create(P, _cfg(P, shape=(16, 8, 4), storage=P.F32))
    n = ctypes.c_size_t()
    assert P.lib().lbm_required_bytes(h, ctypes.byref(n)) == P.OK
    assert n.value >= 16 * 8 * 4 * 27 * 4
    # unbound: every data call refuses before launching
    assert P.lib().lbm_step(h, 1) == P.EUNBOUND
    out = (ctypes.c_double * 5)()
    assert P.lib().lbm_reduce(h, out) == P.EUNBOUND
    # misaligned or short blocks are refused without touching them
    assert P.lib().lbm_bind_memory(h, ctypes.c_void_p(0x1001), n.value) == P.EINVAL
    assert P.lib().lbm_bind_memory(h, ctypes.c_void_p(0x100000), n.value - 1) == P.ENOMEM
    assert P.lib().lbm_step(h, -1) == P.EINVAL
    # statistics: refused before any launch
    fake = ctypes.c_void_p(0x100000)
    assert P.lib().lbm_stats_accumulate(h, fake) == P.EUNBOUND
    assert P.lib().lbm_stats_accumulate(h, None) == P.EINVAL
    fin = P.lib().lbm_stats_finalize
    assert fin(h, fake, 0, fake, fake, None, P.DTYPE_F64, 2, 0, 0) == P.EINVAL  # count < 1
    assert fin(h, fake, 1, fake, fake, None, P.DTYPE_F64, 3, 0, 0) == P.EINVAL  # axis
    assert fin(h, fake, 1, None, fake, None, P.DTYPE_F64, 2, 0, 0) == P.EINVAL  # no mean
    assert fin(h, fake, 1, fake, fake, fake, P.DTYPE_F64, 2, 16, 0) == P.EINVAL  # x0 >= nx
    assert fin(h, fake, 1, fake, fake, fake, P.DTYPE_F64, 0, 0, 4) == P.EINVAL  # z0 >= nz
    assert fin(h, fake, 1, fake, fake, fake, 7, 2, 0, 0) == P.EINVAL  # dtype
    # curved-wall links: refused before any launch
    assert P.lib().lbm_set_links(h, fake, fake, 4) == P.EUNBOUND
    assert P.lib().lbm_set_links(h, fake, fake, -1) == P.EINVAL
    assert P.lib().lbm_set_links(h, fake, fake, 1 << 31) == P.EINVAL
    assert P.lib().lbm_set_links(None, None, None, 0) == P.EINVAL
    # jet profile and fits: argument checks before any launch
    jp = P.lib().lbm_jet_profile
    assert jp(h, fake, P.DTYPE_F64, 2, 7.5, 3.5, 8, 0.5, 1, fake, fake, None) == P.EINVAL  # nr
    assert jp(h, fake, P.DTYPE_F64, 2, 16.0, 3.5, 8, 0.5, 8, fake, fake, None) == P.EINVAL  # c0
    assert jp(h, fake, P.DTYPE_F64, 3, 7.5, 3.5, 8, 0.5, 8, fake, fake, None) == P.EINVAL  # axis
    assert jp(h, fake, P.DTYPE_F64, 2, 7.5, 3.5, 8, 0.0, 8, fake, fake, None) == P.EINVAL  # dr
    jf = P.lib().lbm_jet_fit
    assert jf(h, fake, fake, fake, 10, 8, 0.5, 0.0, 0.05, 8.0, 4, 4, fake) == P.EINVAL  # empty
    assert jf(h, fake, fake, fake, 10, 8, 0.5, 0.0, 0.0, 8.0, 0, 10, fake) == P.EINVAL  # u0
    assert jf(h, fake, fake, fake, 10, 8, 0.5, 0.0, 0.05, 8.0, 0, 11, fake) == P.EINVAL  # p1
    P.lib().lbm_destroy(h)


def test_boundary_validation(P):
    _, h = _create(P, _cfg(P))
    bc = P.Boundaries()
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.OK  # all periodic
    bc.face_type[0] = P.WALL  # x- wall with a periodic x+ is inconsistent
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.face_type[1] = P.WALL
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.OK
    bc.face_type[4], bc.face_type[5] = P.INLET, P.OUTFLOW  # inlet without data
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.inlet_u = 0x1000
    bc.inlet_dtype = 9
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.inlet_dtype = P.DTYPE_F64
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.OK
    bc.face_type[2], bc.face_type[3] = P.FREESLIP, P.WALL  # free-slip top, wall bottom
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.OK
    bc.face_type[3] = P.PRESSURE  # fixed-pressure face at density deviation 0.01
    bc.face_drho[3] = 0.01
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.OK
    bc.face_drho[3] = -1.0  # non-positive density
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.face_drho[3] = float("nan")
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.face_drho[3] = 0.0
    bc.face_type[3] = 6  # no such face type
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.face_type[2] = bc.face_type[3] = P.WALL
    bc.face_type[4], bc.face_type[5] = P.WALL, P.WALL
    bc.face_type[0], bc.face_type[1] = P.INLET, P.OUTFLOW  # outflow only on z faces
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.face_type[0], bc.face_type[1] = P.WALL, P.WALL
    bc.face_type[4], bc.face_type[5] = P.OUTFLOW, P.OUTFLOW  # two outflow faces
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    bc.face_type[2] = bc.face_type[3] = 11
    assert P.lib().lbm_set_boundaries(h, ctypes.byref(bc)) == P.EINVAL
    P.lib().lbm_destroy(h)


def test_strerror(P):
    assert "invalid" in P.strerror(P.EINVAL)
    assert P.strerror(P.ENONFINITE)
    assert P.strerror(12345) == "unknown status"


def test_product_never_imports_the_oracle():
    """The library's Python side holds no path to the oracle (test
    infrastructure): no import of it anywhere in the package."""
    pkg = os.path.join(ROOT, "paper_1206_0389_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), fn
                assert "lbm_oracle" not in txt, fn


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library every call raises: there is no fallback."""
    import paper_1206_0389_amd as P
    monkeypatch.setattr(P, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "liblbm.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(RuntimeError):
        P.lib()


def test_binding_mirrors_every_declared_entry_point():
    import paper_1206_0389_amd as P
    missing = [n for n in _declared() if n not in P._SIGS]
    assert not missing, missing


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU: --gpus N with N > 1 exits non-zero with a
    message, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=root)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)
