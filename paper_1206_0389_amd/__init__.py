"""Python binding of the MI355X lattice Boltzmann library (``liblbm.so``).

Argument marshalling only: every step of the lattice update runs in the HIP
kernels of ``csrc/``. PyTorch supplies device memory and the HIP stream.
The module-level functions carry the C ABI names of ``include/lbm.h``
(without the ``lbm_`` prefix); :class:`Lattice` bundles them with the
torch-owned device block.

The library must be built (``python -m paper_1206_0389_amd.build``); there
is no CPU fallback and importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

OK, EINVAL, ENOMEM, EUNBOUND, EHIP, ENONFINITE, ESTATE, EMASS = 0, -1, -2, -3, -4, -5, -6, -7
D3Q19_MRT_LES, D3Q27_FCLB, D3Q27_CLB = 1, 2, 3
F64, F32, F16 = 1, 2, 3
DTYPE_F64, DTYPE_F32 = 1, 2
BASIS_TABLE1, BASIS_DHUMIERES = 0, 1
PERIODIC, WALL, INLET, OUTFLOW, FREESLIP, PRESSURE = 0, 1, 2, 3, 4, 5

# The ABI's velocity order (the tables of Section 2; D3Q19 is the first 19),
# e.g. for the direction index of the wall distances given to set_links.
VELOCITIES = ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
              (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1), (1, 1, 1), (-1, 1, 1),
              (1, -1, 1), (1, 1, -1), (-1, -1, 1), (-1, 1, -1), (1, -1, -1), (-1, -1, -1))
RHO_FULL, RHO_DEVIATION = 0, 1

STORAGE = {"f64": F64, "f32": F32, "f16": F16}
MODEL = {"mrt": D3Q19_MRT_LES, "fclb": D3Q27_FCLB, "clb": D3Q27_CLB}


class LbmError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, strerror(status), status))


class Config(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("mrt_basis", ctypes.c_int32),
        ("nu", ctypes.c_double), ("cs_smag", ctypes.c_double),
        ("rates", ctypes.c_double * 8),
        ("use_default_rates", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class Boundaries(ctypes.Structure):
    _fields_ = [
        ("face_type", ctypes.c_int32 * 6),
        ("face_u", (ctypes.c_double * 3) * 6),
        ("inlet_u", ctypes.c_void_p),
        ("inlet_dtype", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("inlet_mask", ctypes.c_void_p),
        ("inlet_amp", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("face_drho", ctypes.c_double * 6),
    ]


_lib = None
_SIGS = {
    "lbm_create_lattice": [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)],
    "lbm_required_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lbm_bind_memory": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "lbm_set_boundaries": [ctypes.c_void_p, ctypes.POINTER(Boundaries)],
    "lbm_init_equilibrium": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_int, ctypes.c_int64],
    "lbm_set_populations": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64],
    "lbm_get_populations": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "lbm_step": [ctypes.c_void_p, ctypes.c_int64],
    "lbm_get_macroscopic": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                            ctypes.c_int],
    "lbm_reduce": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)],
    "lbm_reduce_static": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_set_check": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double],
    "lbm_stats_accumulate": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_set_solids": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_set_links": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64],
    "lbm_jet_fit": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                    ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                    ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                    ctypes.c_void_p],
    "lbm_jet_profile": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                        ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_stats_finalize": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                           ctypes.c_int, ctypes.c_int],
    "lbm_state_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lbm_save_state": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)],
    "lbm_load_state": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64,
                       ctypes.c_int32],
    "lbm_get_time": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)],
    "lbm_set_stream": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_destroy": [ctypes.c_void_p],
    "lbm_strerror": [ctypes.c_int],
    "lbm_stream_copy": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "lbm_probe_ke": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                     ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_int,
                     ctypes.POINTER(ctypes.c_double)],
    "lbm_step_record": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "lbm_adjoint_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_int, ctypes.c_void_p],
    "lbm_refined_create": [ctypes.POINTER(Config), ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_void_p)],
    "lbm_refined_geometry": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)],
    "lbm_refined_types": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8)],
    "lbm_refined_set_solids": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8)],
    "lbm_refined_set_links": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_float), ctypes.c_int64],
    "lbm_refined_required_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lbm_refined_bind_memory": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "lbm_refined_set_boundaries": [ctypes.c_void_p, ctypes.POINTER(Boundaries),
                                   ctypes.POINTER(ctypes.c_void_p),
                                   ctypes.POINTER(ctypes.c_void_p)],
    "lbm_refined_init_equilibrium": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int, ctypes.c_int64],
    "lbm_refined_set_populations": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_int64],
    "lbm_refined_get_populations": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int],
    "lbm_refined_step": [ctypes.c_void_p, ctypes.c_int64],
    "lbm_refined_get_macroscopic": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_int],
    "lbm_refined_reduce": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)],
    "lbm_refined_get_time": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)],
    "lbm_refined_set_stream": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_refined_destroy": [ctypes.c_void_p],
}


def lib():
    """The loaded ``liblbm.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so is not built: run python -m paper_1206_0389_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "lbm_strerror" else ctypes.c_int
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def strerror(status: int) -> str:
    return lib().lbm_strerror(int(status)).decode()


def _check(rc, where):
    if rc != OK:
        raise LbmError(rc, where)
    return rc


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return DTYPE_F64
    if t.dtype == torch.float32:
        return DTYPE_F32
    raise TypeError("fields must be float64 or float32, got %s" % t.dtype)


def _dev(t: torch.Tensor):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---- C ABI mirrors -------------------------------------------------------

def create_lattice(cfg: Config):
    h = ctypes.c_void_p()
    _check(lib().lbm_create_lattice(ctypes.byref(cfg), ctypes.byref(h)), "lbm_create_lattice")
    return h


def required_bytes(h) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbm_required_bytes(h, ctypes.byref(n)), "lbm_required_bytes")
    return n.value


def bind_memory(h, block: torch.Tensor):
    _check(lib().lbm_bind_memory(h, _dev(block), block.numel() * block.element_size()),
           "lbm_bind_memory")


def set_boundaries(h, bc: Boundaries):
    _check(lib().lbm_set_boundaries(h, ctypes.byref(bc)), "lbm_set_boundaries")


def init_equilibrium(h, drho: torch.Tensor, u: torch.Tensor, t0: int = 0):
    code = _dtype_code(drho)
    assert u.dtype == drho.dtype
    _check(lib().lbm_init_equilibrium(h, _dev(drho), _dev(u), code, int(t0)),
           "lbm_init_equilibrium")


def set_populations(h, f: torch.Tensor, t0: int = 0):
    _check(lib().lbm_set_populations(h, _dev(f), _dtype_code(f), int(t0)), "lbm_set_populations")


def get_populations(h, f: torch.Tensor):
    _check(lib().lbm_get_populations(h, _dev(f), _dtype_code(f)), "lbm_get_populations")


def step(h, n: int):
    _check(lib().lbm_step(h, int(n)), "lbm_step")


def get_macroscopic(h, rho, u, rho_mode=RHO_DEVIATION):
    ref = rho if rho is not None else u
    code = _dtype_code(ref)
    _check(lib().lbm_get_macroscopic(h, _dev(rho) if rho is not None else None,
                                     _dev(u) if u is not None else None, code, int(rho_mode)),
           "lbm_get_macroscopic")


def reduce(h, check: bool = True):
    out = (ctypes.c_double * 5)()
    rc = lib().lbm_reduce(h, out)
    if check:
        _check(rc, "lbm_reduce")
    return list(out), rc


def set_solids(h, solid, masks):
    if solid is None:
        _check(lib().lbm_set_solids(h, None, None), "lbm_set_solids")
        return
    if solid.dtype != torch.uint8 or masks.dtype != torch.int32 or masks.numel() != solid.numel():
        raise TypeError("solid must be uint8 and masks int32 of the same size")
    _check(lib().lbm_set_solids(h, _dev(solid), _dev(masks)), "lbm_set_solids")


def set_links(h, nodes, q):
    if nodes is None:
        _check(lib().lbm_set_links(h, None, None, 0), "lbm_set_links")
        return
    if nodes.dtype != torch.int32 or q.dtype != torch.float32:
        raise TypeError("nodes must be int32 and q float32")
    if q.dim() != 2 or q.shape[0] != nodes.numel():
        raise TypeError("q must be [n][Q] for n nodes")
    _check(lib().lbm_set_links(h, _dev(nodes), _dev(q), int(nodes.numel())), "lbm_set_links")


def jet_profile(h, mean, axis, center, ndir, dr, nr, um, re, prof=None):
    for t in (um, re) + ((prof,) if prof is not None else ()):
        if t.dtype != torch.float64:
            raise TypeError("um, re and prof must be float64")
    _check(lib().lbm_jet_profile(h, _dev(mean), _dtype_code(mean), int(axis), float(center[0]),
                                 float(center[1]), int(ndir), float(dr), int(nr), _dev(um),
                                 _dev(re), _dev(prof) if prof is not None else None),
           "lbm_jet_profile")


def stats_accumulate(h, sums: torch.Tensor):
    if sums.dtype != torch.float64:
        raise TypeError("sums must be float64")
    _check(lib().lbm_stats_accumulate(h, _dev(sums)), "lbm_stats_accumulate")


def stats_finalize(h, sums, count, mean, rms, ti=None, axis=2, point=(0, 0)):
    if sums.dtype != torch.float64:
        raise TypeError("sums must be float64")
    code = _dtype_code(mean)
    if rms.dtype != mean.dtype or (ti is not None and ti.dtype != mean.dtype):
        raise TypeError("mean, rms and ti must share one dtype")
    _check(lib().lbm_stats_finalize(h, _dev(sums), int(count), _dev(mean), _dev(rms),
                                    _dev(ti) if ti is not None else None, code, int(axis),
                                    int(point[0]), int(point[1])), "lbm_stats_finalize")


def state_bytes(h) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbm_state_bytes(h, ctypes.byref(n)), "lbm_state_bytes")
    return n.value


def save_state(h, buf: torch.Tensor):
    t = ctypes.c_int64()
    p = ctypes.c_int32()
    _check(lib().lbm_save_state(h, _dev(buf), buf.numel() * buf.element_size(),
                                ctypes.byref(t), ctypes.byref(p)), "lbm_save_state")
    return t.value, p.value


def load_state(h, buf: torch.Tensor, t: int, parity: int):
    _check(lib().lbm_load_state(h, _dev(buf), buf.numel() * buf.element_size(), int(t),
                                int(parity)), "lbm_load_state")


def get_time(h) -> int:
    t = ctypes.c_int64()
    _check(lib().lbm_get_time(h, ctypes.byref(t)), "lbm_get_time")
    return t.value


def set_stream(h, stream=None):
    _check(lib().lbm_set_stream(h, _stream_handle(stream)), "lbm_set_stream")


def destroy(h):
    lib().lbm_destroy(h)


def stream_copy(dst: torch.Tensor, src: torch.Tensor, nbytes: int, stream=None):
    _check(lib().lbm_stream_copy(_dev(dst), _dev(src), int(nbytes), _stream_handle(stream)),
           "lbm_stream_copy")


def probe_ke(h, lo, hi, lam=None, dtype=DTYPE_F64) -> float:
    lo3 = (ctypes.c_int32 * 3)(*[int(v) for v in lo])
    hi3 = (ctypes.c_int32 * 3)(*[int(v) for v in hi])
    J = ctypes.c_double()
    code = _dtype_code(lam) if lam is not None else dtype
    _check(lib().lbm_probe_ke(h, lo3, hi3, _dev(lam) if lam is not None else None, code,
                              ctypes.byref(J)), "lbm_probe_ke")
    return J.value


def step_record(h, rec: torch.Tensor):
    _check(lib().lbm_step_record(h, _dev(rec), _dtype_code(rec)), "lbm_step_record")


def adjoint_step(h, f: torch.Tensor, lam_next: torch.Tensor, lam: torch.Tensor, grad=None):
    code = _dtype_code(f)
    if _dtype_code(lam_next) != code or _dtype_code(lam) != code:
        raise TypeError("f, lam_next and lam must share one dtype")
    if grad is not None and grad.dtype != torch.float64:
        raise TypeError("grad must be float64")
    _check(lib().lbm_adjoint_step(h, _dev(f), _dev(lam_next), _dev(lam), code,
                                  _dev(grad) if grad is not None else None),
           "lbm_adjoint_step")


# ---- convenience wrapper ---------------------------------------------------

def make_config(model="fclb", storage="f32", shape=(32, 32, 32), nu=0.01, cs_smag=0.0,
                mrt_basis=BASIS_TABLE1, rates=None, stream=None) -> Config:
    c = Config()
    c.model = MODEL[model] if isinstance(model, str) else int(model)
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.nx, c.ny, c.nz = (int(v) for v in shape)
    c.mrt_basis = int(mrt_basis)
    c.nu = float(nu)
    c.cs_smag = float(cs_smag)
    if rates is None:
        c.use_default_rates = 1
    else:
        c.use_default_rates = 0
        for k, v in enumerate(rates):
            c.rates[k] = float(v)
    c.stream = _stream_handle(stream).value
    return c


class Lattice:
    """A lattice whose device block is a torch tensor owned by this object.

    shape = (nx, ny, nz); populations are indexed [Q][nz][ny][nx].
    """

    def __init__(self, model="fclb", storage="f32", shape=(32, 32, 32), nu=0.01,
                 cs_smag=0.0, mrt_basis=BASIS_TABLE1, rates=None, device="cuda", stream=None):
        self.cfg = make_config(model, storage, shape, nu, cs_smag, mrt_basis, rates, stream)
        self.h = create_lattice(self.cfg)
        self.Q = 19 if self.cfg.model == D3Q19_MRT_LES else 27
        self.nx, self.ny, self.nz = self.cfg.nx, self.cfg.ny, self.cfg.nz
        self.N = self.nx * self.ny * self.nz
        self.device = torch.device(device)
        nbytes = required_bytes(self.h)
        self.block = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.block.data_ptr()) % 256
        self._view = self.block[off:off + nbytes]
        bind_memory(self.h, self._view)
        self._keep = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.lbm_destroy(h)
            self.h = None

    @property
    def shape3(self):
        return (self.nz, self.ny, self.nx)

    def set_boundaries(self, faces, face_u=None, inlet_u=None, inlet_mask=None,
                       inlet_amp=0.0, seed=0, face_drho=None):
        """faces: six face types (x-, x+, y-, y+, z-, z+); face_u: WALL
        velocities; face_drho: density deviations of PRESSURE faces."""
        bc = Boundaries()
        for k in range(6):
            bc.face_type[k] = int(faces[k])
        if face_u is not None:
            for k in range(6):
                for c in range(3):
                    bc.face_u[k][c] = float(face_u[k][c])
        if face_drho is not None:
            for k in range(6):
                bc.face_drho[k] = float(face_drho[k])
        keep = []
        dims = (self.nx, self.ny, self.nz)
        if inlet_u is not None:
            d = [k for k in range(6) if int(faces[k]) == INLET]
            if d:
                ax = d[0] // 2
                na = dims[1] if ax == 0 else dims[0]
                nb = dims[1] if ax == 2 else dims[2]
                if tuple(inlet_u.shape) != (3, nb, na):
                    raise ValueError("inlet_u must have shape (3, %d, %d)" % (nb, na))
                if inlet_mask is not None and tuple(inlet_mask.shape) != (nb, na):
                    raise ValueError("inlet_mask must have shape (%d, %d)" % (nb, na))
            iu = inlet_u.to(self.device).contiguous()
            keep.append(iu)
            bc.inlet_u = iu.data_ptr()
            bc.inlet_dtype = _dtype_code(iu)
        if inlet_mask is not None:
            im = inlet_mask.to(device=self.device, dtype=torch.uint8).contiguous()
            keep.append(im)
            bc.inlet_mask = im.data_ptr()
        bc.inlet_amp = float(inlet_amp)
        bc.seed = int(seed)
        set_boundaries(self.h, bc)
        self._keep = keep
        self._solid_bufs = None  # new boundaries clear the solids and links
        self._link_bufs = None

    def _expect(self, t, shape, what):
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s must have shape %s, got %s" % (what, shape, tuple(t.shape)))

    def init_equilibrium(self, drho, u, t0=0):
        drho = torch.as_tensor(drho).to(self.device).contiguous()
        u = torch.as_tensor(u).to(device=self.device, dtype=drho.dtype).contiguous()
        self._expect(drho, self.shape3, "drho")
        self._expect(u, (3,) + self.shape3, "u")
        init_equilibrium(self.h, drho, u, t0)

    def set_populations(self, f, t0=0):
        f = torch.as_tensor(f).to(self.device).contiguous()
        self._expect(f, (self.Q,) + self.shape3, "f")
        set_populations(self.h, f, t0)

    def populations(self, dtype=torch.float64):
        out = torch.empty((self.Q,) + self.shape3, dtype=dtype, device=self.device)
        get_populations(self.h, out)
        return out

    def step(self, n=1):
        step(self.h, n)

    def macroscopic(self, dtype=torch.float64, rho_mode=RHO_DEVIATION):
        rho = torch.empty(self.shape3, dtype=dtype, device=self.device)
        u = torch.empty((3,) + self.shape3, dtype=dtype, device=self.device)
        get_macroscopic(self.h, rho, u, rho_mode)
        return rho, u

    def reduce(self, check=True):
        return reduce(self.h, check)[0]

    def set_check(self, every, mass_tol=-1.0):
        """After every `every`-th step, step() checks the FP64 sums: a
        non-finite sum raises LbmError (status ENONFINITE), and with
        mass_tol >= 0 a mass deviation drifted by more than mass_tol from
        its value now raises LbmError (status EMASS). every = 0: off."""
        _check(lib().lbm_set_check(self.h, int(every), float(mass_tol)), "lbm_set_check")

    def reduce_static(self, out):
        """The sums of reduce() into a device float64 tensor of 5 elements,
        stream-ordered, with the library's static partial-sum buffer (no
        allocation, no synchronisation)."""
        if out.dtype != torch.float64 or out.numel() < 5 or not out.is_cuda \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous CUDA float64 tensor of 5 elements")
        rc = lib().lbm_reduce_static(self.h, ctypes.c_void_p(out.data_ptr()))
        where = "lbm_reduce_static"
        if rc == EINVAL:
            where += " (an x-y plane of %d x %d nodes above the static buffer's 16384 " \
                     "blocks of 256?)" % (self.nx, self.ny)
        _check(rc, where)
        return out

    def set_solids(self, solid):
        """Interior solid nodes from a [nz][ny][nx] mask (nonzero = solid;
        None clears them). The library keeps a per-node mask buffer owned by
        this object until the solids are cleared or the boundaries reset."""
        if solid is None:
            set_solids(self.h, None, None)
            self._solid_bufs = None
            self._link_bufs = None
            return
        solid = torch.as_tensor(solid).to(device=self.device, dtype=torch.uint8).contiguous()
        self._expect(solid, self.shape3, "solid")
        masks = torch.empty(self.shape3, dtype=torch.int32, device=self.device)
        self._solid_bufs = None
        self._link_bufs = None
        set_solids(self.h, solid, masks)
        self._solid_bufs = (solid, masks)

    def set_links(self, nodes, q=None):
        """Curved walls: Bouzidi's interpolated bounce-back on the links of
        the listed fluid nodes (int32 linear indices x + nx (y + ny z)) to
        solid neighbours, q[j][k] the wall's distance along direction k as a
        fraction of the link (other entries ignored); None clears them. The
        solids must be set first; the buffers are kept by this object."""
        if nodes is None:
            set_links(self.h, None, None)
            self._link_bufs = None
            return
        nodes = torch.as_tensor(nodes).to(device=self.device, dtype=torch.int32).contiguous()
        q = torch.as_tensor(q).to(device=self.device, dtype=torch.float32).contiguous()
        self._expect(q, (nodes.numel(), self.Q), "q")
        set_links(self.h, nodes, q)
        self._link_bufs = (nodes, q)

    def jet_profile(self, mean, axis=2, center=None, ndir=32, dr=0.5, nr=64, profile=True):
        """Spreading of the jet from a mean velocity [3][nz][ny][nx] (float64
        or float32): per cross-section normal to axis, u_m at the centre (the
        two other coordinates in increasing order; default the lattice's
        middle), the radius where the bilinear mean falls to 0.368 u_m on
        ndir rays (min, max, mean) and the ray-averaged profile u(k dr) / u_m
        (k < nr). Returns (um [n_p], re [3][n_p], prof [n_p][nr] or None)."""
        self._expect(mean, (3,) + self.shape3, "mean")
        n3 = (self.nx, self.ny, self.nz)
        other = [d for d in range(3) if d != axis]
        if center is None:
            center = tuple((n3[d] - 1) / 2.0 for d in other)
        f64 = dict(dtype=torch.float64, device=self.device)
        um = torch.empty(n3[axis], **f64)
        re = torch.empty((3, n3[axis]), **f64)
        prof = torch.empty((n3[axis], nr), **f64) if profile else None
        jet_profile(self.h, mean.contiguous(), axis, center, ndir, dr, nr, um, re, prof)
        return um, re, prof

    def jet_fit(self, um, re, prof, dr, x0, u0, d, p0=0, p1=None):
        """Jet laws fitted to a jet_profile result (Eqs. (22)-(24)): returns
        a float64 device tensor (k_par, k_perp, profile residual, number of
        profile samples) over the sections p0 <= p < p1 past the exit x0."""
        np_ = um.numel()
        p1 = np_ if p1 is None else p1
        self._expect(re, (3, np_), "re")
        if prof is None or prof.dim() != 2 or prof.shape[0] != np_:
            raise ValueError("prof must be [n_p][nr]")
        for t in (um, re, prof):
            if t.dtype != torch.float64:
                raise TypeError("um, re and prof must be float64")
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        _check(lib().lbm_jet_fit(self.h, _dev(um), _dev(re), _dev(prof), int(np_),
                                 int(prof.shape[1]), float(dr), float(x0), float(u0), float(d),
                                 int(p0), int(p1), _dev(out)), "lbm_jet_fit")
        return out

    def stats_buffer(self):
        """Zeroed FP64 running sums for stats_accumulate ([6][nz][ny][nx])."""
        return torch.zeros((6,) + self.shape3, dtype=torch.float64, device=self.device)

    def stats_accumulate(self, sums):
        """Add the current velocity (and its squares) to the running sums."""
        self._expect(sums, (6,) + self.shape3, "sums")
        stats_accumulate(self.h, sums)

    def stats_finalize(self, sums, count, axis=2, point=None, dtype=torch.float64):
        """Mean velocity, rms fluctuation ([3][nz][ny][nx] each) and, if the
        jet-axis point (the two coordinates other than axis, increasing
        order) is given, the turbulent intensity of Eq. (25) ([nz][ny][nx])."""
        self._expect(sums, (6,) + self.shape3, "sums")
        mean = torch.empty((3,) + self.shape3, dtype=dtype, device=self.device)
        rms = torch.empty_like(mean)
        ti = torch.empty(self.shape3, dtype=dtype, device=self.device) if point is not None \
            else None
        stats_finalize(self.h, sums, count, mean, rms, ti, axis,
                       point if point is not None else (0, 0))
        return mean, rms, ti

    def save_state(self):
        buf = torch.empty(state_bytes(self.h), dtype=torch.uint8, device=self.device)
        t, p = save_state(self.h, buf)
        return buf, t, p

    def load_state(self, buf, t, parity):
        load_state(self.h, buf, t, parity)

    @property
    def time(self):
        return get_time(self.h)

    @property
    def adjoint_dtype(self):
        """Arithmetic type of the adjoint: float64 for FP64 storage, else float32."""
        return torch.float64 if self.cfg.storage == STORAGE["f64"] else torch.float32

    def probe_ke(self, lo, hi, lam=None):
        """Mean |j|^2 / (2 rho) over the box [lo, hi) (x, y, z order) of the
        current state; lam, if given ([Q][nz][ny][nx]), receives dJ/df."""
        if lam is not None:
            self._expect(lam, (self.Q,) + self.shape3, "lam")
        return probe_ke(self.h, lo, hi, lam)

    def step_record(self, rec):
        """One step, writing the pre-collision state it collides into rec."""
        self._expect(rec, (self.Q,) + self.shape3, "rec")
        step_record(self.h, rec)

    def adjoint_step(self, f, lam_next, lam, grad=None):
        for t, what in ((f, "f"), (lam_next, "lam_next"), (lam, "lam")):
            self._expect(t, (self.Q,) + self.shape3, what)
        adjoint_step(self.h, f, lam_next, lam, grad)


class RefinedLattice:
    """Nested time refinement on a block grid (C ABI lbm_refined_*).

    shape = level-0 (nx, ny, nz); level_map = uint8 [nz/B][ny/B][nx/B], the
    finest level of each block (``mask``, a 0/1 map, gives two levels).
    Boundaries (faces, face_u, inlet arrays per level: ``level_inlet_u`` /
    ``level_inlet_mask`` lists indexed by level, entry 0 unused, or for two
    levels ``fine_inlet_u`` / ``fine_inlet_mask``), solids and curved links are
    set before the device block is bound, as the ABI requires. ``solids``:
    per-level list of uint8 masks over the level's whole domain (nz_l, ny_l,
    nx_l) or None; ``links``: per-level list of (nodes, q) with nodes linear
    indices over the level's whole domain and q [n][Q] float32, or None.
    Every level holds post-collision populations over its box: ``levels[l]``
    gives its origin ``lo`` (x, y, z), extent ``dims`` (x pitch, y, z) and
    node counts; ``shape3(l)`` is (dims z, dims y, dims x).
    """

    def __init__(self, model="fclb", storage="f32", shape=(32, 32, 32), nu=0.01, cs_smag=0.0,
                 mrt_basis=BASIS_TABLE1, rates=None, block=16, level_map=None, nlevels=None,
                 mask=None, faces=None, face_u=None, inlet_u=None, inlet_mask=None,
                 level_inlet_u=None, level_inlet_mask=None, fine_inlet_u=None,
                 fine_inlet_mask=None, inlet_amp=0.0, seed=0, solids=None, links=None,
                 device="cuda", stream=None, face_drho=None):
        import numpy as np
        self.cfg = make_config(model, storage, shape, nu, cs_smag, mrt_basis, rates, stream)
        self.Q = 19 if self.cfg.model == D3Q19_MRT_LES else 27
        self.nx, self.ny, self.nz = self.cfg.nx, self.cfg.ny, self.cfg.nz
        self.device = torch.device(device)
        if level_map is None:
            level_map = mask
        m = np.ascontiguousarray(level_map, dtype=np.uint8)
        if m.shape != (self.nz // block, self.ny // block, self.nx // block):
            raise ValueError("level map must have shape (nz/B, ny/B, nx/B)")
        self.L = int(nlevels) if nlevels is not None else int(m.max()) + 1
        self._map = m
        self.h = ctypes.c_void_p()
        _check(lib().lbm_refined_create(ctypes.byref(self.cfg), int(block), self.L,
                                        m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        ctypes.byref(self.h)), "lbm_refined_create")
        self._keep = []
        if level_inlet_u is None and fine_inlet_u is not None:
            level_inlet_u = [None, fine_inlet_u]
            level_inlet_mask = [None, fine_inlet_mask]
        if faces is not None:
            bc = Boundaries()
            for k in range(6):
                bc.face_type[k] = int(faces[k])
            if face_u is not None:
                for k in range(6):
                    for c in range(3):
                        bc.face_u[k][c] = float(face_u[k][c])
            if face_drho is not None:
                for k in range(6):
                    bc.face_drho[k] = float(face_drho[k])
            ptr_u = (ctypes.c_void_p * self.L)()
            ptr_m = (ctypes.c_void_p * self.L)()
            if inlet_u is not None:
                ax = [k for k in range(6) if int(faces[k]) == INLET][0] // 2
                dims = (self.nx, self.ny, self.nz)
                na = dims[1] if ax == 0 else dims[0]
                nb = dims[1] if ax == 2 else dims[2]
                iu = inlet_u.to(self.device).contiguous()
                if tuple(iu.shape) != (3, nb, na):
                    raise ValueError("inlet_u must be (3, nb, na)")
                self._keep.append(iu)
                bc.inlet_u = iu.data_ptr()
                bc.inlet_dtype = _dtype_code(iu)
                if inlet_mask is not None:
                    im = inlet_mask.to(device=self.device, dtype=torch.uint8).contiguous()
                    if tuple(im.shape) != (nb, na):
                        raise ValueError("inlet_mask must be (nb, na)")
                    self._keep.append(im)
                    bc.inlet_mask = im.data_ptr()
                for l in range(1, self.L):
                    lu = level_inlet_u[l].to(device=self.device, dtype=iu.dtype).contiguous()
                    if tuple(lu.shape) != (3, nb << l, na << l):
                        raise ValueError("level %d inlet_u must be (3, %d, %d)"
                                         % (l, nb << l, na << l))
                    self._keep.append(lu)
                    ptr_u[l] = lu.data_ptr()
                    if inlet_mask is not None:
                        lm = level_inlet_mask[l].to(device=self.device,
                                                    dtype=torch.uint8).contiguous()
                        if tuple(lm.shape) != (nb << l, na << l):
                            raise ValueError("level %d inlet_mask must be (%d, %d)"
                                             % (l, nb << l, na << l))
                        self._keep.append(lm)
                        ptr_m[l] = lm.data_ptr()
            bc.inlet_amp = float(inlet_amp)
            bc.seed = int(seed)
            _check(lib().lbm_refined_set_boundaries(self.h, ctypes.byref(bc), ptr_u, ptr_m),
                   "lbm_refined_set_boundaries")
        self._geometry()
        for l in range(self.L):
            sm = solids[l] if solids is not None and l < len(solids) else None
            if sm is not None:
                box = self._to_box(l, np.asarray(sm, dtype=np.uint8))
                _check(lib().lbm_refined_set_solids(
                    self.h, l, box.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
                    "lbm_refined_set_solids")
            lk = links[l] if links is not None and l < len(links) else None
            if lk is not None:
                nodes, q = self._links_to_box(l, *lk)
                _check(lib().lbm_refined_set_links(
                    self.h, l, nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    q.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), len(nodes)),
                    "lbm_refined_set_links")
        self._geometry()
        n = ctypes.c_size_t()
        _check(lib().lbm_refined_required_bytes(self.h, ctypes.byref(n)),
               "lbm_refined_required_bytes")
        self.block = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self.block.data_ptr()) % 256
        self._view = self.block[off:off + n.value]
        _check(lib().lbm_refined_bind_memory(self.h, _dev(self._view), n.value),
               "lbm_refined_bind_memory")

    def _geometry(self):
        self.levels = []
        for l in range(self.L):
            lo = (ctypes.c_int32 * 3)()
            dims = (ctypes.c_int32 * 3)()
            cnt = (ctypes.c_int64 * 5)()
            _check(lib().lbm_refined_geometry(self.h, l, lo, dims, cnt), "lbm_refined_geometry")
            self.levels.append({"lo": tuple(lo), "dims": tuple(dims),
                                "n": (self.nx << l, self.ny << l, self.nz << l),
                                "counts": dict(zip(("fluid", "band", "covered", "ghost",
                                                    "solid"), tuple(cnt)))})
        if self.L > 1:  # the two-level names used by callers of the fine level
            self.fine_lo = self.levels[1]["lo"]
            self.fine_dims = self.levels[1]["dims"]
        c = {k: 0 for k in ("fluid", "band", "covered", "ghost", "solid")}
        for v in self.levels[1:]:
            c["fluid"] += v["counts"]["fluid"] + v["counts"]["band"]
            c["ghost"] += v["counts"]["ghost"]
        c["covered"] = sum(v["counts"]["covered"] for v in self.levels)
        c["band"] = sum(v["counts"]["band"] for v in self.levels)
        self.counts = c

    def box_slices(self, level):
        """(z, y, x) slices of the box in the level's domain and, for x, the
        number of box columns inside the domain."""
        v = self.levels[level]
        (ox, oy, oz), (mx, my, mz), (nx, _, _) = v["lo"], v["dims"], v["n"]
        wx = min(mx, nx - ox)
        return slice(oz, oz + mz), slice(oy, oy + my), slice(ox, ox + wx), wx

    def to_box(self, level, a):
        """A [..., nz_l, ny_l, nx_l] array of the level's whole domain cut to
        its box (columns beyond the domain zero)."""
        import numpy as np
        sz, sy, sx, wx = self.box_slices(level)
        mx, my, mz = self.levels[level]["dims"]
        out = np.zeros(a.shape[:-3] + (mz, my, mx), dtype=a.dtype)
        out[..., :wx] = a[..., sz, sy, sx]
        return out

    _to_box = to_box

    def _links_to_box(self, level, nodes, q):
        import numpy as np
        nx, ny, nz = self.levels[level]["n"]
        (ox, oy, oz), (mx, my, mz) = self.levels[level]["lo"], self.levels[level]["dims"]
        nodes = np.asarray(nodes, dtype=np.int64)
        x, y, z = nodes % nx, (nodes // nx) % ny, nodes // (nx * ny)
        bx, by, bz = x - ox, y - oy, z - oz
        keep = (bx >= 0) & (bx < mx) & (by >= 0) & (by < my) & (bz >= 0) & (bz < mz)
        box = ((bz * my + by) * mx + bx)[keep].astype(np.int32)
        return np.ascontiguousarray(box), np.ascontiguousarray(np.asarray(q, np.float32)[keep])

    def types(self, level):
        import numpy as np
        t = np.zeros(self.shape3(level), dtype=np.uint8)
        _check(lib().lbm_refined_types(self.h, level,
                                       t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
               "lbm_refined_types")
        return t

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.lbm_refined_destroy(h)
            self.h = None

    def shape3(self, level):
        d = self.levels[level]["dims"]
        return (d[2], d[1], d[0])

    def init_equilibrium(self, level, drho, u, t0=0):
        drho = torch.as_tensor(drho).to(self.device).contiguous()
        u = torch.as_tensor(u).to(device=self.device, dtype=drho.dtype).contiguous()
        if tuple(drho.shape) != self.shape3(level) or tuple(u.shape) != (3,) + self.shape3(level):
            raise ValueError("field shapes do not match level %d" % level)
        _check(lib().lbm_refined_init_equilibrium(self.h, int(level), _dev(drho), _dev(u),
                                                  _dtype_code(drho), int(t0)),
               "lbm_refined_init_equilibrium")

    def set_populations(self, level, f, t0=0):
        f = torch.as_tensor(f).to(self.device).contiguous()
        if tuple(f.shape) != (self.Q,) + self.shape3(level):
            raise ValueError("population shape does not match level %d" % level)
        _check(lib().lbm_refined_set_populations(self.h, int(level), _dev(f), _dtype_code(f),
                                                 int(t0)), "lbm_refined_set_populations")

    def populations(self, level, dtype=torch.float64):
        out = torch.empty((self.Q,) + self.shape3(level), dtype=dtype, device=self.device)
        _check(lib().lbm_refined_get_populations(self.h, int(level), _dev(out),
                                                 _dtype_code(out)),
               "lbm_refined_get_populations")
        return out

    def step(self, n=1):
        _check(lib().lbm_refined_step(self.h, int(n)), "lbm_refined_step")

    def macroscopic(self, level, dtype=torch.float64, rho_mode=RHO_DEVIATION):
        rho = torch.empty(self.shape3(level), dtype=dtype, device=self.device)
        u = torch.empty((3,) + self.shape3(level), dtype=dtype, device=self.device)
        _check(lib().lbm_refined_get_macroscopic(self.h, int(level), _dev(rho), _dev(u),
                                                 _dtype_code(rho), int(rho_mode)),
               "lbm_refined_get_macroscopic")
        return rho, u

    def reduce(self, check=True):
        out = (ctypes.c_double * 5)()
        rc = lib().lbm_refined_reduce(self.h, out)
        if check:
            _check(rc, "lbm_refined_reduce")
        return list(out)

    @property
    def time(self):
        t = ctypes.c_int64()
        _check(lib().lbm_refined_get_time(self.h, ctypes.byref(t)), "lbm_refined_get_time")
        return t.value
