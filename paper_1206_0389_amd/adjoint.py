"""Gradient of a downstream kinetic-energy probe with respect to an inlet
velocity perturbation, through many FCLB or MRT-LES steps, as a
torch.autograd.Function.

The forward pass runs the lattice from a given state with the inlet's u_z
raised by ``delta`` on a square of the inlet face, keeps a copy of the raw
lattice state every ``every`` steps (device-to-device copies), and returns
J = mean |j|^2 / (2 rho) over the probe box after the last step.

The backward pass seeds lambda_T = dJ/df_T (lbm_probe_ke), then walks the
segments in reverse: restore the segment's checkpoint, recompute its steps
while recording each pre-collision state (lbm_step_record), and run
lbm_adjoint_step back through them, which also accumulates dJ/du_in on the
inlet face. With ``every`` about sqrt(nsteps) the memory is two sets of
sqrt(nsteps) states and the work one extra forward pass.

All arithmetic runs in the library's HIP kernels; torch only provides the
device buffers and the stream.
"""
from __future__ import annotations

import math

import torch

from . import INLET, Lattice, save_state, state_bytes


class InletProbeObjective:
    """J(delta) for a lattice with an INLET face.

    lattice: a Lattice (FCLB or MRT-LES; FP64 or FP32 storage).
    faces, face_u: boundary description as for Lattice.set_boundaries.
    base_inlet_u: [3, nb, na] float64 inlet velocity without the perturbation.
    square: (b0, b1, a0, a1) index bounds of the perturbed square on the face.
    probe_lo, probe_hi: probe box [lo, hi) in (x, y, z).
    nsteps: steps from the initial state; every: checkpoint spacing (default
    about sqrt(nsteps)).
    f0: initial pre-collision deviations [Q][nz][ny][nx] (default: rest).
    t0: time of the initial state.
    """

    def __init__(self, lattice: Lattice, faces, face_u, base_inlet_u, square, probe_lo,
                 probe_hi, nsteps, every=None, f0=None, t0=0):
        if INLET not in [int(f) for f in faces]:
            raise ValueError("the objective needs an INLET face")
        self.lat = lattice
        self.faces = list(faces)
        self.face_u = face_u
        self.base = torch.as_tensor(base_inlet_u, dtype=torch.float64).to(lattice.device)
        self.square = tuple(int(v) for v in square)
        self.lo = tuple(int(v) for v in probe_lo)
        self.hi = tuple(int(v) for v in probe_hi)
        self.nsteps = int(nsteps)
        self.every = int(every) if every else max(1, int(round(math.sqrt(self.nsteps))))
        self.f0 = None if f0 is None else torch.as_tensor(f0).to(lattice.device).contiguous()
        self.t0 = int(t0)
        self._ckpt = []   # (buffer, t, parity) at the start of each segment
        self._final = None
        self._rec = []    # recorded pre-collision states of one segment
        self._inlet = None
        self._fwd_inlet = None  # inlet of the last forward pass (its checkpoints)
        self.forward_count = 0  # forward passes so far (checkpoint generation)

    # -- forward ----------------------------------------------------------
    def _reset(self, delta):
        lat = self.lat
        b0, b1, a0, a1 = self.square
        inlet = self.base.clone()
        inlet[2, b0:b1, a0:a1] += delta.detach().to(device=inlet.device, dtype=torch.float64)
        if self.f0 is None:
            z = torch.zeros(lat.shape3, dtype=torch.float64, device=lat.device)
            lat.init_equilibrium(z, torch.zeros((3,) + lat.shape3, dtype=torch.float64,
                                                device=lat.device), t0=self.t0)
        else:
            lat.set_populations(self.f0, t0=self.t0)
        lat.set_boundaries(self.faces, face_u=self.face_u, inlet_u=inlet)
        self._inlet = inlet

    def _buffers(self, nseg):
        while len(self._ckpt) < nseg:
            self._ckpt.append([None, 0, 0])
        for c in self._ckpt[:nseg]:
            if c[0] is None:
                c[0] = torch.empty(self._state_bytes(), dtype=torch.uint8, device=self.lat.device)
        if self._final is None:
            self._final = [torch.empty(self._state_bytes(), dtype=torch.uint8,
                                       device=self.lat.device), 0, 0]

    def _state_bytes(self):
        return state_bytes(self.lat.h)

    def forward(self, delta) -> float:
        lat = self.lat
        self._reset(delta)
        nseg = (self.nsteps + self.every - 1) // self.every
        self._buffers(nseg)
        for s in range(nseg):
            c = self._ckpt[s]
            c[1], c[2] = save_state(lat.h, c[0])
            lat.step(min(self.every, self.nsteps - s * self.every))
        self._final[1], self._final[2] = save_state(lat.h, self._final[0])
        self._fwd_inlet = self._inlet
        self.forward_count += 1
        return lat.probe_ke(self.lo, self.hi)

    def value(self, delta) -> float:
        """J(delta) without keeping checkpoints (for finite differences). The
        checkpoints of the last forward pass stay valid: backward restores that
        pass's inlet before recomputing."""
        self._reset(delta)
        self.lat.step(self.nsteps)
        return self.lat.probe_ke(self.lo, self.hi)

    # -- backward ---------------------------------------------------------
    def backward(self):
        """dJ/du_in on the whole inlet face ([3, nb, na], float64) and
        dJ/df at the initial state, for the last forward pass (whatever ran
        since: a value() call changes the lattice's inlet, so the forward
        pass's boundaries are applied again, at the first checkpoint, whose
        in-place parity is even)."""
        if self.forward_count == 0:
            raise RuntimeError("backward needs a forward pass first")
        lat = self.lat
        nseg = (self.nsteps + self.every - 1) // self.every
        # the first checkpoint, or with no step the final (= initial) state
        buf, t, parity = self._ckpt[0] if nseg > 0 else self._final
        lat.load_state(buf, t, parity)
        lat.set_boundaries(self.faces, face_u=self.face_u, inlet_u=self._fwd_inlet)
        self._inlet = self._fwd_inlet
        dt = lat.adjoint_dtype
        shape = (lat.Q,) + lat.shape3
        lam = torch.empty(shape, dtype=dt, device=lat.device)
        lam2 = torch.empty_like(lam)
        lat.load_state(self._final[0], self._final[1], self._final[2])
        lat.probe_ke(self.lo, self.hi, lam)
        grad = torch.zeros_like(self._inlet)
        while len(self._rec) < self.every:
            self._rec.append(torch.empty(shape, dtype=dt, device=lat.device))
        for s in reversed(range(nseg)):
            buf, t, parity = self._ckpt[s]
            lat.load_state(buf, t, parity)
            n = min(self.every, self.nsteps - s * self.every)
            for k in range(n):
                lat.step_record(self._rec[k])
            for k in reversed(range(n)):
                lat.adjoint_step(self._rec[k], lam, lam2, grad)
                lam, lam2 = lam2, lam
        return grad, lam

    def __call__(self, delta):
        return _ProbeKE.apply(delta, self)


class _ProbeKE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, delta, obj):
        J = obj.forward(delta)
        ctx.obj = obj
        ctx.generation = obj.forward_count
        ctx.dtype = delta.dtype
        return torch.tensor(J, dtype=torch.float64, device=delta.device)

    @staticmethod
    def backward(ctx, gJ):
        if ctx.obj.forward_count != ctx.generation:
            raise RuntimeError("the objective ran another forward pass after the one being "
                               "differentiated: its checkpoints are gone")
        grad, _ = ctx.obj.backward()
        b0, b1, a0, a1 = ctx.obj.square
        g = grad[2, b0:b1, a0:a1]
        return (gJ.to(g.device) * g).to(ctx.dtype), None
