"""Convenience layer over the C ABI: one periodic system (or replica batch) on the GPU.

Holds device tensors and a context, calls the entry points in order, and
retries a Verlet run whose neighbour rows overflowed (the context grows its
capacity when ``md_get_status`` reports it).  ``MDForces`` exposes forces and
energies to torch.autograd with the hand-written adjoint as backward.
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np
import torch

from . import binding as B


def _dev(a, device):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device).contiguous()


class MDSystem:
    def __init__(self, pos, boxes, offsets, pot, skin: float, vel=None, device: str = "cuda"):
        self.device = device
        self.pot = pot
        self.dpot = B.DevicePotential(pot, device=device)
        self.boxes = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 3))
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.skin = float(skin)
        self.pos = pos if isinstance(pos, torch.Tensor) else _dev(pos, device)
        self.n = int(self.pos.shape[1])
        self.vel = (torch.zeros_like(self.pos) if vel is None
                    else (vel if isinstance(vel, torch.Tensor) else _dev(vel, device)))
        self.ctx = B.Context(self.n, self.offsets)
        self.R = self.ctx.n_replicas
        self._built = None

    @classmethod
    def from_workload(cls, w, device: str = "cuda", pos=None):
        return cls(w.pos if pos is None else pos, w.boxes, w.offsets, w.pot, w.skin, vel=w.vel,
                   device=device)

    # -------------------------------------------------------------- building blocks
    def build(self, kind: int = B.MD_LIST_FULL, pos: Optional[torch.Tensor] = None):
        p = self.pos if pos is None else pos
        B.md_build_cells(self.ctx, p, self.boxes, self.pot.rc, self.skin)
        B.md_build_neighbor_list(self.ctx, kind)
        self._built = (p.data_ptr(), p._version, kind)

    def forces(self, precision: int = B.MD_FP64, kind: int = B.MD_LIST_FULL,
               rebuild: bool = True, dpot: Optional[B.DevicePotential] = None):
        """(F [3][N], E [R], W [R]) at self.pos."""
        if rebuild:
            self.build(kind)
        F = torch.empty_like(self.pos)
        E = torch.zeros(self.R, dtype=torch.float64, device=self.device)
        W = torch.zeros(self.R, dtype=torch.float64, device=self.device)
        B.md_compute_forces(self.ctx, dpot or self.dpot, precision, F, E, W)
        return F, E, W

    def run(self, n_steps: int, dt: float, mass: float = 1.0, precision: int = B.MD_FP64,
            kind: int = B.MD_LIST_FULL, record: bool = True, max_retries: int = 3, every: int = 1):
        """Velocity Verlet in place on self.pos / self.vel.  Returns (forces,
        hist [ceil(n_steps / every)][3] (E_pot, KE, W after steps every,
        2 every, ... and the last) or None, rebuild count)."""
        if self._built is None:
            B.md_build_cells(self.ctx, self.pos, self.boxes, self.pot.rc, self.skin)
        x0, v0 = self.pos.clone(), self.vel.clone()
        F = torch.empty_like(self.pos)
        rows = (n_steps + every - 1) // every
        hist = torch.zeros((rows, 3), dtype=torch.float64, device=self.device) if record else None
        nreb = torch.zeros(1, dtype=torch.int32, device=self.device)
        for _ in range(max_retries + 1):
            B.md_verlet_step(self.ctx, self.dpot, precision, kind, self.pos, self.vel, F, dt, mass,
                             n_steps, hist, nreb, hist_every=every)
            code, flags, cap = B.md_get_status(self.ctx)
            if code == B.MD_OK:
                self._built = None
                return F, hist, int(nreb.item())
            if code != B.MD_ERR_CAPACITY:
                raise B.MDError(code, f"device flags {flags}")
            self.pos.copy_(x0)
            self.vel.copy_(v0)
        raise B.MDError(B.MD_ERR_CAPACITY, "neighbour list overflow persisted")

    def vjp(self, u, vE=None, precision: int = B.MD_FP64, rebuild: bool = True,
            dpot: Optional[B.DevicePotential] = None):
        """(g_pos [3][N], g_params) of sum_r vE_r E_r + u.F at self.pos."""
        if rebuild:
            self.build(B.MD_LIST_FULL)
        dp = dpot or self.dpot
        u = u if isinstance(u, torch.Tensor) else _dev(u, self.device)
        vE = (torch.zeros(self.R, dtype=torch.float64, device=self.device) if vE is None
              else (vE if isinstance(vE, torch.Tensor) else _dev(np.atleast_1d(vE), self.device)))
        g = torch.empty_like(self.pos)
        gp = torch.zeros(dp.n_params, dtype=torch.float64, device=self.device)
        B.md_force_vjp(self.ctx, dp, precision, None, u, vE, g, gp)
        return g, gp

    def neighbor_list(self):
        return B.md_get_neighbor_list(self.ctx)

    def cells(self):
        return B.md_get_cells(self.ctx)

    def status(self):
        return B.md_get_status(self.ctx)


class MDForces(torch.autograd.Function):
    """(F [3][N], E [R]) = MDForces.apply(pos, params, system, precision).

    Backward runs the hand-written adjoint (md_force_vjp) and returns the
    gradients with respect to pos and to params (LJ {eps, sigma} or the EAM
    tables flattened phi, rho, embed)."""

    @staticmethod
    def forward(ctx, pos, params, system: MDSystem, precision: int = B.MD_FP64):
        dpot = B.DevicePotential(system.pot, device=system.device, params=params.detach().contiguous())
        p = pos.detach().contiguous()
        system.build(B.MD_LIST_FULL, pos=p)
        F = torch.empty_like(p)
        E = torch.zeros(system.R, dtype=torch.float64, device=system.device)
        B.md_compute_forces(system.ctx, dpot, precision, F, E, None)
        ctx.system = system
        ctx.precision = precision
        ctx.dpot = dpot
        ctx.token = system._built
        ctx.save_for_backward(p)
        return F, E

    @staticmethod
    def backward(ctx, gF, gE):
        (p,) = ctx.saved_tensors
        system: MDSystem = ctx.system
        if system._built != ctx.token:
            system.build(B.MD_LIST_FULL, pos=p)
        u = torch.zeros_like(p) if gF is None else gF.contiguous()
        vE = torch.zeros(system.R, dtype=torch.float64, device=p.device) if gE is None else gE.contiguous()
        g = torch.empty_like(p)
        gp = torch.zeros(ctx.dpot.n_params, dtype=torch.float64, device=p.device)
        B.md_force_vjp(system.ctx, ctx.dpot, ctx.precision, None, u, vE, g, gp)
        return g, gp, None, None
