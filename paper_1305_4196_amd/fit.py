"""Batched differentiation for potential fitting: many replicas, one graph.

A batch of uneven-size replicas (one context, all replicas' bricks in each
persistent launch) is fitted to target forces.  One gradient evaluation is

    F      = forces(theta)                                  (md_compute_forces)
    u      = 2 (F - F*) / (3 N)                              (cotangent of the loss)
    g      = d(u . F)/d theta                                (md_force_vjp, v_E = 0)

(the loss holds no energy term, so the forward pass runs the force kernels
without their energy sums unless `with_energy` asks for the per-replica
energies in `E`)

i.e. the gradient of L = sum |F - F*|^2 / (3 N) with respect to the potential
parameters (LJ {eps, sigma}; EAM the three tables' coefficients).  The cutoff
does not depend on the parameters, so the lists are built once per snapshot
set and the evaluation is a fixed sequence of launches: it is captured in a
HIP graph (torch.cuda.CUDAGraph) and replayed.  The graph holds only the
library's kernels and two element-wise products; it allocates nothing and
records no memset.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import binding as B
from .system import MDSystem


class BatchedFit:
    def __init__(self, system: MDSystem, target_forces: torch.Tensor, params: torch.Tensor,
                 precision: int = B.MD_FP64, with_energy: bool = False, tune: bool = True):
        """tune: pick the brick shape and workgroup size with the autotuner,
        timing forces + adjoint (cached per system signature)."""
        self.s = system
        self.precision = precision
        self.with_energy = with_energy
        self.F_star = target_forces.contiguous()
        self.params = params.detach().clone().contiguous()    # the graph reads this buffer
        self.dpot = B.DevicePotential(system.pot, device=system.device, params=self.params)
        n = system.n
        self.scale = 2.0 / (3.0 * n)
        self.F = torch.empty_like(system.pos)
        self.E = torch.zeros(system.R, dtype=torch.float64, device=system.device)
        self.u = torch.empty_like(system.pos)
        self.vE = torch.zeros(system.R, dtype=torch.float64, device=system.device)
        self.g_pos = torch.empty_like(system.pos)
        self.g = torch.zeros(self.dpot.n_params, dtype=torch.float64, device=system.device)
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.tuning = None
        if tune:
            from . import tune as tuner
            self.tuning = tuner.tune(system, precision=precision, objective="fit")
        system.build(B.MD_LIST_FULL)

    def set_params(self, theta: torch.Tensor):
        """Copy new parameter values into the buffer the graph reads."""
        self.params.copy_(theta)

    def _evaluate(self):
        B.md_compute_forces(self.s.ctx, self.dpot, self.precision, self.F,
                            self.E if self.with_energy else None, None)
        torch.sub(self.F, self.F_star, out=self.u)
        self.u.mul_(self.scale)
        B.md_force_vjp(self.s.ctx, self.dpot, self.precision, None, self.u, self.vE, self.g_pos, self.g)

    def gradient_eager(self) -> torch.Tensor:
        """One evaluation without the graph; returns dL/dtheta (a view of the output buffer)."""
        self._evaluate()
        return self.g

    def capture(self, warmup: int = 2):
        """Capture one evaluation in a HIP graph (after eager warm-up calls that
        set the kernels' LDS attributes and size everything)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._evaluate()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._evaluate()
        torch.cuda.synchronize()

    def gradient(self) -> torch.Tensor:
        """One evaluation by graph replay (captures on first use)."""
        if self.graph is None:
            self.capture()
        self.graph.replay()
        return self.g

    def loss(self) -> float:
        """L of the last evaluation (synchronises)."""
        d = self.F - self.F_star
        return float((d * d).sum().item()) / (3.0 * self.s.n)
