"""Device-resident problem: mesh + layout + X/Y/S buffers on one GPU.

Glue for callers (benchmark, tests, serving loop): plans the mesh and the
BCSR layout through the C ABI, uploads the potential, packs the orbital
values into BCSR order and keeps every device buffer alive.
"""

from __future__ import annotations

from typing import Callable, Optional, Sequence

import numpy as np

from .api import (DOT_WORK_DOUBLES, FP64, OP_H, OP_M, Layout, Mesh, apply_H, apply_H_tuned,
                  apply_op, energy, energy_work_bytes, mmult, mv_axpy, mv_dot, mv_update, tmmult,
                  tmmult_tuned)


class DeviceProblem:
    def __init__(self, cells: Sequence[int], L: Sequence[float], degree: int, dirichlet: int,
                 centres: np.ndarray, radius, colblock_sizes, potential: Callable[[np.ndarray], np.ndarray],
                 device: str = "cuda", stream=None,
                 node_map: Optional[Callable[[np.ndarray], np.ndarray]] = None):
        """node_map: curved cells, the box's node positions -> the mesh's."""
        import torch
        self.device = device
        self.mesh = Mesh(cells[0], cells[1], cells[2], L, degree, dirichlet)
        if node_map is not None:
            self.mesh.set_nodes(node_map(self.mesh.node_points()))
        qp = self.mesh.qp_points()
        self.mesh.set_potential(np.asarray(potential(qp.reshape(-1, 3)), dtype=np.float64))
        self.layout = Layout(self.mesh, centres, radius, colblock_sizes)
        self.mesh.bind(device, stream)
        self.layout.bind(device, stream)
        self.M = self.layout.M
        self.nvalues = self.layout.nvalues
        self.X = self.layout.new_values(device)
        self.Y = self.layout.new_values(device)
        self.work = self.layout.new_work(device)
        self.S = torch.zeros((self.M, self.M), dtype=torch.float64, device=device)
        self.trace = torch.zeros(1, dtype=torch.float64, device=device)

    def set_X_coo(self, node, orb, val) -> None:
        import torch
        host = self.layout.pack(node, orb, val)
        self.X.copy_(torch.from_numpy(host).to(self.device))

    def set_X_values(self, values: np.ndarray) -> None:
        import torch
        self.X.copy_(torch.from_numpy(np.ascontiguousarray(values, dtype=np.float64)).to(self.device))

    def apply(self, prec: int = FP64, stream=None, X=None, Y=None) -> None:
        apply_H(self.mesh, self.layout, self.X if X is None else X, self.Y if Y is None else Y,
                prec, stream)

    def apply_tuned(self, prec: int = FP64, kernel: int = 1, grid: int = 0, stream=None,
                    X=None, Y=None) -> None:
        apply_H_tuned(self.mesh, self.layout, self.X if X is None else X,
                      self.Y if Y is None else Y, self.work, prec, kernel, grid, stream)

    def overlap(self, stream=None, X=None, Y=None) -> None:
        tmmult(self.layout, self.X if X is None else X, self.Y if Y is None else Y, self.S,
               self.trace, self.work, stream)

    def overlap_tuned(self, unit_steps: int = 0, long_steps: int = 0, stream=None) -> None:
        tmmult_tuned(self.layout, self.X, self.Y, self.S, self.trace, self.work, unit_steps,
                     long_steps, stream)

    def overlap_into(self, S, trace, X=None, Y=None, stream=None) -> None:
        tmmult(self.layout, self.X if X is None else X, self.Y if Y is None else Y, S, trace,
               self.work, stream)

    def update(self, S, S2, tau: float, stream=None) -> None:
        mv_update(self.layout, self.X, self.Y, S, S2, tau, stream)

    def enable_closure(self) -> None:
        """Closure layout and its buffers: H X and M X kept entirely, the
        projected matrices Hbar = X^T H X, Mbar = X^T M X and the energy."""
        import torch
        if getattr(self, "closure", None) is not None:
            return
        self.closure = self.layout.closure()
        self.closure.bind(self.device)
        self.YH = self.closure.new_values(self.device)
        self.YM = self.closure.new_values(self.device)
        self.work_c = self.closure.new_work(self.device)
        self.Hbar = torch.zeros((self.M, self.M), dtype=torch.float64, device=self.device)
        self.Mbar = torch.zeros_like(self.Hbar)
        self.tr_c = torch.zeros(2, dtype=torch.float64, device=self.device)
        self.E = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.work_e = torch.zeros(energy_work_bytes(self.M) // 8, dtype=torch.float64,
                                  device=self.device)

    def energy(self, prec: int = FP64, stream=None) -> None:
        """E(X) of eq. energy: H X and M X onto the closure, the two
        projected matrices, then E = tr((2 I - Mbar) Hbar); all on the GPU."""
        self.enable_closure()
        c = self.closure
        apply_op(self.mesh, self.layout, c, OP_H, self.X, self.YH, prec, stream)
        apply_op(self.mesh, self.layout, c, OP_M, self.X, self.YM, prec, stream)
        tmmult(c, self.X, self.YH, self.Hbar, self.tr_c[0:1], self.work_c, stream)
        tmmult(c, self.X, self.YM, self.Mbar, self.tr_c[1:2], self.work_c, stream)
        energy(self.M, self.Mbar, self.Hbar, self.E, self.work_e, stream)

    def gradient(self, prec: int = FP64, stream=None) -> None:
        """Energy, then the gradient of eq. gradient on the pattern of X into
        self.G: -2 (M X) Hbar + (H X)(4 I - 2 Mbar), two Alg. 7 products from
        the closure onto X's pattern."""
        import torch
        self.energy(prec, stream)
        if getattr(self, "G", None) is None:
            self.G = self.layout.new_values(self.device)
            self.dots = torch.zeros(2, dtype=torch.float64, device=self.device)
            self.work_d = torch.zeros(DOT_WORK_DOUBLES, dtype=torch.float64, device=self.device)
        c = self.closure
        mmult(c, self.layout, self.YM, self.Hbar, -2.0, 0.0, self.G, False, stream)
        mmult(c, self.layout, self.YH, self.Mbar, -2.0, 4.0, self.G, True, stream)

    def descent_step(self, tau: float, prec: int = FP64, stream=None) -> None:
        """One steepest-descent step of the orbital minimisation: E and G at X,
        dots[0] = tr(G^T G) (minus the directional derivative along -G), then
        X <- X - tau G on X's pattern."""
        self.gradient(prec, stream)
        mv_dot(self.layout, self.G, self.G, self.dots[0:1], self.work_d, stream)
        mv_axpy(self.layout, -float(tau), self.G, self.X, stream)

    def original_order(self, S) -> np.ndarray:
        """An M x M device matrix in library column order, permuted back."""
        S = S.cpu().numpy()
        perm = self.layout.pattern()["col_perm"]
        out = np.empty_like(S)
        out[np.ix_(perm, perm)] = S
        return out

    def S_original_order(self) -> np.ndarray:
        """S permuted back to original orbital ids."""
        S = self.S.cpu().numpy()
        perm = self.layout.pattern()["col_perm"]
        out = np.empty_like(S)
        out[np.ix_(perm, perm)] = S
        return out

    def device_bytes(self) -> int:
        return (3 * 8 * self.nvalues + self.mesh.meta_bytes + self.layout.meta_bytes
                + self.layout.work_bytes + 8 * self.M * self.M)
