"""Sequencing of the four stage calls for one transport problem on the GPU.

Control flow only: every numerical step runs in libmlpg.so.  Host arrays
are moved to the device once; the solve loop works on resident tensors.
Device memory is torch's: each stage gets a workspace tensor of exactly the
size its *_workspace_bytes query returns, kept alive as long as the handle
uses it.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mlpg as api


class GpuProblem:
    def __init__(self, x: np.ndarray, R: np.ndarray, dom_lo, dom_hi, regions=(), fields=(), shells=()):
        self.dim = x.shape[1]
        self.dom_lo, self.dom_hi = tuple(dom_lo), tuple(dom_hi)
        self.x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
        self.R = torch.from_numpy(np.ascontiguousarray(R, dtype=np.float64)).cuda()
        self.nbr_off, total = api.mlpg_neighbors_count(self.x, self.R)
        self.nbr_idx = api.mlpg_neighbors_fill(self.x, self.R, self.nbr_off, total)
        self.ws = {}
        self.ws["geometry"] = api.workspace(api.mlpg_geometry_workspace_bytes(
            self.dim, x.shape[0], total, self.dom_lo, self.dom_hi))
        self.h = api.mlpg_geometry(self.x, self.R, self.nbr_off, self.nbr_idx, dom_lo, dom_hi, regions,
                                   ws=self.ws["geometry"])
        if fields:
            api.mlpg_material_fields(self.h, fields)
        if shells:
            api.mlpg_material_shells(self.h, shells)
        self.info = api.mlpg_get_info(self.h)
        self.n = self.info["n"]
        self.M = 0
        self.precision = api.MLPG_FP64

    def device_bytes(self, opts=None) -> int:
        """Exact device bytes of the problem once assembled: its inputs on the device (positions, radii,
        overlap lists) and the four stage workspaces (the solve's for ``opts``, whether held yet or not)."""
        inputs = sum(t.numel() * t.element_size() for t in (self.x, self.R, self.nbr_off, self.nbr_idx))
        held = sum(v.numel() for k, v in self.ws.items() if k != "solve")
        return inputs + held + api.mlpg_solve_workspace_bytes(self.h, opts)

    def workspace_bytes(self) -> dict:
        """Bytes of every stage workspace held now (the device memory the problem uses beyond its inputs)."""
        return {k: v.numel() for k, v in self.ws.items()}

    def move(self, x: np.ndarray, R: np.ndarray):
        """New point positions and radii (same count): neighbour lists and cells
        are rebuilt; integrate and assemble again before the next step."""
        self.x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
        self.R = torch.from_numpy(np.ascontiguousarray(R, dtype=np.float64)).cuda()
        self.nbr_off, total = api.mlpg_neighbors_count(self.x, self.R)
        self.nbr_idx = api.mlpg_neighbors_fill(self.x, self.R, self.nbr_off, total)
        need = api.mlpg_geometry_workspace_bytes(self.dim, self.n, total, self.dom_lo, self.dom_hi)
        if self.ws["geometry"].numel() < need:
            self.ws["geometry"] = api.workspace(need)
        api.mlpg_update_points(self.h, self.x, self.R, self.nbr_off, self.nbr_idx, ws=self.ws["geometry"])
        return self.refresh()

    def refresh(self):
        self.info = api.mlpg_get_info(self.h)
        return self.info

    def _grow(self, name, need):
        cur = self.ws.get(name)
        if cur is None or cur.numel() < need:
            self.ws[name] = api.workspace(need)
        return self.ws[name]

    def integrate(self, rk_order: int):
        ws = self._grow("integrate", api.mlpg_integrate_workspace_bytes(self.h, rk_order))
        api.mlpg_integrate(self.h, rk_order, ws=ws)
        return self.refresh()

    def boundary_points(self):
        return api.mlpg_boundary_points(self.h, self.info["n_bq"], self.dim)

    def assemble(self, omega, w, sigma_t, sigma_s, inv_c_dt, tau, precision=api.MLPG_FP64):
        if np.isscalar(tau):
            tau = torch.full((self.n,), float(tau), dtype=torch.float64, device="cuda")
        need = api.mlpg_assemble_workspace_bytes(self.h, omega.shape[0], precision)
        old = self.ws.get("assemble")
        if old is not None and old.numel() >= need:
            ws = old   # same workspace: the state stays in place
        else:
            ws = api.workspace(need)   # the library copies the state over from `old`
        api.mlpg_assemble(self.h, omega, w, sigma_t, sigma_s, inv_c_dt, tau, precision, ws=ws)
        self.ws["assemble"] = ws
        self.M = omega.shape[0]
        self.precision = precision
        return self.refresh()

    def set_state(self, psi):
        api.mlpg_set_state(self.h, psi)

    def solve_workspace(self, opts=None):
        return self._grow("solve", api.mlpg_solve_workspace_bytes(self.h, opts))

    def step(self, q, psi_b=None, opts=None, want_psi=True):
        return api.mlpg_solve(self.h, q, psi_b, opts, want_psi, ws=self.solve_workspace(opts))

    def close(self):
        if self.h is not None:
            api.mlpg_destroy(self.h)
            self.h = None
        self.ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
