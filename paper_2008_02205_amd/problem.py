"""Sequencing of the four stage calls for one transport problem on the GPU.

Control flow only: every numerical step runs in libmlpg.so.  Host arrays
are moved to the device once; the solve loop works on resident tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mlpg as api


class GpuProblem:
    def __init__(self, x: np.ndarray, R: np.ndarray, dom_lo, dom_hi, regions=(), fields=(), shells=()):
        self.dim = x.shape[1]
        self.x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
        self.R = torch.from_numpy(np.ascontiguousarray(R, dtype=np.float64)).cuda()
        self.nbr_off, total = api.mlpg_neighbors_count(self.x, self.R)
        self.nbr_idx = api.mlpg_neighbors_fill(self.x, self.R, self.nbr_off, total)
        self.h = api.mlpg_geometry(self.x, self.R, self.nbr_off, self.nbr_idx, dom_lo, dom_hi, regions)
        if fields:
            api.mlpg_material_fields(self.h, fields)
        if shells:
            api.mlpg_material_shells(self.h, shells)
        self.info = api.mlpg_get_info(self.h)
        self.n = self.info["n"]
        self.M = 0

    def move(self, x: np.ndarray, R: np.ndarray):
        """New point positions and radii (same count): neighbour lists and cells
        are rebuilt; integrate and assemble again before the next step."""
        self.x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
        self.R = torch.from_numpy(np.ascontiguousarray(R, dtype=np.float64)).cuda()
        self.nbr_off, total = api.mlpg_neighbors_count(self.x, self.R)
        self.nbr_idx = api.mlpg_neighbors_fill(self.x, self.R, self.nbr_off, total)
        api.mlpg_update_points(self.h, self.x, self.R, self.nbr_off, self.nbr_idx)
        return self.refresh()

    def refresh(self):
        self.info = api.mlpg_get_info(self.h)
        return self.info

    def integrate(self, rk_order: int):
        api.mlpg_integrate(self.h, rk_order)
        return self.refresh()

    def boundary_points(self):
        return api.mlpg_boundary_points(self.h, self.info["n_bq"], self.dim)

    def assemble(self, omega, w, sigma_t, sigma_s, inv_c_dt, tau, precision=api.MLPG_FP64):
        if np.isscalar(tau):
            tau = torch.full((self.n,), float(tau), dtype=torch.float64, device="cuda")
        api.mlpg_assemble(self.h, omega, w, sigma_t, sigma_s, inv_c_dt, tau, precision)
        self.M = omega.shape[0]
        return self.refresh()

    def set_state(self, psi):
        api.mlpg_set_state(self.h, psi)

    def step(self, q, psi_b=None, opts=None, want_psi=True):
        return api.mlpg_solve(self.h, q, psi_b, opts, want_psi)

    def close(self):
        if self.h is not None:
            api.mlpg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
