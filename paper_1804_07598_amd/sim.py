"""Thin Python owners of a library context: device memory comes from PyTorch,
every computation runs in libfpm.so kernels.

`ParticleSim` mirrors the objects of the paper's MD listing (section 4.1): a
box with boundary conditions, an interaction radius, a particle set with
velocity and force properties, neighbour lists and a velocity-Verlet loop.
"""
from __future__ import annotations

import math

import torch

from . import _lib as F


def _stream_handle() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def default_max_nbr(n: int, volume: float, r_list: float) -> int:
    """List capacity: 1.6x the ideal-gas neighbour count plus slack, multiple of 8."""
    mean = 4.0 / 3.0 * math.pi * r_list ** 3 * n / volume
    return int(min(4096, max(32, math.ceil((1.6 * mean + 48) / 8) * 8)))


class ParticleSim:
    """One particle system on one device."""

    def __init__(self, pos, L, periodic=(1, 1, 1), *, vel=None, typ=None, r_cut: float = 2.5,
                 skin: float = 0.3, max_nbr: int | None = None, device="cuda"):
        self.device = torch.device(device)
        self.pos0 = torch.as_tensor(pos, dtype=torch.float32, device=self.device).contiguous()
        self.n = int(self.pos0.shape[0])
        self.L = [float(x) for x in (L if hasattr(L, "__len__") else (L, L, L))]
        self.periodic = tuple(int(p) for p in periodic)
        vel_t = None if vel is None else torch.as_tensor(vel, dtype=torch.float32,
                                                         device=self.device).contiguous()
        typ_t = None if typ is None else torch.as_tensor(typ, dtype=torch.int32,
                                                         device=self.device).contiguous()
        if max_nbr is None:
            max_nbr = default_max_nbr(self.n, self.L[0] * self.L[1] * self.L[2], r_cut + skin)
        self.r_cut, self.skin, self.max_nbr = float(r_cut), float(skin), int(max_nbr)
        self.ctx = F.fpm_create(_stream_handle())
        F.fpm_set_box(self.ctx, self.L, self.periodic)
        F.fpm_set_neighbor_params(self.ctx, self.r_cut, self.skin, self.max_nbr)
        nbytes = F.fpm_workspace_size(self.ctx, self.n)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws = self.ws[off:off + nbytes]
        F.fpm_set_workspace(self.ctx, self.ws)
        F.fpm_set_particles(self.ctx, self.pos0, vel_t, typ_t)
        self._keep = (vel_t, typ_t)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            F.fpm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state ----
    def get(self):
        """(pos, vel, frc) in caller order as (n, 3) float32 device tensors."""
        p = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        v = torch.empty_like(p)
        f = torch.empty_like(p)
        F.fpm_get_particles(self.ctx, p, v, f)
        return p, v, f

    # ---- neighbour structures ----
    def build_cell_list(self):
        F.fpm_build_cell_list(self.ctx)

    def cell_list(self):
        """(ncell, offsets, order): grid, exclusive scan of counts, slot -> caller index."""
        ncell = F.fpm_get_cell_list(self.ctx)
        ncells = ncell[0] * ncell[1] * ncell[2]
        off = torch.empty(ncells + 1, dtype=torch.int32, device=self.device)
        order = torch.empty(self.n, dtype=torch.int32, device=self.device)
        F.fpm_get_cell_list(self.ctx, off, order)
        return ncell, off, order

    def build_verlet(self):
        F.fpm_build_verlet(self.ctx)

    def neighbors(self):
        """(counts (n,), cols (n, max_nbr)) in caller indices, rows unordered."""
        counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        cols = torch.full((self.n, self.max_nbr), -1, dtype=torch.int32, device=self.device)
        F.fpm_get_neighbors(self.ctx, counts, cols)
        return counts, cols

    # ---- LJ ----
    def lj_forces(self, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), n_types: int = 1):
        """Forces (kept in the context) and FP64 [U, 0, W6] on the device."""
        out = torch.zeros(8, dtype=torch.float64, device=self.device)
        F.fpm_lj_forces(self.ctx, F.lj_params(eps, sig, n_types), out)
        return out

    def integrate(self, dt: float, half: int):
        F.fpm_integrate(self.ctx, dt, half)

    def step(self, nsteps: int, dt: float = 0.005, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0),
             n_types: int = 1, thermo: torch.Tensor | None = None):
        """nsteps velocity-Verlet steps; returns the (nsteps, 8) FP64 thermo tensor
        {U, KE, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz} (or writes into `thermo`)."""
        if thermo is None:
            thermo = torch.zeros((max(nsteps, 1), 8), dtype=torch.float64, device=self.device)
        F.fpm_step(self.ctx, F.lj_params(eps, sig, n_types), dt, nsteps, thermo)
        return thermo

    # ---- SPH ----
    def set_density(self, rho):
        r = torch.as_tensor(rho, dtype=torch.float32, device=self.device).contiguous()
        F.fpm_set_density(self.ctx, r)
        self._rho = r

    def sph_rates(self, prm):
        """Rates of Eqs. 1-2 at the current state; returns the CFL dt (device, FP32)."""
        dt = torch.zeros(1, dtype=torch.float32, device=self.device)
        F.fpm_sph_rates(self.ctx, prm, dt)
        return dt

    def sph_step(self, nsteps: int, prm, hist: torch.Tensor | None = None):
        """nsteps KDK steps; returns the (nsteps, 4) FP64 history {t, dt, KE, max|v|}."""
        if hist is None:
            hist = torch.zeros((max(nsteps, 1), 4), dtype=torch.float64, device=self.device)
        F.fpm_sph_step(self.ctx, prm, nsteps, hist)
        return hist

    def get_sph(self):
        """(rho, drho/dt) in caller order."""
        rho = torch.empty(self.n, dtype=torch.float32, device=self.device)
        dr = torch.empty_like(rho)
        F.fpm_get_sph(self.ctx, rho, dr)
        return rho, dr

    # ---- status ----
    def check(self):
        F.fpm_check(self.ctx)

    def counters(self):
        """(rebuilds, longest list of the last build, total list entries of the last build)."""
        return F.fpm_read_counters(self.ctx)
