"""Thin Python owners of a library context: device memory comes from PyTorch,
every computation runs in libfpm.so kernels.

`ParticleSim` mirrors the objects of the paper's MD listing (section 4.1): a
box with boundary conditions, an interaction radius, a particle set with
velocity and force properties, neighbour lists and a velocity-Verlet loop.
`BatchSim` runs many independent systems of uneven size through the same
kernels, one launch per step for the whole batch.
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


def _as(t, dtype, device):
    return None if t is None else torch.as_tensor(t, dtype=dtype, device=device).contiguous()


class _Sim:
    """Context, workspace and the calls shared by single systems and batches."""

    def _open(self, pos, vel, typ, r_cut, skin, max_nbr, device, set_boxes, tuning,
              dem_contacts=0, symmetric=False):
        self.device = torch.device(device)
        self.pos0 = _as(pos, torch.float32, self.device)
        self.n = int(self.pos0.shape[0])
        self.r_cut, self.skin, self.max_nbr = float(r_cut), float(skin), int(max_nbr)
        self._vel = _as(vel, torch.float32, self.device)
        self._typ = _as(typ, torch.int32, self.device)
        self.ctx = F.fpm_create(_stream_handle())
        set_boxes()
        F.fpm_set_neighbor_params(self.ctx, self.r_cut, self.skin, self.max_nbr)
        self.dem_contacts = int(dem_contacts)
        if self.dem_contacts:
            F.fpm_set_dem(self.ctx, self.dem_contacts)
        self.symmetric = bool(symmetric)
        if self.symmetric:
            F.fpm_set_symmetric(self.ctx, True)
        if tuning is not None:
            F.fpm_set_tuning(self.ctx, *tuning)
        self._load(self.pos0, self._vel)

    def _load(self, pos, vel):
        nbytes = F.fpm_workspace_size(self.ctx, self.n)
        if getattr(self, "ws", None) is None or self.ws.numel() < nbytes:
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-ws.data_ptr()) % 256
            self.ws = ws[off:off + nbytes]
            F.fpm_set_workspace(self.ctx, self.ws)
        F.fpm_set_particles(self.ctx, pos, vel, self._typ)

    def set_tuning(self, verlet_path: int = 0, zblock: int = 0, unroll: int = 0):
        """Launch shapes (see fpm_set_tuning); reloads the current state."""
        p, v, _ = self.get()
        F.fpm_set_tuning(self.ctx, verlet_path, zblock, unroll)
        self._load(p, v)

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

    def set_particles(self, pos, vel=None):
        """Replace the state (same count, types and boxes); rebuilds all structures."""
        p = _as(pos, torch.float32, self.device)
        v = _as(vel, torch.float32, self.device)
        F.fpm_set_particles(self.ctx, p, v, self._typ)
        self._keep_state = (p, v)

    def set_positions(self, pos):
        """New positions for the current particles (lists rebuilt only if needed)."""
        p = _as(pos, torch.float32, self.device)
        F.fpm_set_positions(self.ctx, p)
        self._keep_pos = p

    # ---- neighbour structures ----
    def build_cell_list(self):
        F.fpm_build_cell_list(self.ctx)

    def build_verlet(self):
        F.fpm_build_verlet(self.ctx)

    def neighbors(self):
        """(counts (n,), cols (n, max_nbr)) in caller indices, rows unordered."""
        counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        cols = torch.full((self.n, self.max_nbr), -1, dtype=torch.int32, device=self.device)
        F.fpm_get_neighbors(self.ctx, counts, cols)
        return counts, cols

    # ---- LJ ----
    def _lj_out(self):
        return torch.zeros((self.nsys, 8), dtype=torch.float64, device=self.device)

    def lj_forces(self, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), n_types: int = 1):
        """Forces (kept in the context) and FP64 [U, 0, W6] per system on the device."""
        out = self._lj_out()
        F.fpm_lj_forces(self.ctx, F.lj_params(eps, sig, n_types), out)
        return out[0] if self.nsys == 1 else out

    def force_vjp(self, lam, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), n_types: int = 1):
        """(dL/dx (n, 3) FP64, dL/dtheta (nsys, 6) FP64) for lam = dL/dF (n, 3)."""
        lam = _as(lam, torch.float64, self.device)
        gx = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        gt = torch.zeros((self.nsys, 6), dtype=torch.float64, device=self.device)
        F.fpm_lj_force_vjp(self.ctx, F.lj_params(eps, sig, n_types), lam, gx, gt)
        return gx, gt

    def adjoint_step(self, dt, floss, xbar, vbar, fbar, gtheta, eps=(1.0, 1.0, 1.0),
                     sig=(1.0, 1.0, 1.0), n_types: int = 1, last: bool = False):
        """One reverse velocity-Verlet step (see fpm_lj_adjoint_step), in place."""
        F.fpm_lj_adjoint_step(self.ctx, F.lj_params(eps, sig, n_types), dt, floss, xbar, vbar,
                              fbar, gtheta, 1 if last else 0)

    def integrate(self, dt: float, half: int):
        F.fpm_integrate(self.ctx, dt, half)

    def step(self, nsteps: int, dt: float = 0.005, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0),
             n_types: int = 1, thermo: torch.Tensor | None = None):
        """nsteps velocity-Verlet steps; returns the FP64 thermo rows
        {U, KE, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz}: (nsteps, 8) for one system,
        (nsteps, nsys, 8) for a batch (or writes into `thermo`)."""
        if thermo is None:
            thermo = torch.zeros((max(nsteps, 1), self.nsys, 8), dtype=torch.float64,
                                 device=self.device)
            if self.nsys == 1:
                thermo = thermo[:, 0]
        F.fpm_step(self.ctx, F.lj_params(eps, sig, n_types), dt, nsteps, thermo)
        return thermo

    # ---- status ----
    def check(self):
        F.fpm_check(self.ctx)

    def counters(self):
        """(rebuilds, longest list of the last build, total list entries of the last build)."""
        return F.fpm_read_counters(self.ctx)


class ParticleSim(_Sim):
    """One particle system on one device."""

    def __init__(self, pos, L, periodic=(1, 1, 1), *, vel=None, typ=None, r_cut: float = 2.5,
                 skin: float = 0.3, max_nbr: int | None = None, device="cuda", tuning=None,
                 dem_contacts: int = 0, symmetric: bool = False):
        self.L = [float(x) for x in (L if hasattr(L, "__len__") else (L, L, L))]
        self.periodic = tuple(int(p) for p in periodic)
        self.nsys = 1
        n = len(pos)
        if max_nbr is None:
            max_nbr = default_max_nbr(n, self.L[0] * self.L[1] * self.L[2], r_cut + skin)
        self._open(pos, vel, typ, r_cut, skin, max_nbr, device,
                   lambda: F.fpm_set_box(self.ctx, self.L, self.periodic), tuning, dem_contacts,
                   symmetric)

    def cell_list(self):
        """(ncell, offsets, order): grid, exclusive scan of counts, slot -> caller index."""
        ncell = F.fpm_get_cell_list(self.ctx)
        ncells = ncell[0] * ncell[1] * ncell[2]
        off = torch.empty(ncells + 1, dtype=torch.int32, device=self.device)
        order = torch.empty(self.n, dtype=torch.int32, device=self.device)
        F.fpm_get_cell_list(self.ctx, off, order)
        return ncell, off, order

    # ---- SPH ----
    def set_density(self, rho):
        r = _as(rho, torch.float32, self.device)
        F.fpm_set_density(self.ctx, r)
        self._rho = r

    def sph_rates(self, prm):
        """Rates of Eqs. 1-2 at the current state; returns the CFL dt (device, FP32)."""
        dt = torch.zeros(1, dtype=torch.float32, device=self.device)
        F.fpm_sph_rates(self.ctx, prm, dt)
        return dt

    def sph_step(self, nsteps: int, prm, hist: torch.Tensor | None = None):
        """nsteps steps of prm's scheme (kick-drift-kick or Verlet); returns the
        (nsteps, 4) FP64 history {t, dt, KE, max|v|}."""
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


    # ---- DEM (dem_contacts > 0) ----
    def set_omega(self, omega=None):
        F.fpm_set_omega(self.ctx, None if omega is None else _as(omega, torch.float32, self.device))

    def dem_forces(self, prm):
        """Forces and torques of the grain model, advancing the contact history."""
        F.fpm_dem_forces(self.ctx, prm)

    def dem_step(self, nsteps: int, prm):
        F.fpm_dem_step(self.ctx, prm, nsteps)

    def get_dem(self):
        """(omega (n, 3), torque (n, 3), contact counts (n,)) in caller order."""
        w = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        t = torch.empty_like(w)
        nc = torch.empty(self.n, dtype=torch.int32, device=self.device)
        F.fpm_get_dem(self.ctx, w, t, nc)
        return w, t, nc

    def contacts(self):
        """(ids (n, C), u_t (n, C, 3)): partners by caller index (-1 empty)."""
        C_ = self.dem_contacts
        ids = torch.empty((self.n, C_), dtype=torch.int32, device=self.device)
        ut = torch.empty((self.n, C_, 3), dtype=torch.float32, device=self.device)
        F.fpm_get_contacts(self.ctx, ids, ut)
        return ids, ut


class BatchSim(_Sim):
    """Independent periodic systems of uneven size, stepped together.

    `systems` is a list of (pos (n_s, 3), L (3,) or scalar) with optional
    per-system velocities and types; caller-order arrays concatenate the
    systems in list order."""

    def __init__(self, pos_list, L_list, periodic=(1, 1, 1), *, vel_list=None, typ_list=None,
                 r_cut: float = 2.5, skin: float = 0.3, max_nbr: int | None = None,
                 device="cuda", tuning=None, symmetric: bool = False):
        self.nsys = len(pos_list)
        self.counts = [len(p) for p in pos_list]
        self.L = [[float(x) for x in (L if hasattr(L, "__len__") else (L, L, L))]
                  for L in L_list]
        self.periodic = [tuple(int(p) for p in periodic)] * self.nsys
        self.offsets = [0]
        for c in self.counts:
            self.offsets.append(self.offsets[-1] + c)
        pos = torch.cat([torch.as_tensor(p, dtype=torch.float32) for p in pos_list])
        vel = None if vel_list is None else torch.cat(
            [torch.as_tensor(v, dtype=torch.float32) for v in vel_list])
        typ = None if typ_list is None else torch.cat(
            [torch.as_tensor(t, dtype=torch.int32) for t in typ_list])
        if max_nbr is None:
            max_nbr = max(default_max_nbr(c, L[0] * L[1] * L[2], r_cut + skin)
                          for c, L in zip(self.counts, self.L))
        self._open(pos, vel, typ, r_cut, skin, max_nbr, device,
                   lambda: F.fpm_set_systems(self.ctx, self.L, self.periodic, self.counts),
                   tuning, 0, symmetric)

    def system_info(self, s: int):
        """{n, first caller index, cells, first offsets entry, nc_x, nc_y, nc_z, zblock}."""
        keys = ("n", "caller_base", "ncells", "off_base", "ncx", "ncy", "ncz", "zblock")
        return dict(zip(keys, F.fpm_system_info(self.ctx, s)))

    def cell_list(self):
        """(offsets, order): per-system cell offsets concatenated (system s owns
        entries off_base .. off_base + ncells, in the packed caller numbering)
        and the slot -> caller index order of the whole batch."""
        total = sum(self.system_info(s)["ncells"] + 1 for s in range(self.nsys))
        off = torch.empty(total, dtype=torch.int32, device=self.device)
        order = torch.empty(self.n, dtype=torch.int32, device=self.device)
        F.fpm_get_cell_list(self.ctx, off, order)
        return off, order

    def split(self, t):
        """Split a caller-order tensor into per-system pieces."""
        return [t[self.offsets[s]:self.offsets[s + 1]] for s in range(self.nsys)]
