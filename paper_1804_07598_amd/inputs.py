"""Seeded synthetic inputs shared by the tests, the bench and the smoke run.

This module only draws and lays out input arrays; it contains none of the
method's arithmetic (no neighbour search, no pair interaction, no time
stepping).  Both the FP64 CPU oracle and the HIP path consume its output.

Recipes (paper section 4.1 starts the LJ fluid on a regular Cartesian lattice;
section 4.2 starts SPH from a fluid column resting on boundary particles):

* LJ lattice: box side L64 = (N/rho)^(1/3) rounded once to FP32 (that FP32
  value is *the* box for everyone); n = ceil(N^(1/3)) sites per axis, spacing
  a = L32/n; site (i+1/2)*a plus a U(-jitter, +jitter) offset per coordinate,
  computed in FP64 and rounded once to FP32.  When N < n^3 a random subset of
  the n^3 sites is kept (in lattice order).  Draw order: site subset, jitter,
  velocities, types.
* Velocities: N(0, sqrt(T/m)) per component in FP64, minus the mean, rescaled
  so that 2 KE / (3N - 3) = T exactly, then rounded to FP32.
* Binary mixture: exactly N/2 particles of type 0 (A) and N - N/2 of type 1 (B)
  chosen by a random permutation.
* SPH column: a fluid lattice nf x nf x nz at spacing dx over a three-layer
  floor of boundary particles, periodic in x and y, hydrostatic density.
* SPH dam break (section 4.2's benchmark, a water column released in one
  corner of a tank onto a fixed obstacle): synthetic geometry, closed box.
* DEM grains (section 4.5): a block of grains on a Cartesian lattice of
  spacing `spacing` (below 2R: the grains start slightly overlapped) with a
  uniform jitter, Gaussian velocities and angular velocities.

All generators use numpy.random.Generator(PCG64(seed)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "LJSystem", "lj_lattice", "lj_config", "batched_table", "batched_system",
    "SPHSystem", "sph_column", "sph_dambreak", "DEMSystem", "dem_block", "dem_avalanche",
    "LJ_CONFIGS",
]


@dataclasses.dataclass
class LJSystem:
    """One periodic LJ system in the caller's (original) particle order."""
    pos: np.ndarray      # (N, 3) float32, in [0, L)
    vel: np.ndarray      # (N, 3) float32
    typ: np.ndarray      # (N,) int32, 0 = A, 1 = B
    L: float             # FP32-representable box side (cubic)
    seed: int
    rho: float
    T: float

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def box(self) -> np.ndarray:
        return np.full(3, self.L, dtype=np.float32)


def _box_side(n: int, rho: float) -> float:
    return float(np.float32((n / rho) ** (1.0 / 3.0)))


def lj_lattice(n: int, rho: float, T: float, seed: int, *, jitter: float = 0.05,
               mixture: bool = False, mass: float = 1.0) -> LJSystem:
    """Jittered simple-cubic lattice with Gaussian velocities (recipe above)."""
    if n < 2:
        raise ValueError("need at least two particles")
    rng = np.random.Generator(np.random.PCG64(seed))
    L32 = _box_side(n, rho)
    m = int(round(n ** (1.0 / 3.0)))
    if m ** 3 < n:
        m += 1
    a = L32 / m
    idx = np.indices((m, m, m)).reshape(3, -1).T  # x slowest
    if m ** 3 != n:
        keep = np.sort(rng.permutation(m ** 3)[:n])
        idx = idx[keep]
    sites = (idx.astype(np.float64) + 0.5) * a
    sites += rng.uniform(-jitter, jitter, size=sites.shape)
    pos = sites.astype(np.float32)
    # guard the half-open box (never triggers for jitter < a/2)
    pos = np.where(pos >= np.float32(L32), pos - np.float32(L32), pos)
    pos = np.where(pos < 0, pos + np.float32(L32), pos).astype(np.float32)

    v = rng.normal(0.0, math.sqrt(T / mass), size=(n, 3))
    v -= v.mean(axis=0)
    ke = 0.5 * mass * float((v * v).sum())
    v *= math.sqrt(T / (2.0 * ke / (3 * n - 3)))
    vel = v.astype(np.float32)

    typ = np.zeros(n, dtype=np.int32)
    if mixture:
        perm = rng.permutation(n)
        typ[perm[n // 2:]] = 1
    return LJSystem(pos=pos, vel=vel, typ=typ, L=L32, seed=seed, rho=rho, T=T)


# The five workloads.  Sizes follow the LJ benchmark of section 4.1 (a jittered
# lattice liquid), the SPH column of section 4.2, a batch of independent boxes
# and a binary mixture for the differentiable form.
LJ_CONFIGS = {
    "lj4096": dict(n=4096, rho=0.8442, T=1.0, seed=1),
    "lj1m": dict(n=1_000_000, rho=0.8442, T=1.0, seed=2),
    "mix32k": dict(n=32768, rho=1.2, T=1.0, seed=5, mixture=True),
}

# Pair tables in upper-triangular order (AA, AB, BB).
LJ_SINGLE = dict(eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0))
LJ_MIXTURE = dict(eps=(1.0, 1.5, 0.5), sig=(1.0, 0.8, 0.88))


def lj_config(name: str) -> LJSystem:
    return lj_lattice(**LJ_CONFIGS[name])


def batched_table(n_sys: int = 512, seed: int = 4):
    """(N_s, rho_s, T_s) for the batch of independent boxes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(256, 8193, size=n_sys).astype(np.int64)
    rhos = rng.uniform(0.6, 0.9, size=n_sys)
    Ts = rng.uniform(0.8, 1.5, size=n_sys)
    return ns, rhos, Ts


def batched_system(s: int, ns, rhos, Ts) -> LJSystem:
    return lj_lattice(int(ns[s]), float(rhos[s]), float(Ts[s]), 4000 + s)


@dataclasses.dataclass
class SPHSystem:
    pos: np.ndarray      # (N, 3) float32
    vel: np.ndarray      # (N, 3) float32
    rho: np.ndarray      # (N,) float32
    kind: np.ndarray     # (N,) int32, 0 = fluid, 1 = boundary
    L: np.ndarray        # (3,) float32 box extent; x, y periodic, z not
    dx: float
    H: float             # fluid column height


def sph_column(nf: int = 128, nz: int | None = None, dx: float = 0.01, *,
               n_floor: int = 3, headroom: int = 32, rho0: float = 1000.0,
               g: float = 9.81, gamma: float = 7.0, c0_factor: float = 20.0) -> SPHSystem:
    """Fluid column of nf x nf x nz particles on an n_floor-layer floor.

    The floor occupies z in [0, n_floor*dx); fluid particles start at
    z = n_floor*dx + (k + 1/2) dx.  Density is set hydrostatically from the
    Tait equation of state (section 4.2, Eqs. 3-4) with the sound speed
    c0 = c0_factor * sqrt(g H) and b = c0^2 rho0 / gamma, so that the initial
    pressure is rho0 g (H - z') at height z' above the floor.
    """
    nz = nf if nz is None else nz
    H = nz * dx
    c0 = c0_factor * math.sqrt(g * H)
    b = c0 * c0 * rho0 / gamma
    ii = (np.arange(nf) + 0.5) * dx
    zf = n_floor * dx + (np.arange(nz) + 0.5) * dx
    zb = (np.arange(n_floor) + 0.5) * dx
    X, Y, Z = np.meshgrid(ii, ii, zf, indexing="ij")
    fluid = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    Xb, Yb, Zb = np.meshgrid(ii, ii, zb, indexing="ij")
    bnd = np.stack([Xb.ravel(), Yb.ravel(), Zb.ravel()], axis=1)
    pos64 = np.concatenate([fluid, bnd], axis=0)
    kind = np.concatenate([np.zeros(len(fluid), np.int32), np.ones(len(bnd), np.int32)])
    depth = H - (pos64[:, 2] - n_floor * dx)
    rho = rho0 * (1.0 + rho0 * g * depth / b) ** (1.0 / gamma)
    L = np.array([nf * dx, nf * dx, (n_floor + nz + headroom) * dx], dtype=np.float32)
    return SPHSystem(pos=pos64.astype(np.float32), vel=np.zeros_like(pos64, dtype=np.float32),
                     rho=rho.astype(np.float32), kind=kind, L=L, dx=dx, H=H)


def _lattice(lo, hi, dp):
    """Sites (i + 1/2) dp of the box [lo, hi) (FP64), one per cell of side dp."""
    axes = [lo[k] + (np.arange(int(round((hi[k] - lo[k]) / dp))) + 0.5) * dp for k in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def sph_dambreak(dp: float = 0.01, *, tank=(1.6, 0.67, 0.4), column=(0.4, 0.67, 0.3),
                 obstacle=((0.9, 0.24), (0.12, 0.12), 0.45), n_wall: int = 3,
                 height: float = 1.0, rho0: float = 1000.0, g: float = 9.81,
                 gamma: float = 7.0, c0_factor: float = 20.0) -> SPHSystem:
    """Dam break in a closed tank (synthetic stand-in for section 4.2's case).

    Tank interior [0, tank) (x, y, z; open top), walled by n_wall layers of
    boundary particles at spacing dp on the floor and the four sides; a fluid
    column [0, column) in the corner at x = 0; a solid obstacle block of
    boundary particles with lower corner (x, y) = obstacle[0], footprint
    obstacle[1] and height obstacle[2] standing on the floor.  Coordinates
    are shifted by n_wall dp so that everything lies in the (closed) box
    L = tank + 2 n_wall dp in x and y and `height` + n_wall dp in z.  The
    fluid starts at rest with hydrostatic Tait density for the column height
    H = column[2], c0 = c0_factor sqrt(g H); boundary particles at rho0.
    With the defaults (dp = 0.01) N = 179,154 (80,400 fluid), near the paper's 171,496.
    """
    w = n_wall * dp
    tx, ty, tz = tank
    outer = _lattice((-w, -w, -w), (tx + w, ty + w, tz), dp)
    inner = ((outer[:, 0] > 0) & (outer[:, 0] < tx) & (outer[:, 1] > 0) & (outer[:, 1] < ty)
             & (outer[:, 2] > 0))
    walls = outer[~inner]
    (ox, oy), (fx, fy), oh = obstacle
    block = _lattice((ox, oy, 0.0), (ox + fx, oy + fy, oh), dp)
    fluid = _lattice((0.0, 0.0, 0.0), column, dp)
    H = float(column[2])
    c0 = c0_factor * math.sqrt(g * H)
    b = c0 * c0 * rho0 / gamma
    rho_f = rho0 * (1.0 + rho0 * g * (H - fluid[:, 2]) / b) ** (1.0 / gamma)
    pos64 = np.concatenate([fluid, walls, block], axis=0) + w
    kind = np.concatenate([np.zeros(len(fluid), np.int32),
                           np.ones(len(walls) + len(block), np.int32)])
    rho = np.concatenate([rho_f, np.full(len(walls) + len(block), rho0)])
    L = np.array([tx + 2 * w, ty + 2 * w, height + w], dtype=np.float32)
    return SPHSystem(pos=pos64.astype(np.float32), vel=np.zeros_like(pos64, dtype=np.float32),
                     rho=rho.astype(np.float32), kind=kind, L=L, dx=dp, H=H)


@dataclasses.dataclass
class DEMSystem:
    pos: np.ndarray      # (N, 3) float32
    vel: np.ndarray      # (N, 3) float32
    omega: np.ndarray    # (N, 3) float32
    L: np.ndarray        # (3,) float32 box
    periodic: tuple
    R: float


def dem_block(shape, R: float, spacing: float, L, periodic=(1, 1, 1), origin=(0.0, 0.0, 0.0),
              seed: int = 0, jitter: float = 0.0, vel_sigma: float = 0.0,
              omega_sigma: float = 0.0) -> DEMSystem:
    """Grains at origin + (i + 1/2) spacing on a shape[0] x shape[1] x shape[2]
    lattice, each coordinate plus U(-jitter, jitter) (FP64, rounded once);
    velocities N(0, vel_sigma) and angular velocities N(0, omega_sigma) per
    component.  Draw order: jitter, velocities, angular velocities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.indices(shape).reshape(3, -1).T.astype(np.float64)
    pos = np.asarray(origin, np.float64) + (idx + 0.5) * spacing
    n = len(pos)
    pos = pos + rng.uniform(-jitter, jitter, (n, 3))
    vel = rng.normal(0.0, vel_sigma, (n, 3)) if vel_sigma > 0 else np.zeros((n, 3))
    om = rng.normal(0.0, omega_sigma, (n, 3)) if omega_sigma > 0 else np.zeros((n, 3))
    return DEMSystem(pos=pos.astype(np.float32), vel=vel.astype(np.float32),
                     omega=om.astype(np.float32), L=np.asarray(L, np.float32),
                     periodic=tuple(int(p) for p in periodic), R=float(R))


# Grain constants of the avalanche in section 4.5 (R, m, I, k_n, k_t, gamma_n as
# printed).  The paper states neither gamma_t, mu, |g| nor the time step; the
# values here are this workload's choices: |g| = 5e-4 keeps the Hertz overlap
# under the deepest column of the 688k-grain block below 10 % of a diameter
# (k_n = 7.849 is soft for m = 1), and dt = 0.01 resolves the stiffest contact
# period (about 2 time units) in some 200 steps.
DEM_AVALANCHE = dict(R=0.06, mass=1.0, inertia=1.44e-3, kn=7.849, kt=2.243, gn=3.401, gt=1.0,
                     mu=0.5, g_abs=5e-4, tilt_deg=30.0, dt=0.01, walls=3)


def dem_avalanche_gravity(g_abs: float = DEM_AVALANCHE["g_abs"],
                          tilt_deg: float = DEM_AVALANCHE["tilt_deg"]):
    """Gravity rotated by the plane's inclination: down the slope along +x."""
    t = np.radians(tilt_deg)
    return (float(g_abs * np.sin(t)), 0.0, float(-g_abs * np.cos(t)))


def dem_avalanche(scale: float = 1.0, R: float = 0.06, seed: int = 11) -> DEMSystem:
    """The grain avalanche of section 4.5 (synthetic stand-in): a domain of
    8.4 x 3.0 x 3.18 times `scale` with walls in x, periodic in y and open in
    +z above a floor; the grains start as a lattice block of 4.26 x 3.06 x
    1.26 times `scale` (capped to the domain's y extent) at spacing 2R in the
    corner at x = 0, at rest.  Gravity is tilted by 30 degrees by the caller."""
    Ld = np.array([8.4, 3.0, 3.18]) * scale
    blk = np.array([4.26, min(3.06, 3.0), 1.26]) * scale
    shape = tuple(int(v) for v in np.floor(blk / (2 * R)))
    return dem_block(shape, R, 2 * R, Ld, (0, 1, 0), origin=(0.0, 0.0, 0.0), seed=seed,
                     jitter=0.01 * R)
