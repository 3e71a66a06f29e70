"""The workload recipes against the constants the paper prints (fixtures in
tests/golden, each citing its section), and two closed forms those printed
grain constants satisfy."""
import math
import os

import numpy as np
import pytest

from paper_1804_07598_amd import inputs

HERE = os.path.join(os.path.dirname(__file__), "golden")


def fixture(name):
    out = {}
    for line in open(os.path.join(HERE, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        out[k] = [float(x) for x in v] if len(v) > 1 else float(v[0])
    return out


def test_dem_recipe_uses_the_printed_constants():
    g = fixture("dem_avalanche_constants.txt")
    A = inputs.DEM_AVALANCHE
    for k, key in (("R", "R"), ("mass", "mass"), ("inertia", "inertia"), ("kn", "kn"),
                   ("kt", "kt"), ("gamma_n", "gn"), ("inclination_deg", "tilt_deg")):
        assert A[key] == g[k], k
    s = inputs.dem_avalanche(1.0)
    assert np.allclose(s.L, g["domain"], rtol=0, atol=1e-6)
    assert s.periodic == (0, 1, 0)  # walls in x, periodic y, open above the floor
    # the block fits the printed initial box (its y extent capped by the
    # domain's), up to the lattice jitter of 0.01 R at either end
    ext = s.pos.max(axis=0) - s.pos.min(axis=0) + 2 * A["R"]
    cap = np.minimum(np.array(g["initial_block"]), np.array(g["domain"]))
    jit = 2 * 0.01 * A["R"] + 1e-6
    assert np.all(ext <= cap + jit) and np.all(ext >= cap - 2 * 2 * A["R"])
    # the benchmark scale stands in for the printed grain count within 2 %
    n = len(inputs.dem_avalanche(4.2).pos)
    assert abs(n - g["benchmark_grains"]) / g["benchmark_grains"] < 0.02


def test_printed_grain_constants_closed_forms():
    g = fixture("dem_avalanche_constants.txt")
    # the moment of inertia of a solid sphere, 2/5 m R^2
    assert g["inertia"] == pytest.approx(0.4 * g["mass"] * g["R"] ** 2, rel=1e-12)
    # tangential stiffness 2/7 of the normal one, to the printed digits
    assert abs(g["kt"] - 2.0 / 7.0 * g["kn"]) < 5e-4


def test_sph_recipes_use_the_printed_constants():
    g = fixture("sph_dambreak_constants.txt")
    assert g["cutoff_over_nearest_neighbour_distance"] == pytest.approx(2 * math.sqrt(3), rel=1e-15)
    s = inputs.sph_column(8, 8)
    # hydrostatic start of the column from b = c0^2 rho0 / gamma with the
    # printed gamma and c0 = 20 sqrt(g H): top particle closest to rho0
    H, gacc, rho0 = s.H, 9.81, 1000.0
    c0 = g["c_sound_factor"] * math.sqrt(gacc * H)
    b = c0 * c0 * rho0 / g["gamma"]
    fluid = s.kind == 0
    z0 = float(s.pos[fluid, 2].min()) - 0.5 * s.dx
    depth = H - (s.pos[fluid, 2].astype(np.float64) - z0)
    expect = rho0 * (1.0 + rho0 * gacc * depth / b) ** (1.0 / g["gamma"])
    assert np.allclose(s.rho[fluid], expect, rtol=2e-6)
    d = inputs.sph_dambreak()
    # the dam-break stand-in is within 5 % of the printed particle count
    assert abs(len(d.pos) - g["dambreak_particles"]) / g["dambreak_particles"] < 0.05
