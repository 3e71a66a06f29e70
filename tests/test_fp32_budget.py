"""Error budget of FP32 pair arithmetic, the alternative to the FP64 pair math
of the force kernels (section 4.1's force, evaluated over the same FP32 pair
set): squared distances, 1/r^2, the force factor and the per-particle sums in
FP32 (each operation rounded, sums in ascending neighbour order), against the
FP64 oracle, on every atom of the 4096-atom liquid and on 4096 sampled atoms
of the 1M-atom liquid (errors as the largest and the 99.9th-percentile force
component error in units of the RMS force).

Two ways to form the separation: in FP32 (x_i - x_j rounded, then the
periodic shift +-L added and rounded again), and exactly (the FP32 rounding of
the exact separation of the image).  The second rounding of the first way
costs up to half an ulp of the box length, 3.8e-6 at L = 105.8, which the
steep r^-13 force turns into errors above the 1e-5 parity bar for image pairs
of the 1M-atom box; with exact separations FP32 arithmetic stays below the
bar, with a margin of about three.  The kernels take exact FP64 separations
and FP64 pair math, whose error is orders of magnitude below the bar."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1804_07598_amd import inputs

PER = (1, 1, 1)
RC = 2.5


def fp32_forces(pos, L, rows, counts, cols, exact_sep=False):
    """FP32 LJ forces (eps = sig = 1) on `rows` from their neighbour columns."""
    f32 = np.float32
    p = pos.astype(f32)
    Lf = L.astype(f32)
    half = Lf / f32(2)
    rc2 = O.radius2(RC)
    F = np.zeros((len(rows), 3), f32)
    pi = p[rows]
    for k in range(int(counts.max())):
        on = counts > k
        j = np.where(on, cols[:, k], rows)
        d = pi - p[j]                      # x_i - x_j, FP32
        t = -d                             # the predicate's q - p
        if exact_sep:
            d = pi.astype(np.float64) - p[j].astype(np.float64)
            L64 = Lf.astype(np.float64)
            d = np.where(t > half, d + L64, np.where(t < -half, d - L64, d)).astype(f32)
        else:
            d = np.where(t > half, d + Lf, np.where(t < -half, d - Lf, d)).astype(f32)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]).astype(f32) + (d[:, 2] * d[:, 2]).astype(f32)
        r2 = r2.astype(f32)
        use = on & (r2 <= rc2) & (r2 > 0)
        r2i = (f32(1) / np.where(use, r2, f32(1))).astype(f32)
        r6i = (r2i * r2i * r2i).astype(f32)
        s = (r6i * r2i * (f32(48) * r6i - f32(24))).astype(f32)
        s = np.where(use, s, f32(0))
        F = (F + s[:, None] * d).astype(f32)
    return F.astype(np.float64)


def budget(s, rows):
    R2 = O.radius2(RC)
    counts, cols = O.neighbors(s.pos, s.box, PER, R2, rows=rows, cap=160)
    F64, _, _, _, _ = O.lj(s.pos, s.box, PER, R2, rows=rows)
    out = []
    for exact in (False, True):
        F32 = fp32_forces(s.pos, s.box, rows, counts, cols, exact)
        err = np.abs(F32 - F64) / math.sqrt((F64 ** 2).mean())
        out.append((float(err.max()), float(np.quantile(err, 0.999))))
    return out


@pytest.mark.parametrize("name,nrows", [("lj4096", None), ("lj1m", 4096)])
def test_fp32_pair_math_error_budget(name, nrows):
    s = inputs.lj_config(name)
    rng = np.random.default_rng(0)
    rows = (np.arange(s.n) if nrows is None else np.sort(rng.choice(s.n, nrows, replace=False)))
    (mx, p999), (mx_e, p999_e) = budget(s, rows.astype(np.int64))
    print(f"\n{name} ({len(rows)} atoms), FP32 pair math, |dF| / RMS(F): FP32 separations "
          f"max {mx:.2e}, p99.9 {p999:.2e}; exact separations max {mx_e:.2e}, p99.9 {p999_e:.2e}")
    assert mx_e <= 1e-5 and p999_e <= mx_e <= mx
    if name == "lj1m":
        assert mx > 1e-5  # the twice-rounded image separations miss the bar
