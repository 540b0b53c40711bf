"""Seeded synthetic inputs for the HWFV1 workloads.

This module is shared by the CPU oracle and the HIP path.  It holds only the
recipes that produce inputs (bed, initial state, forcing and the problem
parameters); none of the method's arithmetic lives here.  All arrays are
float64, row-major [j, i] with j the row (y, south to north) and i the column
(x, west to east), sampled at cell centres ((i + 1/2) dx, (j + 1/2) dy).

Workloads (square 2^L x 2^L grids):
  dambreak_bumps_l6        1 x 1 m box, 8 Gaussian bumps, walls, eps 1e-3,
                           dam break eta 2 m / 1 m at x = 0.5 m, t_end 0.05 s
  circular_dambreak_l10    1000 x 1000 m, fractal bed (relief 10 m), 5 m deep
                           cylinder of radius 100 m over a dry bed, Manning
                           0.035, open boundaries, 500 steps
  hydrograph_l12           10 x 10 km, fractal bed (relief 50 m), dry start,
                           triangular west-edge inflow (500 m^3/s peak at
                           1800 s, base 3600 s) through a closed west edge,
                           other edges open, Manning 0.035, 2000 steps
  hydrograph_wet_window    the hydrograph terrain and forcing from t0 = 1500 s
                           with a pond 2 m deep at the inlet's centre (test)
  ensemble_64              64 members with L in {8..11}, eps in
                           {1e-4, 1e-3, 1e-2}, own fractal bed (relief 5-50 m),
                           dam-break or hydrograph forcing, Manning U(0.01,
                           0.06), 1000 steps
  sheetflow_l13            10 x 10 km, fractal bed (relief 500 m), 1 mm sheet,
                           50 mm/h rain, Manning 0.05, eps 1e-4, 1000 steps
"""
from dataclasses import dataclass, field
import math

import numpy as np

G = 9.80665


@dataclass
class Workload:
    name: str
    params: dict
    h: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    z: np.ndarray
    n_steps: int
    meta: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return int(self.params["L"])


def base_params(L: int, length: float, eps: float, **kw) -> dict:
    """Problem parameters with the shared defaults (g, CFL 0.5, h_tol)."""
    dx = length / (1 << L)
    p = dict(L=L, eps=eps, g=G, cfl=0.5, h_tol=1e-6, dx=dx, dy=dx,
             dt_max=0.5 * dx / math.sqrt(G * 1.0), manning_n=0.0,
             rain_rate=0.0, bc=("wall",) * 4, inlet_y0=0.0, inlet_y1=0.0,
             q_peak=0.0, t_peak=1.0, t_base=2.0, t_end=math.inf)
    p.update(kw)
    return p


def cell_centres(L: int, length: float):
    n = 1 << L
    dx = length / n
    c = (np.arange(n) + 0.5) * dx
    x = np.broadcast_to(c[None, :], (n, n))
    y = np.broadcast_to(c[:, None], (n, n))
    return x, y


def gaussian_bumps(L: int, length: float, count: int, seed: int,
                   amp=(0.0, 0.2), width=(0.02, 0.1)) -> np.ndarray:
    """Sum of Gaussian bumps; amplitude, width (standard deviation) and the
    two centre coordinates are drawn in that order as arrays of `count`."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(amp[0], amp[1], count)
    w = rng.uniform(width[0], width[1], count) * length
    xc = rng.uniform(0.0, 1.0, count) * length
    yc = rng.uniform(0.0, 1.0, count) * length
    x, y = cell_centres(L, length)
    z = np.zeros((1 << L, 1 << L))
    for k in range(count):
        r2 = (x - xc[k]) ** 2 + (y - yc[k]) ** 2
        z += a[k] * np.exp(-r2 / (2.0 * w[k] ** 2))
    return z


def fractal_bed(L: int, relief: float, seed: int,
                exponent: float = -2.5) -> np.ndarray:
    """Spectral fractal terrain: white noise shaped so that its power
    spectrum falls as |k|^exponent, zero mean, scaled to [0, relief]."""
    n = 1 << L
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n))
    spec = np.fft.rfft2(white)
    del white
    ky = np.fft.fftfreq(n)[:, None]
    kx = np.fft.rfftfreq(n)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    k[0, 0] = 1.0
    spec *= k ** (exponent / 2.0)
    spec[0, 0] = 0.0
    del k
    z = np.fft.irfft2(spec, s=(n, n))
    del spec
    lo, hi = z.min(), z.max()
    z -= lo
    z *= relief / (hi - lo)
    return z


def dambreak_bumps_l6(seed: int = 1, L: int = 6) -> Workload:
    length = 1.0
    p = base_params(L, length, 1e-3, t_end=0.05, bc=("wall",) * 4)
    z = gaussian_bumps(L, length, 8, seed)
    x, _ = cell_centres(L, length)
    eta = np.where(x < 0.5, 2.0, 1.0)
    h = np.maximum(0.0, eta - z)
    zero = np.zeros_like(h)
    return Workload(f"dambreak_bumps_l{L}", p, h, zero, zero.copy(), z,
                    n_steps=10_000, meta=dict(seed=seed))


def circular_dambreak_l10(seed: int = 2, L: int = 10,
                          n_steps: int = 500) -> Workload:
    length = 1000.0
    p = base_params(L, length, 1e-3, manning_n=0.035, bc=("open",) * 4)
    z = fractal_bed(L, 10.0, seed)
    x, y = cell_centres(L, length)
    r = np.sqrt((x - 500.0) ** 2 + (y - 500.0) ** 2)
    h = np.where(r < 100.0, 5.0, 0.0)
    zero = np.zeros_like(h)
    return Workload(f"circular_dambreak_l{L}", p, h, zero, zero.copy(), z,
                    n_steps=n_steps, meta=dict(seed=seed))


def hydrograph_l12(seed: int = 3, L: int = 12, n_steps: int = 2000,
                   relief: float = 50.0, q_peak: float = 500.0) -> Workload:
    length = 10_000.0
    # The inflow edge is closed: the hydrograph is the only water entering
    # there (a zero-gradient copy would import water wherever the inflow
    # pushes the flow away from the edge).
    p = base_params(L, length, 1e-3, manning_n=0.035,
                    bc=("wall", "open", "open", "open"),
                    inlet_y0=4500.0, inlet_y1=5500.0, q_peak=q_peak,
                    t_peak=1800.0, t_base=3600.0)
    z = fractal_bed(L, relief, seed)
    zero = np.zeros((1 << L, 1 << L))
    return Workload(f"hydrograph_l{L}", p, zero, zero.copy(), zero.copy(), z,
                    n_steps=n_steps, meta=dict(seed=seed))


def flooded_basin_l12(seed: int = 3, L: int = 12, n_steps: int = 200,
                      relief: float = 50.0) -> Workload:
    """The hydrograph terrain under still water 10 m above its highest point,
    with a 2 m higher circular mound (radius 500 m) at the centre released
    at t = 0: every cell is wet, so every leaf takes the full update."""
    length = 10_000.0
    p = base_params(L, length, 1e-3, manning_n=0.035, bc=("open",) * 4)
    z = fractal_bed(L, relief, seed)
    x, y = cell_centres(L, length)
    r = np.sqrt((x - 5000.0) ** 2 + (y - 5000.0) ** 2)
    eta = relief + 10.0 + np.where(r < 500.0, 2.0, 0.0)
    h = eta - z
    zero = np.zeros_like(h)
    return Workload(f"flooded_basin_l{L}", p, h, zero, zero.copy(), z,
                    n_steps=n_steps, meta=dict(seed=seed))


def hydrograph_wet_window(seed: int = 3, L: int = 12, t0: float = 1500.0,
                          relief: float = 50.0) -> Workload:
    """A wet window of the hydrograph run: its terrain, inflow and
    boundaries, started at t0 (near the peak) with water already stored at
    the inlet: a pond whose surface lies 2 m above the bed at the inlet's
    centre, filling the bed below it within 2.5 km of the west edge and
    2 km of the inlet's centre line, flowing east at 0.2 m/s.  Wet and dry
    cells, a moving front and the inflow in one step (meta t0: the start
    time both sides set)."""
    w = hydrograph_l12(seed=seed, L=L, relief=relief)
    length = 10_000.0
    x, y = cell_centres(L, length)
    z = w.z
    n = 1 << L
    j0 = min(n - 1, int(5000.0 / length * n))
    eta0 = z[j0, 0] + 2.0
    inside = (x < 2500.0) & (np.abs(y - 5000.0) < 2000.0)
    h = np.where(inside, np.maximum(0.0, eta0 - z), 0.0)
    qx = 0.2 * h
    zero = np.zeros_like(h)
    return Workload(f"hydrograph_wet_window_l{L}", dict(w.params), h, qx, zero, z,
                    n_steps=5, meta=dict(seed=seed, t0=t0, eta0=float(eta0)))


def sheetflow_l13(seed: int = 5, L: int = 13, n_steps: int = 1000) -> Workload:
    length = 10_000.0
    p = base_params(L, length, 1e-4, manning_n=0.05, bc=("open",) * 4,
                    rain_rate=0.05 / 3600.0)
    z = fractal_bed(L, 500.0, seed)
    h = np.full((1 << L, 1 << L), 1e-3)
    zero = np.zeros_like(h)
    return Workload(f"sheetflow_l{L}", p, h, zero, zero.copy(), z,
                    n_steps=n_steps, meta=dict(seed=seed))


def ensemble_member(i: int, n_steps: int = 1000, levels=(8, 9, 10, 11),
                    base_seed: int = 1000) -> Workload:
    """Member i of the batched ensemble; its own generator draws L, eps,
    relief, Manning n, the forcing kind and the terrain seed."""
    rng = np.random.default_rng(base_seed + i)
    L = int(rng.choice(levels))
    eps = float(rng.choice([1e-4, 1e-3, 1e-2]))
    relief = float(rng.uniform(5.0, 50.0))
    n_m = float(rng.uniform(0.01, 0.06))
    kind = "dambreak" if rng.uniform() < 0.5 else "hydrograph"
    tseed = int(rng.integers(0, 2**31 - 1))
    length = 1000.0
    z = fractal_bed(L, relief, tseed)
    zero = np.zeros((1 << L, 1 << L))
    if kind == "dambreak":
        p = base_params(L, length, eps, manning_n=n_m, bc=("open",) * 4)
        x, y = cell_centres(L, length)
        r = np.sqrt((x - 500.0) ** 2 + (y - 500.0) ** 2)
        h = np.where(r < 100.0, 5.0, 0.0)
    else:
        p = base_params(L, length, eps, manning_n=n_m,
                        bc=("wall", "open", "open", "open"),
                        inlet_y0=450.0, inlet_y1=550.0, q_peak=50.0,
                        t_peak=1800.0, t_base=3600.0)
        h = zero.copy()
    return Workload(f"ensemble_member_{i}_l{L}", p, h, zero.copy(),
                    zero.copy(), z, n_steps=n_steps,
                    meta=dict(member=i, kind=kind, relief=relief,
                              terrain_seed=tseed))


def ensemble_64(n: int = 64, n_steps: int = 1000, levels=(8, 9, 10, 11)):
    return [ensemble_member(i, n_steps, levels) for i in range(n)]


# Small scenarios used by tests ------------------------------------------------
def lake_at_rest(L: int, eta: float, seed: int, eps: float,
                 length: float = 1.0, amp=(0.1, 0.6)) -> Workload:
    """Still water at free-surface eta over Gaussian bumps (dry where the
    bumps rise above eta), closed walls."""
    p = base_params(L, length, eps, bc=("wall",) * 4)
    z = gaussian_bumps(L, length, 6, seed, amp=amp, width=(0.05, 0.15))
    h = np.maximum(0.0, eta - z)
    zero = np.zeros_like(h)
    return Workload(f"lake_at_rest_l{L}", p, h, zero, zero.copy(), z,
                    n_steps=1000, meta=dict(seed=seed, eta=eta))


def dambreak_strip(L: int, h_left: float, h_right: float, x_dam: float,
                   length: float, eps: float, t_end: float,
                   axis: str = "x") -> Workload:
    """1D dam break across a square domain: walls parallel to the flow,
    open ends, flat frictionless bed."""
    if axis == "x":
        bc = ("open", "open", "wall", "wall")
    else:
        bc = ("wall", "wall", "open", "open")
    p = base_params(L, length, eps, bc=bc, t_end=t_end)
    x, y = cell_centres(L, length)
    coord = x if axis == "x" else y
    h = np.where(coord < x_dam, h_left, h_right).astype(np.float64)
    zero = np.zeros_like(h)
    return Workload(f"dambreak_strip_l{L}", p, h, zero, zero.copy(),
                    zero.copy(), n_steps=100_000,
                    meta=dict(h_left=h_left, h_right=h_right, x_dam=x_dam))


def circular_dambreak_flat(L: int = 8, eps: float = 1e-3, radius: float = 2.5,
                           t_end: float = 3.5, centre=(21.3, 20.7)) -> Workload:
    """Circular dam break of Section 3.2: closed [-20, 20]^2 m domain (here
    [0, 40]^2), flat frictionless bed, depth 2.5 m inside the dam and 0.5 m
    outside, run to 3.5 s.  The paper does not print the dam's radius; 2.5 m
    is taken.  The dam is centred at (1.3, 0.7) m from the domain centre: a
    dam centred on the corner shared by the root's four quadrants gives the
    root (and every coarse cell centred on it) zero details by symmetry, and
    the tree, which stops at the first cell without a significant detail,
    would then be the root alone."""
    length = 40.0
    p = base_params(L, length, eps, bc=("wall",) * 4, t_end=t_end)
    x, y = cell_centres(L, length)
    r = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2)
    h = np.where(r < radius, 2.5, 0.5)
    zero = np.zeros_like(h)
    return Workload(f"circular_dambreak_flat_l{L}", p, h, zero, zero.copy(), zero.copy(),
                    n_steps=100_000, meta=dict(radius=radius))


def pseudo2d_dambreak(L: int = 8, eps: float = 1e-3, t_end: float = 40.0) -> Workload:
    """Pseudo-2D dam break of Section 3.2: flat frictionless bed, 6 m of
    water upstream of a dam at x = 10 m and 2 m downstream, open ends, run
    to 40 s (shock and rarefaction leave the domain; the flow then smooths).
    The paper's domain is 50 m x 25 m; the flow does not depend on y, so the
    square 50 m x 50 m domain (walls along the flow) carries the same
    solution on every row."""
    w = dambreak_strip(L, 6.0, 2.0, 10.0, 50.0, eps, t_end, axis="x")
    w.name = f"pseudo2d_dambreak_l{L}"
    return w


def pseudo2d_channel(L: int = 8, eps: float = 1e-3, t_end: float = 40.0) -> Workload:
    """The pseudo-2D dam break on the paper's 50 m x 25 m domain: the
    channel fills the lower half of the 50 m square grid (rows along y),
    the upper half is dry ground 1000 m above the water (a closed edge in
    the hydrostatic reconstruction)."""
    w = pseudo2d_dambreak(L, eps, t_end)
    n = 1 << L
    # s_max of the bed over the channel's own cells (the guard value 1 on
    # this flat bed), not over the padding
    w.params = dict(w.params, zsmax=max(1.0, float(np.abs(w.z[: n // 2]).max())))
    w.h[n // 2:, :] = 0.0
    w.z[n // 2:, :] = 1000.0
    w.name = f"pseudo2d_channel_l{L}"
    w.meta = dict(w.meta, channel_rows=n // 2)
    return w


HUMP_ETA = {"smooth": 0.875, "steeper": 1.78, "rectangular": 1.95}


def humps_lake_at_rest(profile: str, L: int = 8, eps: float = 1e-3,
                       t_end: float = 100.0) -> Workload:
    """Still water over three humps in a closed 70 m x 30 m basin (the
    well-balancedness case of Section 3.1, whose hump shapes are only
    drawn): free surface eta of Table 3, zero discharges.  Humps at (30, 6),
    (30, 24) and (47.5, 15) m, chosen so that the water is dry around the
    highest one, critical (h = 0) at the peak of the one whose peak equals
    eta, and wet above the lowest:
      smooth       cones of peak 0.875, 0.875, 3 m and radius 8, 8, 10 m;
      steeper      cones of peak 1.0, 1.78, 3 m and radius 2.5, 3, 5 m;
      rectangular  square blocks of height 1.0, 1.95, 3 m and side 6, 6, 8 m.
    The basin is rows 0..ny-1 of the 2^L-cell-wide square grid (cell size
    70 / 2^L, ny = 30 m / cell rounded), the rows above are dry ground
    1000 m above the water (a closed edge, like the walls); the bed's s_max
    is that of the basin (params zsmax)."""
    eta = HUMP_ETA[profile]
    length = 70.0
    n = 1 << L
    dx = length / n
    ny = int(round(30.0 / dx))
    p = base_params(L, length, eps, bc=("wall",) * 4, t_end=t_end,
                    dt_max=0.5 * dx / math.sqrt(G * 1e-3))
    x, y = cell_centres(L, length)
    centres = [(30.0, 6.0), (30.0, 24.0), (47.5, 15.0)]
    z = np.zeros((n, n))
    if profile == "rectangular":
        for (cx, cy), top, side in zip(centres, (1.0, 1.95, 3.0), (6.0, 6.0, 8.0)):
            inside = (np.abs(x - cx) <= side / 2) & (np.abs(y - cy) <= side / 2)
            z = np.where(inside, np.maximum(z, top), z)
    else:
        peaks, radii = {"smooth": ((0.875, 0.875, 3.0), (8.0, 8.0, 10.0)),
                        "steeper": ((1.0, 1.78, 3.0), (2.5, 3.0, 5.0))}[profile]
        for (cx, cy), top, rad in zip(centres, peaks, radii):
            r = np.hypot(x - cx, y - cy)
            z = np.maximum(z, top * np.maximum(0.0, 1.0 - r / rad))
    h = np.maximum(0.0, eta - z)
    # s_max of the bed over the basin's own cells (3 m, the highest hump),
    # not over the padding
    p["zsmax"] = max(1.0, float(np.abs(z[:ny]).max()))
    z[ny:, :] = 1000.0
    h[ny:, :] = 0.0
    zero = np.zeros_like(h)
    return Workload(f"humps_{profile}_l{L}", p, h, zero, zero.copy(), z,
                    n_steps=3000, meta=dict(eta=eta, basin_rows=ny, profile=profile))


def humps_dambreak(L: int = 8, eps: float = 1e-3, t_end: float = 12.0) -> Workload:
    """The frictional dam break of Section 3.1 over the smooth humps of
    humps_lake_at_rest: water surface 1.875 m behind a dam at x = 16 m
    (depth 1.875 m - z where positive), dry beyond it, zero discharges,
    Manning n = 0.018, closed 70 m x 30 m basin."""
    w = humps_lake_at_rest("smooth", L, eps, t_end)
    rows = w.meta["basin_rows"]
    x, _ = cell_centres(L, 70.0)
    h = np.where(x < 16.0, np.maximum(0.0, 1.875 - w.z), 0.0)
    h[rows:, :] = 0.0
    w.h = h
    w.params = dict(w.params, manning_n=0.018)
    w.name = f"humps_dambreak_l{L}"
    w.meta = dict(w.meta, x_dam=16.0, surface=1.875)
    return w


def dry_patches(L: int, seed: int, n_rect: int = 4, n_single: int = 12,
                inlet: bool = False, rain: float = 0.0) -> Workload:
    """Mostly dry domain over a rough bed (uniform noise of 1 m on every
    cell, so that every detail of z is significant and every leaf is
    finest): a few wet rectangles and single wet cells of depth 0.3 m, and
    cells whose depth equals h_tol (dry) or twice it (wet).  Drawn in that
    order: bed, rectangle corners and sizes, single-cell positions, the
    h_tol cells.  Optional west-edge inlet over the middle fifth and rain."""
    rng = np.random.default_rng(seed)
    n = 1 << L
    tol = 1e-3
    kw = dict(h_tol=tol, bc=("wall", "open", "wall", "open"), rain_rate=rain)
    if inlet:
        kw.update(inlet_y0=0.4, inlet_y1=0.6, q_peak=0.05, t_peak=1.0, t_base=2.0)
    p = base_params(L, 1.0, 1e-3, **kw)
    z = rng.uniform(0.0, 1.0, (n, n))
    h = np.zeros((n, n))
    for _ in range(n_rect):
        j0, i0 = rng.integers(0, n, 2)
        hj, hi = rng.integers(1, max(2, n // 8) + 1, 2)
        h[j0:j0 + hj, i0:i0 + hi] = 0.3
    jj, ii = rng.integers(0, n, (2, n_single))
    h[jj, ii] = 0.3
    jt, it = rng.integers(0, n, (2, n_single))
    h[jt, it] = np.where(np.arange(n_single) % 2 == 0, tol, 2 * tol)
    zero = np.zeros_like(h)
    return Workload(f"dry_patches_l{L}", p, h, zero, zero.copy(), z,
                    n_steps=10, meta=dict(seed=seed))


BY_NAME = {
    "dambreak_bumps_l6": dambreak_bumps_l6,
    "circular_dambreak_l10": circular_dambreak_l10,
    "hydrograph_l12": hydrograph_l12,
    "sheetflow_l13": sheetflow_l13,
}
