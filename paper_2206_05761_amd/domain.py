"""Rectangular domains and gridded DEMs on the 2^L x 2^L grid.

The multiresolution hierarchy needs a square grid of 2^L cells a side.  A
domain of ny x nx cells (row-major, rows along y) is placed in the lower-left
corner of the smallest such grid (or of a given L) and the rest, together
with any cell the domain marks as missing (a DEM's NODATA cells), is filled
with dry cells whose bed lies far above any water surface in the domain.  In
the hydrostatic reconstruction every face between a wet cell and such a
cell has zero depth on both sides: no mass crosses it, and the pressure of
the wet cell's own depth is balanced by the bed-slope term, so the padding
acts as a closed edge.  The padded cells stay dry; the bed step makes their
edge a significant detail, so the grid is refined along it.

The bed's s_max of the significance test (Section 2.1.2: the largest bed
coefficient of the finest level) is taken over the domain's own cells and
handed to the library as the problem's `zsmax`, so that the padding's high
ground does not rescale the bed details inside the domain.

Host-side input preparation only (numpy); the simulation itself is
unchanged."""
from dataclasses import dataclass

import numpy as np


@dataclass
class Padded:
    L: int
    h: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    z: np.ndarray
    shape: tuple          # (ny, nx) of the domain
    wall_z: float
    zsmax: float          # s_max of the bed over the domain's cells
    valid: np.ndarray     # padded grid: True on the domain's own cells

    def crop(self, a):
        """The domain's part of a padded 2^L x 2^L row-major array."""
        ny, nx = self.shape
        return np.asarray(a).reshape(1 << self.L, 1 << self.L)[:ny, :nx]


def bed_smax(z, valid=None) -> float:
    """max(1, max |z|) over the valid cells (the guarded s_max)."""
    z = np.asarray(z, dtype=np.float64)
    if valid is not None:
        z = z[np.asarray(valid, dtype=bool)]
    m = float(np.max(np.abs(z))) if z.size else 0.0
    return m if m > 1.0 else 1.0


def pad_to_grid(h, qx, qy, z, L=None, wall_z=None, valid=None) -> Padded:
    """Pad row-major ny x nx fields to 2^L x 2^L.  L defaults to the smallest
    level whose grid holds the domain; valid (ny x nx booleans, default all)
    marks the domain's own cells, the others become padding as well;
    wall_z (the bed of the padding) defaults to 1000 m above the highest
    water surface or bed of the domain."""
    arrs = [np.asarray(a, dtype=np.float64) for a in (h, qx, qy, z)]
    shape = arrs[0].shape
    if len(shape) != 2 or any(a.shape != shape for a in arrs):
        raise ValueError("h, qx, qy, z must be 2-D arrays of one shape")
    ny, nx = shape
    ok = np.ones(shape, dtype=bool) if valid is None else np.asarray(valid, dtype=bool)
    if ok.shape != shape:
        raise ValueError("valid must have the domain's shape")
    if not ok.any():
        raise ValueError("the domain has no valid cell")
    need = max(int(np.ceil(np.log2(max(ny, nx, 1)))), 0)
    if L is None:
        L = need
    elif L < need:
        raise ValueError(f"L = {L} holds at most {1 << L} cells a side, the domain has {ny} x {nx}")
    if wall_z is None:
        wall_z = float(np.max((arrs[3] + np.maximum(arrs[0], 0.0))[ok])) + 1000.0
    n = 1 << L
    out = []
    for k, a in enumerate(arrs):
        fill = wall_z if k == 3 else 0.0
        p = np.full((n, n), fill)
        p[:ny, :nx] = np.where(ok, a, fill)
        out.append(p)
    mask = np.zeros((n, n), dtype=bool)
    mask[:ny, :nx] = ok
    return Padded(L, out[0], out[1], out[2], out[3], (ny, nx), float(wall_z),
                  bed_smax(arrs[3], ok), mask)


@dataclass
class Dem:
    z: np.ndarray         # row-major [j, i], j = 0 the southernmost row
    valid: np.ndarray     # False where the file holds NODATA
    cellsize: float
    xll: float            # lower-left corner of the grid (m)
    yll: float


def read_esri_ascii(path) -> Dem:
    """Gridded DEM in the ESRI ASCII format: a header of ncols, nrows,
    xllcorner (or xllcenter), yllcorner (or yllcenter), cellsize and an
    optional NODATA_value, then nrows rows of ncols heights from the
    northernmost row down.  Rows are flipped so that j grows northwards."""
    head = {}
    with open(path) as fh:
        lines = fh.read().split("\n")
    k = 0
    while k < len(lines):
        parts = lines[k].split()
        if not parts:
            k += 1
            continue
        key = parts[0].lower()
        if key in ("ncols", "nrows", "xllcorner", "yllcorner", "xllcenter",
                   "yllcenter", "cellsize", "nodata_value"):
            if len(parts) != 2:
                raise ValueError(f"malformed header line: {lines[k]!r}")
            head[key] = float(parts[1])
            k += 1
        else:
            break
    for key in ("ncols", "nrows", "cellsize"):
        if key not in head:
            raise ValueError(f"header lacks {key}")
    nx, ny = int(head["ncols"]), int(head["nrows"])
    cs = head["cellsize"]
    if nx < 1 or ny < 1 or not cs > 0:
        raise ValueError("ncols, nrows and cellsize must be positive")
    vals = np.array(" ".join(lines[k:]).split(), dtype=np.float64)
    if vals.size != nx * ny:
        raise ValueError(f"expected {nx * ny} heights, found {vals.size}")
    z = vals.reshape(ny, nx)[::-1].copy()
    valid = np.isfinite(z)
    if "nodata_value" in head:
        valid &= z != head["nodata_value"]
    if "xllcorner" in head:
        xll = head["xllcorner"]
    else:
        xll = head.get("xllcenter", 0.5 * cs) - 0.5 * cs
    if "yllcorner" in head:
        yll = head["yllcorner"]
    else:
        yll = head.get("yllcenter", 0.5 * cs) - 0.5 * cs
    z = np.where(valid, z, 0.0)
    return Dem(z, valid, cs, xll, yll)


def dem_domain(dem: Dem, h=None, qx=None, qy=None, L=None, wall_z=None) -> Padded:
    """A DEM (and optional initial depth and discharges on its grid, zero by
    default) padded to the square grid, its NODATA cells closed off like the
    padding."""
    zero = np.zeros_like(dem.z)
    h = zero if h is None else np.where(dem.valid, h, 0.0)
    qx = zero if qx is None else np.where(dem.valid, qx, 0.0)
    qy = zero if qy is None else np.where(dem.valid, qy, 0.0)
    return pad_to_grid(h, qx, qy, dem.z, L=L, wall_z=wall_z, valid=dem.valid)
