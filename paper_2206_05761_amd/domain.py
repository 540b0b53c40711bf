"""Rectangular domains on the 2^L x 2^L grid.

The multiresolution hierarchy needs a square grid of 2^L cells a side.  A
domain of ny x nx cells (row-major, rows along y) is placed in the lower-left
corner of the smallest such grid (or of a given L) and the rest is filled
with dry cells whose bed lies far above any water surface in the domain.  In
the hydrostatic reconstruction every face between a wet cell and such a
cell has zero depth on both sides: no mass crosses it, and the pressure of
the wet cell's own depth is balanced by the bed-slope term, so the padding
acts as a closed edge.  The padded cells stay dry; the bed step makes their
edge a significant detail, so the grid is refined along it.

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

    def crop(self, a):
        """The domain's part of a padded 2^L x 2^L row-major array."""
        ny, nx = self.shape
        return np.asarray(a).reshape(1 << self.L, 1 << self.L)[:ny, :nx]


def pad_to_grid(h, qx, qy, z, L=None, wall_z=None) -> Padded:
    """Pad row-major ny x nx fields to 2^L x 2^L.  L defaults to the smallest
    level whose grid holds the domain; wall_z (the bed of the padding)
    defaults to 1000 m above the highest water surface or bed in the
    domain."""
    arrs = [np.asarray(a, dtype=np.float64) for a in (h, qx, qy, z)]
    shape = arrs[0].shape
    if len(shape) != 2 or any(a.shape != shape for a in arrs):
        raise ValueError("h, qx, qy, z must be 2-D arrays of one shape")
    ny, nx = shape
    need = max(int(np.ceil(np.log2(max(ny, nx, 1)))), 0)
    if L is None:
        L = need
    elif L < need:
        raise ValueError(f"L = {L} holds at most {1 << L} cells a side, the domain has {ny} x {nx}")
    if wall_z is None:
        wall_z = float(np.max(arrs[3] + np.maximum(arrs[0], 0.0))) + 1000.0
    n = 1 << L
    out = []
    for k, a in enumerate(arrs):
        p = np.full((n, n), wall_z if k == 3 else 0.0)
        p[:ny, :nx] = a
        out.append(p)
    return Padded(L, out[0], out[1], out[2], out[3], (ny, nx), float(wall_z))
