"""Reference for the circular dam break: the shallow-water equations under
radial symmetry, solved in one dimension (test infrastructure, plain FP64
numpy, independent of the oracle and of the GPU path).

With depth h(r, t) and radial discharge q = h u, per radian:
    (r h)_t + (r q)_r = 0
    (r q)_t + (r (q u + g h^2 / 2))_r = g h^2 / 2
Finite volumes on rings [r_i - dr/2, r_i + dr/2]: HLL fluxes through the
ring faces (area r_face), the hoop pressure g h^2 / 2 as a source, a wall at
r = 0 (zero face area: nothing crosses it) and a zero-gradient outer edge.
Forward Euler, CFL 0.45."""
import math

import numpy as np

G = 9.80665


def _hll(hl, ql, hr, qr, g, tol):
    ul = np.where(hl > tol, ql / np.maximum(hl, tol), 0.0)
    ur = np.where(hr > tol, qr / np.maximum(hr, tol), 0.0)
    cl, cr = np.sqrt(g * hl), np.sqrt(g * hr)
    sl = np.minimum(ul - cl, ur - cr)
    sr = np.maximum(ul + cl, ur + cr)
    fl = np.stack([ql, ql * ul + 0.5 * g * hl * hl])
    fr = np.stack([qr, qr * ur + 0.5 * g * hr * hr])
    dl, dr_ = np.stack([hl, ql]), np.stack([hr, qr])
    den = np.where(sr - sl > 0.0, sr - sl, 1.0)
    mid = (sr * fl - sl * fr + sl * sr * (dr_ - dl)) / den
    return np.where(sl >= 0.0, fl, np.where(sr <= 0.0, fr, mid))


def radial_dambreak(h_in, h_out, r_dam, r_max, n, t_end, g=G, cfl=0.45, tol=1e-12):
    """Depth and discharge at ring centres r_i = (i + 1/2) dr at t_end."""
    dr = r_max / n
    rc = (np.arange(n) + 0.5) * dr
    rf = np.arange(n + 1) * dr          # face radii; rf[0] = 0 is the axis
    h = np.where(rc < r_dam, h_in, h_out).astype(np.float64)
    q = np.zeros(n)
    t = 0.0
    while t < t_end:
        u = np.where(h > tol, q / np.maximum(h, tol), 0.0)
        smax = float(np.max(np.abs(u) + np.sqrt(g * h)))
        dt = min(cfl * dr / smax, t_end - t)
        # faces 1..n-1 interior; face n zero-gradient; face 0 has zero area
        hl = np.concatenate([h[:1], h])
        ql = np.concatenate([-q[:1], q])
        hr = np.concatenate([h, h[-1:]])
        qr = np.concatenate([q, q[-1:]])
        F = _hll(hl, ql, hr, qr, g, tol)          # (2, n + 1)
        rF = F * rf[None, :]
        vol = rc * dr
        h = h - dt * (rF[0, 1:] - rF[0, :-1]) / vol
        q = q - dt * (rF[1, 1:] - rF[1, :-1]) / vol + dt * 0.5 * g * hl[1:] ** 2 * dr / vol
        t += dt
    return rc, h, q


def ring_mass(rc, h, dr):
    return float(np.sum(2.0 * math.pi * rc * dr * h))
