"""Exact solution of the 1D shallow-water Riemann problem on a flat,
frictionless bed (E. F. Toro, Shock-Capturing Methods for Free-Surface
Shallow Flows, Wiley 2001, chapter 5; the dry-bed case is Ritter's solution).

Used only as an independent pin of the oracle's FV1 operator: the oracle never
calls it.
"""
import math

import numpy as np


def _f(h, hk, g):
    """Depth function of one wave: rarefaction when h <= hk, shock else."""
    if h <= hk:
        return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))
    return (h - hk) * math.sqrt(0.5 * g * (h + hk) / (h * hk))


def _df(h, hk, g):
    if h <= hk:
        return math.sqrt(g / h)
    a = math.sqrt(0.5 * g * (h + hk) / (h * hk))
    return a - 0.25 * g * (h - hk) / (a * h * h)


def star_state(hl, ul, hr, ur, g):
    """Depth and velocity between the two waves (wet bed on both sides)."""
    cl, cr = math.sqrt(g * hl), math.sqrt(g * hr)
    # two-rarefaction initial guess
    h = (0.5 * (cl + cr) - 0.25 * (ur - ul)) ** 2 / g
    h = max(h, 1e-8)
    for _ in range(100):
        F = _f(h, hl, g) + _f(h, hr, g) + ur - ul
        d = _df(h, hl, g) + _df(h, hr, g)
        hn = max(h - F / d, 1e-12)
        if abs(hn - h) <= 1e-15 * max(1.0, h):
            h = hn
            break
        h = hn
    u = 0.5 * (ul + ur) + 0.5 * (_f(h, hr, g) - _f(h, hl, g))
    return h, u


def sample(hl, ul, hr, ur, g, xi):
    """Depth and velocity at the similarity coordinates xi = (x - x0) / t."""
    xi = np.asarray(xi, dtype=np.float64)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    cl = math.sqrt(g * hl)
    if hr == 0.0:
        # Ritter: rarefaction into a dry bed.
        head, front = ul - cl, ul + 2.0 * cl
        for k, x in enumerate(xi):
            if x <= head:
                h[k], u[k] = hl, ul
            elif x < front:
                c = (ul + 2.0 * cl - x) / 3.0
                h[k], u[k] = c * c / g, (ul + 2.0 * cl + 2.0 * x) / 3.0
            else:
                h[k], u[k] = 0.0, 0.0
        return h, u
    cr = math.sqrt(g * hr)
    hs, us = star_state(hl, ul, hr, ur, g)
    cs = math.sqrt(g * hs)
    for k, x in enumerate(xi):
        if x <= us:  # left of the contact
            if hs > hl:  # left shock
                s = ul - cl * math.sqrt(0.5 * (hs + hl) * hs / (hl * hl))
                h[k], u[k] = (hl, ul) if x <= s else (hs, us)
            else:  # left rarefaction
                head, tail = ul - cl, us - cs
                if x <= head:
                    h[k], u[k] = hl, ul
                elif x >= tail:
                    h[k], u[k] = hs, us
                else:
                    c = (ul + 2.0 * cl - x) / 3.0
                    h[k], u[k] = c * c / g, (ul + 2.0 * cl + 2.0 * x) / 3.0
        else:
            if hs > hr:  # right shock
                s = ur + cr * math.sqrt(0.5 * (hs + hr) * hs / (hr * hr))
                h[k], u[k] = (hs, us) if x <= s else (hr, ur)
            else:  # right rarefaction
                head, tail = ur + cr, us + cs
                if x >= head:
                    h[k], u[k] = hr, ur
                elif x <= tail:
                    h[k], u[k] = hs, us
                else:
                    c = (-ur + 2.0 * cr + x) / 3.0
                    h[k], u[k] = c * c / g, (ur - 2.0 * cr + 2.0 * x) / 3.0
    return h, u
