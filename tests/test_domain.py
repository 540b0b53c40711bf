"""Rectangular domains padded to the 2^L x 2^L grid (host-side helper) and,
on the oracle, the closed edge the padding makes: the pseudo-2D dam break on
the paper's 50 m x 25 m channel equals the square-domain run row by row."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2206_05761_amd.domain import pad_to_grid


def test_pad_to_grid_places_and_crops():
    rng = np.random.default_rng(2)
    h, qx, qy, z = (rng.uniform(0, 1, (5, 12)) for _ in range(4))
    p = pad_to_grid(h, qx, qy, z)
    assert p.L == 4 and p.h.shape == (16, 16)
    for a, b in ((p.h, h), (p.qx, qx), (p.qy, qy), (p.z, z)):
        assert np.array_equal(p.crop(a), b)
    assert not p.h[5:].any() and not p.h[:, 12:].any()
    assert np.all(p.z[5:] == p.wall_z) and np.all(p.z[:, 12:] == p.wall_z)
    assert p.wall_z >= np.max(z + h) + 1000.0
    assert pad_to_grid(h, qx, qy, z, L=6).h.shape == (64, 64)
    with pytest.raises(ValueError):
        pad_to_grid(h, qx, qy, z, L=3)
    with pytest.raises(ValueError):
        pad_to_grid(h, qx, qy[:4], z)


def test_padded_channel_equals_square_domain_on_the_oracle():
    L = 6
    sq = W.pseudo2d_dambreak(L, t_end=2.5)
    ch = W.pseudo2d_channel(L, t_end=2.5)
    rows = ch.meta["channel_rows"]
    a = O.Oracle(sq.params, sq.h, sq.qx, sq.qy, sq.z)
    b = O.Oracle(ch.params, ch.h, ch.qx, ch.qy, ch.z)
    assert a.run(10_000) == b.run(10_000)
    fa, fb = a.fine(), b.fine()
    assert np.array_equal(fa[0][:rows], fb[0][:rows])
    assert np.array_equal(fa[1][:rows], fb[1][:rows])
    assert np.max(np.abs(fb[2][:rows])) <= 1e-12
    assert not fb[0][rows:].any()
