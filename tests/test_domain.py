"""Rectangular domains and gridded DEMs padded to the 2^L x 2^L grid
(host-side helpers) and, on the oracle, what the padding must preserve: the
closed edge it makes (the pseudo-2D dam break on the paper's 50 m x 25 m
channel equals the square-domain run row by row) and the significance test
inside the domain (the bed's s_max is the domain's own)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2206_05761_amd.domain import bed_smax, dem_domain, pad_to_grid, read_esri_ascii


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
    assert p.zsmax == 1.0 and p.valid.sum() == 60
    assert pad_to_grid(h, qx, qy, 3.0 + z, L=6).zsmax == np.max(3.0 + z)
    assert pad_to_grid(h, qx, qy, z, L=6).h.shape == (64, 64)
    with pytest.raises(ValueError):
        pad_to_grid(h, qx, qy, z, L=3)
    with pytest.raises(ValueError):
        pad_to_grid(h, qx, qy[:4], z)


def test_masked_cells_become_padding():
    rng = np.random.default_rng(3)
    h, qx, qy = (rng.uniform(0, 1, (6, 7)) for _ in range(3))
    z = rng.uniform(-40, 2, (6, 7))
    valid = np.ones((6, 7), dtype=bool)
    valid[2:4, 3:5] = False
    z[2:4, 3:5] = -9999.0          # a NODATA marker must not reach s_max
    p = pad_to_grid(h, qx, qy, z, valid=valid)
    assert p.zsmax == bed_smax(z, valid) == np.abs(z[valid]).max()
    assert np.all(p.z[2:4, 3:5] == p.wall_z) and not p.h[2:4, 3:5].any()
    assert not p.qx[2:4, 3:5].any() and not p.qy[2:4, 3:5].any()
    assert p.valid[:6, :7].sum() == 38 and not p.valid[6:].any()


def _write_esri(path, z_rows_north_first, cellsize, nodata=None, centre=False):
    ny, nx = z_rows_north_first.shape
    with open(path, "w") as fh:
        fh.write(f"ncols {nx}\nnrows {ny}\n")
        if centre:
            fh.write(f"xllcenter {0.5 * cellsize}\nyllcenter {0.5 * cellsize}\n")
        else:
            fh.write("xllcorner 0.0\nyllcorner 0.0\n")
        fh.write(f"cellsize {cellsize}\n")
        if nodata is not None:
            fh.write(f"NODATA_value {nodata}\n")
        for row in z_rows_north_first:
            fh.write(" ".join(repr(float(v)) for v in row) + "\n")


def test_read_esri_ascii_orients_rows_and_masks_nodata(tmp_path):
    z = np.arange(12, dtype=np.float64).reshape(3, 4)   # [j][i], j = 0 south
    file_rows = z[::-1].copy()
    file_rows[0, 1] = -9999.0                          # northern row, column 1
    path = tmp_path / "dem.asc"
    _write_esri(path, file_rows, 2.5, nodata=-9999)
    dem = read_esri_ascii(path)
    assert dem.cellsize == 2.5 and dem.xll == 0.0 and dem.yll == 0.0
    assert dem.z.shape == (3, 4)
    assert not dem.valid[2, 1] and dem.valid.sum() == 11
    assert np.array_equal(dem.z[dem.valid], z[dem.valid])
    _write_esri(tmp_path / "c.asc", z[::-1], 2.0, centre=True)
    dc = read_esri_ascii(tmp_path / "c.asc")
    assert dc.xll == 0.0 and dc.yll == 0.0 and dc.valid.all()
    bad = tmp_path / "bad.asc"
    bad.write_text("ncols 2\nnrows 2\ncellsize 1\n1 2 3\n")
    with pytest.raises(ValueError):
        read_esri_ascii(bad)


def test_padding_keeps_the_significance_test_of_the_domain():
    """A 2^(L-1)-square domain padded to level L is the subtree of the
    root's first child: with the domain's own bed s_max its bed flags there
    equal those of the unpadded domain, level for level (Section 2.1.2's
    s_max is the domain's largest finest coefficient).  Normalising by the
    padded grid's largest bed instead changes them."""
    L = 6
    z = W.gaussian_bumps(L - 1, 1.0, 6, seed=4, amp=(0.5, 2.0))
    zero = np.zeros_like(z)
    p_dom = W.base_params(L - 1, 1.0, 1e-2)
    o_dom = O.Oracle(p_dom, zero, zero, zero, z)
    pad = pad_to_grid(zero, zero, zero, z, L=L)
    p_pad = W.base_params(L, 2.0, 1e-2, zsmax=pad.zsmax)
    o_pad = O.Oracle(p_pad, pad.h, pad.qx, pad.qy, pad.z)
    assert o_pad.scalars()["smax_z"] == o_dom.scalars()["smax_z"] == pad.zsmax
    f_dom, f_pad = o_dom.flags("zraw"), o_pad.flags("zraw")
    off = lambda n: (4 ** n - 1) // 3
    for n in range(L - 1):
        cnt = 4 ** n
        # level n of the domain is level n + 1 of the padded grid, first quarter
        assert np.array_equal(f_pad[off(n + 1):off(n + 1) + cnt], f_dom[off(n):off(n) + cnt]), n
    o_big = O.Oracle(dict(p_pad, zsmax=0.0), pad.h, pad.qx, pad.qy, pad.z)
    assert o_big.scalars()["smax_z"] == pad.wall_z
    f_big = o_big.flags("zraw")
    assert any(not np.array_equal(f_big[off(n + 1):off(n + 1) + 4 ** n], f_dom[off(n):off(n) + 4 ** n])
               for n in range(L - 1))


def test_dem_with_nodata_runs_closed_on_the_oracle(tmp_path):
    """A DEM file with a NODATA hole and a ragged NODATA edge: the masked
    cells stay dry and closed, no water leaves the walled domain."""
    dem_file = tmp_path / "valley.asc"
    ny, nx = 25, 40
    x = (np.arange(nx) + 0.5)[None, :]
    y = (np.arange(ny) + 0.5)[:, None]
    z = 0.02 * x + 0.05 * (y - 12.5) ** 2 / 12.5
    z = np.broadcast_to(z, (ny, nx)).copy()
    mask = np.ones((ny, nx), dtype=bool)
    mask[10:14, 18:22] = False                       # a hole
    mask[:, 36:] = (y[:, 0, None] < 6) | (y[:, 0, None] > 19)   # ragged east end
    rows = np.where(mask, z, -9999.0)[::-1]
    _write_esri(dem_file, rows, 1.0, nodata=-9999)
    dem = read_esri_ascii(dem_file)
    assert np.array_equal(dem.valid, mask)
    h = np.where(x < 10.0, np.maximum(0.0, 1.0 - dem.z), 0.0) * dem.valid
    pad = dem_domain(dem, h=h)
    assert pad.L == 6 and pad.zsmax == bed_smax(z, mask)
    p = W.base_params(pad.L, (1 << pad.L) * dem.cellsize, 1e-3, zsmax=pad.zsmax, t_end=2.0)
    o = O.Oracle(p, pad.h, pad.qx, pad.qy, pad.z)
    m0 = o.scalars()["mass"]
    o.run(100_000)
    hh, qx, qy = o.fine()
    assert o.scalars()["t"] == 2.0
    assert not hh[~pad.valid].any() and not qx[~pad.valid].any() and not qy[~pad.valid].any()
    assert abs(o.scalars()["mass"] - m0) <= 1e-10 * m0
    assert hh[pad.valid].max() > 0.0


def test_padded_channel_equals_square_domain_on_the_oracle():
    L = 6
    sq = W.pseudo2d_dambreak(L, t_end=2.5)
    ch = W.pseudo2d_channel(L, t_end=2.5)
    rows = ch.meta["channel_rows"]
    assert ch.params["zsmax"] == 1.0
    a = O.Oracle(sq.params, sq.h, sq.qx, sq.qy, sq.z)
    b = O.Oracle(ch.params, ch.h, ch.qx, ch.qy, ch.z)
    assert a.run(10_000) == b.run(10_000)
    fa, fb = a.fine(), b.fine()
    assert np.array_equal(fa[0][:rows], fb[0][:rows])
    assert np.array_equal(fa[1][:rows], fb[1][:rows])
    assert np.max(np.abs(fb[2][:rows])) <= 1e-12
    assert not fb[0][rows:].any()
