"""GPU: a rectangular domain padded to the 2^L x 2^L grid with dry high
ground (the paper's 50 m x 25 m pseudo-2D channel) against the oracle, and
against the square-domain run, whose rows carry the same flow.  FP64 bar:
1e-10 max-abs, identical leaf lists."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_utils import compare_leaf_lists, oracle_tie_band

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2206_05761_amd as hw
    return hw


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def test_padded_channel_matches_oracle_and_square_domain(hw):
    L = 7
    ch = W.pseudo2d_channel(L, t_end=2.5)
    rows = ch.meta["channel_rows"]
    sim = hw.Simulation(ch.params, ch.h, ch.qx, ch.qy, ch.z)
    st = sim.run(100_000)
    o = O.Oracle(ch.params, ch.h, ch.qx, ch.qy, ch.z)
    n = o.run(100_000)
    print("  channel steps", st["steps"], n, "leaves", o.scalars()["n_leaves"], flush=True)
    sys.stdout.flush()
    assert st["steps"] == n and st["t"] == 2.5
    f = sim.export()
    fo = o.fine()
    assert max(_max_abs(x, y) for x, y in zip(f, fo)) <= 1e-10
    compare_leaf_lists(L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    assert not f[0][rows:].any()
    sq = W.pseudo2d_dambreak(L, t_end=2.5)
    ssim = hw.Simulation(sq.params, sq.h, sq.qx, sq.qy, sq.z)
    ssim.run(100_000)
    fs = ssim.export()
    assert _max_abs(f[0][:rows], fs[0][:rows]) <= 1e-12
    assert _max_abs(f[1][:rows], fs[1][:rows]) <= 1e-12
    sim.close()
    ssim.close()
    u = hw.Simulation(ch.params, ch.h, ch.qx, ch.qy, ch.z)
    plan = hw.Plan([u.problem], [u.buffers], uniform=True)
    hw.hwfv1_run(u.problem, u.buffers, 100_000, plan=plan)
    plan.close()
    ou = O.Oracle(ch.params, ch.h, ch.qx, ch.qy, ch.z)
    while ou.scalars()["t"] < 2.5:
        ou.uniform_fv1_step()
    assert max(_max_abs(x, y) for x, y in zip(u.export(), ou.fine())) <= 1e-10
    u.close()


def test_dem_with_nodata_matches_oracle(hw, tmp_path):
    """A gridded DEM (ESRI ASCII, written here) with a NODATA hole and a
    ragged NODATA edge, padded to the square grid with the domain's own bed
    s_max: GPU against the oracle, masked cells dry and closed."""
    from paper_2206_05761_amd.domain import dem_domain, read_esri_ascii
    from parity_utils import compare_leaf_lists, oracle_tie_band
    ny, nx = 100, 160
    x = (np.arange(nx) + 0.5)[None, :]
    y = (np.arange(ny) + 0.5)[:, None]
    z = np.broadcast_to(0.005 * x + 0.2 * ((y - 50.0) / 50.0) ** 2
                        + 0.3 * np.exp(-((x - 90.0) ** 2 + (y - 40.0) ** 2) / 60.0),
                        (ny, nx)).copy()
    mask = np.ones((ny, nx), dtype=bool)
    mask[40:56, 70:86] = False
    mask[:, 140:] = ((y < 30) | (y > 70))[:, :1] * np.ones((1, 20), dtype=bool)
    path = tmp_path / "dem.asc"
    with open(path, "w") as fh:
        fh.write(f"ncols {nx}\nnrows {ny}\nxllcorner 0\nyllcorner 0\ncellsize 0.5\n"
                 "NODATA_value -9999\n")
        for row in np.where(mask, z, -9999.0)[::-1]:
            fh.write(" ".join(repr(float(v)) for v in row) + "\n")
    dem = read_esri_ascii(path)
    h = np.where(x < 30.0, np.maximum(0.0, 0.8 - dem.z), 0.0) * dem.valid
    pad = dem_domain(dem, h=h)
    p = dict(W.base_params(pad.L, (1 << pad.L) * dem.cellsize, 1e-3, zsmax=pad.zsmax,
                           manning_n=0.02), t_end=1.5)
    sim = hw.Simulation(p, pad.h, pad.qx, pad.qy, pad.z)
    st = sim.run(100_000)
    o = O.Oracle(p, pad.h, pad.qx, pad.qy, pad.z)
    n = o.run(100_000)
    log("  DEM L", pad.L, "steps", st["steps"], n, "leaves", o.scalars()["n_leaves"],
        "zsmax", pad.zsmax, "smax_z", sim.scalars()["smax"][3])
    assert st["steps"] == n and st["t"] == 1.5
    assert sim.scalars()["smax"][3] == o.scalars()["smax_z"] == pad.zsmax
    f = sim.export()
    assert max(_max_abs(a, b) for a, b in zip(f, o.fine())) <= 1e-10
    compare_leaf_lists(pad.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    assert not f[0][~pad.valid].any() and not f[1][~pad.valid].any()
    sim.close()
