"""Pins of the oracle's FV1 operator and time loop: flux consistency and
symmetry, eps = 0 equals uniform-grid FV1, lake at rest (well-balancing),
mass conservation, exact 1D dam-break solutions, Manning friction against its
ODE, rain, inflow volume, and bitwise checkpoint/resume."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from exact_riemann import sample, star_state

G = 9.80665


# --------------------------------------------------------------------------
# Face flux
# --------------------------------------------------------------------------
def _phys_flux(h, qn, qt):
    u = qn / h
    return np.array([qn, qn * u + 0.5 * G * h * h, qn * qt / h])


def test_flux_consistency_equal_states_flat_bed():
    p = W.base_params(4, 1.0, 0.0)
    for h, qn, qt in [(1.0, 0.3, -0.2), (2.5, -1.0, 0.7), (0.01, 0.0, 0.0)]:
        s = [h, qn, qt, 0.0]
        F, hs = O.face_flux(p, s, s)
        assert np.allclose(F, _phys_flux(h, qn, qt), rtol=1e-14, atol=1e-15)
        assert hs[0] == h and hs[1] == h


def test_flux_supersonic_upwinding():
    p = W.base_params(4, 1.0, 0.0)
    left = [1.0, 10.0, 0.5, 0.0]     # u = 10 > c: all waves go right
    right = [0.5, 5.5, 0.0, 0.0]
    F, _ = O.face_flux(p, left, right)
    assert np.allclose(F, _phys_flux(1.0, 10.0, 0.5), rtol=1e-14)
    F2, _ = O.face_flux(p, [0.5, -6.0, 0.0, 0.0], [1.0, -10.0, 0.2, 0.0])
    assert np.allclose(F2, _phys_flux(1.0, -10.0, 0.2), rtol=1e-14)


def test_flux_mirror_symmetry():
    """Reflecting x -> -x swaps the states and negates normal velocities:
    mass flux and tangential flux change sign, momentum flux does not."""
    p = W.base_params(4, 1.0, 0.0)
    rng = np.random.default_rng(1)
    for _ in range(100):
        hl, hr = rng.uniform(0.1, 3.0, 2)
        ql, qr, tl, tr = rng.uniform(-2, 2, 4)
        zl, zr = rng.uniform(-0.5, 0.5, 2)
        F, hs = O.face_flux(p, [hl, ql, tl, zl], [hr, qr, tr, zr])
        Fm, hsm = O.face_flux(p, [hr, -qr, tr, zr], [hl, -ql, tl, zl])
        assert Fm[0] == pytest.approx(-F[0], rel=1e-12, abs=1e-13)
        assert Fm[1] == pytest.approx(F[1], rel=1e-12, abs=1e-13)
        assert Fm[2] == pytest.approx(-F[2], rel=1e-12, abs=1e-13)
        assert hsm[0] == hs[1] and hsm[1] == hs[0]


def test_flux_dry_both_sides_and_step_reconstruction():
    p = W.base_params(4, 1.0, 0.0)
    F, hs = O.face_flux(p, [0.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0])
    assert np.all(F == 0.0) and np.all(hs == 0.0)
    # still water at eta = 1 against a bed step from 0.2 to 0.5: both
    # reconstructed depths equal eta - max(z) = 0.5, velocity zero
    F, hs = O.face_flux(p, [0.8, 0.0, 0.0, 0.2], [0.5, 0.0, 0.0, 0.5])
    assert hs[0] == pytest.approx(0.5, abs=1e-15)
    assert hs[1] == pytest.approx(0.5, abs=1e-15)
    assert F[0] == 0.0
    assert F[1] == pytest.approx(0.5 * G * 0.25, rel=1e-14)
    # bed step above the water: the wet side's face depth is zero
    F, hs = O.face_flux(p, [0.3, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.6])
    assert hs[0] == 0.0 and hs[1] == 0.0 and np.all(F == 0.0)


# --------------------------------------------------------------------------
# eps = 0 reduces to uniform FV1 (bitwise)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("maker", ["bumps", "circular"])
def test_eps_zero_equals_uniform_fv1(maker):
    if maker == "bumps":
        w = W.dambreak_bumps_l6(L=5)
        steps = 20
    else:
        w = W.circular_dambreak_l10(L=6)
        steps = 30
    p = dict(w.params, eps=0.0, t_end=math.inf)
    a = O.Oracle(p, w.h, w.qx, w.qy, w.z)
    b = O.Oracle(p, w.h, w.qx, w.qy, w.z)
    for _ in range(steps):
        assert a.step()
        b.uniform_fv1_step()
        for x, y in zip(a.fine(), b.fine()):
            assert np.array_equal(x, y)
        sa, sb = a.scalars(), b.scalars()
        assert sa["t"] == sb["t"] and sa["dt"] == sb["dt"]


# --------------------------------------------------------------------------
# Well-balancing: lake at rest (Section 3.1 property)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("eta,eps", [(1.0, 1e-3), (1.0, 1e-2), (0.45, 0.0)])
def test_lake_at_rest_stays_at_rest(eta, eps):
    """All wet (eta = 1 above bumps up to 0.6 m) at eps > 0, and with dry
    islands (eta = 0.45) at eps = 0: discharges stay at round-off."""
    L = 5
    w = W.lake_at_rest(L, eta, 11, eps)
    if eta < 0.6:
        assert (w.h == 0).any()
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    o.step()
    # after the first step the finest depth under a coarse leaf is the leaf
    # average (copy-down); from then on nothing may move
    h1, _, _ = o.fine()
    if eps == 0.0:
        assert np.abs(h1 - w.h).max() <= 1e-13
    o.run(999)
    h, qx, qy = o.fine()
    assert max(np.abs(qx).max(), np.abs(qy).max()) <= 1e-10
    assert np.abs(h - h1).max() <= 1e-10
    # the free surface of every leaf is the lake level
    o.phase_encode()
    hh, zz = o.hierarchy("h"), o.hierarchy("z")
    leaves = o.leaves()
    wet = hh[leaves] > 0
    assert np.abs(hh[leaves][wet] + zz[leaves][wet] - eta).max() <= 1e-12


# --------------------------------------------------------------------------
# Mass
# --------------------------------------------------------------------------
def test_mass_conserved_closed_walls_eps0():
    w = W.dambreak_bumps_l6(L=5)
    p = dict(w.params, eps=0.0)
    o = O.Oracle(p, w.h, w.qx, w.qy, w.z)
    m0 = o.scalars()["mass"]
    o.run(200)
    h, _, _ = o.fine()
    m1 = h.sum() * p["dx"] * p["dy"]
    assert abs(m1 - m0) / m0 <= 1e-12
    assert abs(o.scalars()["mass"] - m0) / m0 <= 1e-12


def test_mass_drift_at_level_jumps_is_small():
    """At eps > 0 the same-level neighbour rule is not conservative at
    level jumps; the drift stays at the level of eps."""
    w = W.dambreak_bumps_l6()
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    m0 = o.scalars()["mass"]
    o.run(10_000)
    assert abs(o.scalars()["mass"] - m0) / m0 <= 1e-4


# --------------------------------------------------------------------------
# 1D dam breaks against the exact Riemann solution
# --------------------------------------------------------------------------
def _strip_error(L, hl, hr, eps, axis="x", t_end=2.5):
    length, x_dam = 50.0, 10.0
    w = W.dambreak_strip(L, hl, hr, x_dam, length, eps, t_end, axis=axis)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    o.run(100_000)
    assert o.scalars()["t"] == pytest.approx(t_end, abs=1e-12)
    h, qx, qy = o.fine()
    n = 1 << L
    xc = (np.arange(n) + 0.5) * (length / n)
    he, ue = sample(hl, 0.0, hr, 0.0, G, (xc - x_dam) / t_end)
    prof = h[n // 2, :] if axis == "x" else h[:, n // 2]
    l1 = np.mean(np.abs(prof - he))
    return l1, h, qx, qy


def test_exact_riemann_helper_rankine_hugoniot():
    hl, hr = 6.0, 2.0
    hs, us = star_state(hl, 0.0, hr, 0.0, G)
    s = us * hs / (hs - hr)   # mass jump condition across the right shock
    mom = (hs * us * us + 0.5 * G * hs * hs - 0.5 * G * hr * hr) / (hs * us)
    assert s == pytest.approx(mom, rel=1e-12)
    # left rarefaction: Riemann invariant u + 2c conserved
    assert us + 2 * math.sqrt(G * hs) == pytest.approx(2 * math.sqrt(G * hl))


@pytest.mark.parametrize("hr", [2.0, 0.0])
def test_dambreak_converges_to_exact_solution(hr):
    errs = []
    for L in (6, 7, 8):
        l1, h, qx, qy = _strip_error(L, 6.0, hr, 0.0)
        errs.append(l1)
        # flow is one-dimensional: no transverse discharge
        assert np.abs(qy).max() <= 1e-12
    assert errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[2] / 6.0 <= 1e-2
    # first order: error roughly halves per level (loosely)
    assert errs[2] <= 0.75 * errs[0]


def test_dambreak_along_y_is_transpose_of_x():
    """Same problem along y: h is transposed and qx/qy trade places."""
    L = 6
    _, hx, qxx, qyx = _strip_error(L, 6.0, 2.0, 1e-3, axis="x", t_end=1.0)
    _, hy, qxy, qyy = _strip_error(L, 6.0, 2.0, 1e-3, axis="y", t_end=1.0)
    assert np.allclose(hy, hx.T, rtol=0, atol=1e-12)
    assert np.allclose(qyy, qxx.T, rtol=0, atol=1e-12)
    assert np.allclose(qxy, qyx.T, rtol=0, atol=1e-12)


def _leaf_levels(leaves):
    return np.floor(np.log(3.0 * leaves.astype(np.float64) + 1.0)
                    / np.log(4.0) + 1e-9).astype(int)


def test_adaptive_dambreak_keeps_fidelity_of_its_finest_level():
    """With details zeroed below leaves and neighbour-only regularisation,
    the adaptive grid never refines past the finest level present in the
    data (here the dam sits on a level-6 cell boundary, so level 6).  The
    adaptive answer then matches uniform FV1 at that level: its error
    against the exact solution is within 25 % of the uniform one."""
    L = 7
    w = W.dambreak_strip(L, 6.0, 2.0, 10.0, 50.0, 1e-3, 2.5)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    o.run(100_000)
    top = int(_leaf_levels(o.leaves()).max())
    assert top == L - 1
    l1_a, _, _, _ = _strip_error(L, 6.0, 2.0, 1e-3)
    l1_u, _, _, _ = _strip_error(top, 6.0, 2.0, 0.0)
    assert l1_a <= 1.25 * l1_u


def test_circular_dambreak_mirror_symmetry():
    """A centred circular dam break over a flat bed stays symmetric under
    x -> -x reflection (h even, qx odd) to round-off."""
    L = 5
    p = W.base_params(L, 40.0, 1e-3, bc=("wall",) * 4)
    x, y = W.cell_centres(L, 40.0)
    r = np.sqrt((x - 20.0) ** 2 + (y - 20.0) ** 2)
    h = np.where(r < 8.0, 2.5, 0.5)
    zero = np.zeros_like(h)
    o = O.Oracle(p, h, zero, zero, zero)
    o.run(60)
    h1, qx1, qy1 = o.fine()
    assert np.allclose(h1, h1[:, ::-1], rtol=0, atol=1e-11)
    assert np.allclose(qx1, -qx1[:, ::-1], rtol=0, atol=1e-11)
    assert np.allclose(qy1, qy1[:, ::-1], rtol=0, atol=1e-11)
    assert np.allclose(h1, h1.T, rtol=0, atol=1e-11)
    assert np.allclose(qx1, qy1.T, rtol=0, atol=1e-11)


# --------------------------------------------------------------------------
# Sources
# --------------------------------------------------------------------------
def test_manning_friction_follows_its_ode():
    """Uniform sheet on a flat bed with open boundaries: no flux divergence,
    so the discharge obeys dq/dt = -g n^2 q|q| / h^(7/3) (Eq. 1 with
    C_f = g n^2 / h^(1/3)), whose solution is q0 / (1 + k q0 t)."""
    L = 3
    h0, q0, n_m = 0.5, 0.4, 0.03
    p = W.base_params(L, 100.0, 1e-3, manning_n=n_m, bc=("open",) * 4,
                      cfl=0.05)
    h = np.full((8, 8), h0)
    qx = np.full((8, 8), q0)
    zero = np.zeros_like(h)
    o = O.Oracle(p, h, qx, zero, zero)
    o.run(400)
    t = o.scalars()["t"]
    hh, qq, qy = o.fine()
    assert np.all(hh == h0) and np.all(qy == 0)
    k = G * n_m ** 2 / h0 ** (7.0 / 3.0)
    exact = q0 / (1.0 + k * q0 * t)
    # first-order implicit scheme: relative error O(dt k q0) per unit time
    assert qq[0, 0] == pytest.approx(exact, rel=2e-3)
    assert np.all(qq == qq[0, 0])


def test_rain_fills_closed_lake_linearly():
    L = 4
    R = 1e-4
    p = W.base_params(L, 10.0, 1e-3, rain_rate=R)
    h0 = 0.3
    h = np.full((16, 16), h0)
    zero = np.zeros_like(h)
    o = O.Oracle(p, h, zero, zero, zero)
    o.run(100)
    t = o.scalars()["t"]
    hh, qx, qy = o.fine()
    assert np.allclose(hh, h0 + R * t, rtol=1e-12, atol=0)
    assert np.abs(qx).max() == 0.0 and np.abs(qy).max() == 0.0
    assert o.scalars()["mass"] == pytest.approx((h0 + R * t) * 100.0, rel=1e-12)


def test_inflow_volume_matches_hydrograph_integral():
    """Closed box, flat bed, west-edge inflow: the stored volume equals the
    integral of the triangular hydrograph, up to the left-Riemann-sum error
    of the explicit source."""
    L = 5
    length = 100.0
    qp, tp, tb = 2.0, 20.0, 40.0
    p = W.base_params(L, length, 1e-3, inlet_y0=40.0, inlet_y1=60.0,
                      q_peak=qp, t_peak=tp, t_base=tb, t_end=50.0,
                      bc=("wall",) * 4)
    zero = np.zeros((1 << L, 1 << L))
    o = O.Oracle(p, zero, zero, zero, zero)
    n = o.run(100_000)
    t = o.scalars()["t"]
    assert t == pytest.approx(50.0, abs=1e-9)
    vol = qp * tb / 2.0
    h, _, _ = o.fine()
    stored = h.sum() * p["dx"] * p["dy"]
    # |error| <= sum over steps of dt^2 |Q'| / 2 <= t * dt_max * |Q'| / 2
    bound = t * p["dt_max"] * (qp / tp) / 2.0 + 1e-9
    assert abs(stored - vol) <= bound
    assert n > 10


def test_hydrograph_workload_stores_the_delivered_volume():
    """The hydrograph workload (closed inflow edge, other edges open) at a
    small L: while no water has reached an open edge the stored volume is
    the delivered hydrograph volume, within the left-Riemann-sum error of
    the explicit source (the rising limb is under-counted, never over)."""
    w = W.hydrograph_l12(L=7)
    p = dict(w.params, t_end=1500.0)
    o = O.Oracle(p, w.h, w.qx, w.qy, w.z)
    o.run(100_000)
    s = o.scalars()
    t = s["t"]
    assert t == 1500.0
    delivered = 0.5 * w.params["q_peak"] * t * t / w.params["t_peak"]
    bound = t * w.params["dt_max"] * (w.params["q_peak"] / w.params["t_peak"]) / 2
    assert delivered - bound <= s["mass"] <= delivered * (1 + 1e-12)
    assert s["clips"] == 0


# --------------------------------------------------------------------------
# Timestep and checkpoint/resume
# --------------------------------------------------------------------------
def test_first_timestep_cfl_of_still_water():
    L = 4
    p = W.base_params(L, 1.0, 1e-3)
    h = np.full((16, 16), 2.0)
    zero = np.zeros_like(h)
    o = O.Oracle(p, h, zero, zero, zero)
    assert o.scalars()["dt"] == pytest.approx(
        0.5 * (1.0 / 16) / math.sqrt(G * 2.0), rel=1e-15)


def test_t_end_is_hit_exactly_and_run_stops():
    w = W.dambreak_bumps_l6(L=5)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    n = o.run(100_000)
    assert o.scalars()["t"] == 0.05
    assert not o.step()
    assert n == o.scalars()["step"]


def test_checkpoint_resume_is_bitwise():
    w = W.circular_dambreak_l10(L=6)
    a = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    a.run(40)
    ref = a.fine()
    b = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    b.run(17)
    s = b.scalars()
    h, qx, qy = b.fine()
    c = O.Oracle(w.params, h, qx, qy, w.z)
    c.set_time(s["t"], s["dt"], int(s["step"]))
    c.run(23)
    for x, y in zip(ref, c.fine()):
        assert np.array_equal(x, y)
    assert c.scalars()["t"] == a.scalars()["t"]
