"""Pins of the oracle's multiresolution analysis: indexing, Haar encoding and
decoding, the significance test, regularisation and the depth-first leaf
list.  Every check compares the oracle with something fixed by the paper or by
mathematics, never with a retyping of the oracle's own formulas."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from conftest import golden


# --------------------------------------------------------------------------
# Z-order indexing (Section 2.2.1, Fig. 5, footnote 2)
# --------------------------------------------------------------------------
def test_morton_matches_fig5_table():
    table = golden("fig5_morton_4x4.txt")["rows"]
    for j in range(4):
        for i in range(4):
            assert O.morton(i, j) == table[j][i]


def test_footnote_zindex_example():
    g = golden("traversal_l2_example.txt")
    assert g["footnote_zindex"] == "L=2 morton=3 index=8"
    # finest cell with Morton code 3 at L = 2 is (i, j) = (1, 1)
    assert O.morton(1, 1) == 3
    assert O.zindex(2, 1, 1) == 8


def test_zindex_levels_are_contiguous_and_disjoint():
    L = 4
    seen = set()
    for n in range(L + 1):
        s = 1 << n
        idx = sorted(O.zindex(n, i, j) for j in range(s) for i in range(s))
        start = sum(4 ** k for k in range(n))
        assert idx == list(range(start, start + s * s))
        seen.update(idx)
    assert len(seen) == (4 ** (L + 1) - 1) // 3


# --------------------------------------------------------------------------
# Haar encoding / decoding (Eq. 3a-3d, Eq. 4a-4d)
# --------------------------------------------------------------------------
def test_haar_parent_is_average_and_decode_inverts():
    rng = np.random.default_rng(0)
    for _ in range(200):
        s = rng.integers(-2**20, 2**20, size=4).astype(np.float64)
        c = O.haar_encode(s)
        # parent is the mean of the children (averaging normalisation)
        assert c[0] == s.sum() / 4.0
        # decoding reproduces the children exactly on small integers
        assert np.array_equal(O.haar_decode(c), s)


def test_haar_details_orientation():
    """Children are ordered (c & 1, c >> 1): a field varying only in x has
    only a beta detail, one varying only in y only an alpha detail, and the
    product x*y only a gamma detail (with the closed-form values)."""
    dx = dy = 0.5
    x0, y0 = 3.0, -2.0
    pos = [(x0, y0), (x0 + dx, y0), (x0, y0 + dy), (x0 + dx, y0 + dy)]
    a, b, cc = 1.75, -0.625, 2.5
    fx = np.array([a * x for x, _ in pos])
    fy = np.array([b * y for _, y in pos])
    fxy = np.array([cc * x * y for x, y in pos])
    ex = O.haar_encode(fx)
    assert ex[1] == 0.0 and ex[3] == 0.0
    assert ex[2] == -a * dx / 2.0
    ey = O.haar_encode(fy)
    assert ey[2] == 0.0 and ey[3] == 0.0
    assert ey[1] == -b * dy / 2.0
    exy = O.haar_encode(fxy)
    assert exy[3] == pytest.approx(cc * dx * dy / 4.0, rel=1e-15)


@pytest.mark.parametrize("L", [1, 3, 6])
def test_roundtrip_exact_on_dyadic_field(L):
    rng = np.random.default_rng(L)
    f = rng.integers(-2**18, 2**18, size=(1 << L, 1 << L)).astype(np.float64)
    assert np.array_equal(O.roundtrip(L, f), f)


def test_roundtrip_random_within_rounding():
    L = 7
    rng = np.random.default_rng(7)
    f = rng.standard_normal((1 << L, 1 << L)) * 10.0
    out = O.roundtrip(L, f)
    assert np.max(np.abs(out - f)) <= 8 * L * np.finfo(float).eps * np.abs(f).max()


def _ramp_oracle(L, a, b, eps, length=1.0):
    """Static bed z = a*x + b*y (sampled at cell centres), still water."""
    p = W.base_params(L, length, eps)
    x, y = W.cell_centres(L, length)
    z = a * x + b * y
    h = np.full_like(z, 1.0)
    zero = np.zeros_like(z)
    o = O.Oracle(p, h, zero, zero, z)
    return o, p, z


def test_linear_ramp_hierarchy_is_cell_centre_value():
    """Cell averages of a linear function equal its value at the cell
    centre, on every level."""
    L = 5
    a, b = 0.75, -0.5
    o, p, _ = _ramp_oracle(L, a, b, 1e-3)
    z = o.hierarchy("z")
    for n in range(L + 1):
        s = 1 << n
        d = 1.0 / s
        for j in range(s):
            for i in range(s):
                want = a * (i + 0.5) * d + b * (j + 0.5) * d
                got = z[O.zindex(n, i, j)]
                assert abs(got - want) <= 8 * np.finfo(float).eps * 2.0


def test_linear_ramp_details_closed_form():
    L = 5
    a, b = 0.75, -0.5
    o, p, _ = _ramp_oracle(L, a, b, 1e-3)
    o.phase_encode()
    d = o.details("z")
    for n in range(L):
        s = 1 << n
        child = 1.0 / (2 * s)   # level n+1 cell width
        for j in range(s):
            for i in range(s):
                k = O.zindex(n, i, j)
                assert d[0, k] == pytest.approx(-b * child / 2, abs=1e-14)
                assert d[1, k] == pytest.approx(-a * child / 2, abs=1e-14)
                assert abs(d[2, k]) <= 1e-14


def test_linear_ramp_leaf_level_closed_form():
    """For z = a*x the normalised detail of level n is a/(2^(n+2) s_max) and
    the threshold 2^(n-L) eps, so every level n <= n* is significant where
    4^n* <= a 2^L / (4 s_max eps) < 4^(n*+1); the leaves form the uniform grid
    of level n* + 1."""
    L = 7
    a = 0.9              # s_max(z) = 1 (guard) because |z| < 1
    for eps in (1e-1, 2e-2, 3e-3):
        o, p, _ = _ramp_oracle(L, a, 0.0, eps)
        o.step()
        ratio = a * 2**L / (4 * 1.0 * eps)
        nstar = int(np.floor(np.log(ratio) / np.log(4.0)))
        nstar = min(nstar, L - 1)
        leaf_level = nstar + 1
        leaves = o.leaves()
        assert len(leaves) == 4 ** leaf_level
        start = (4 ** leaf_level - 1) // 3
        assert np.array_equal(leaves, np.arange(start, start + 4 ** leaf_level))


def _uniform_leaf_level(L, ratio):
    """Leaf level of a field whose level-n normalised detail is
    a / (2^(n+2) s_max) against the threshold 2^(n-L) eps: every level n
    with 4^n <= ratio = a 2^L / (4 s_max eps) is significant."""
    nstar = int(np.floor(np.log(ratio) / np.log(4.0)))
    return min(nstar, L - 1) + 1


def _assert_uniform_leaves(leaves, level):
    start = (4 ** level - 1) // 3
    assert np.array_equal(leaves, np.arange(start, start + 4 ** level)), (
        f"expected the uniform grid of level {level}, got {len(leaves)} leaves")


def test_smax_of_the_bed_is_its_largest_finest_magnitude():
    """Section 2.1.2 normalises by the largest coefficient of the finest
    level.  A falling bed z = -(a x + c) with a = 3, c = 2 has
    max |z^(L)| = a (1 - 2^-(L+1)) + c (the last cell centre), well above
    the guard of 1; eps is chosen so that the closed-form leaf level with
    that s_max differs from the one obtained with the guard value (s_max
    = 1, as a dropped abs would give for this negative bed) and with the
    root's magnitude (a coarse-level normaliser)."""
    L, a, c = 7, 3.0, 2.0
    smax = a * (1.0 - 2.0 ** -(L + 1)) + c
    eps = a * 2 ** L / (4.0 * smax * (3.2 * 4 ** 3))   # ratio 204.8: level 4
    p = W.base_params(L, 1.0, eps)
    x, _ = W.cell_centres(L, 1.0)
    z = -(a * x + c)
    one = np.ones_like(z)
    zero = np.zeros_like(z)
    o = O.Oracle(p, one, zero, zero, z)
    assert o.scalars()["smax_z"] == smax
    o.phase_encode()
    o.phase_regularise()
    o.phase_traverse()
    ratio = a * 2 ** L / (4.0 * smax * eps)
    level = _uniform_leaf_level(L, ratio)
    assert level == 4
    # the misreadings give another level on this field
    assert _uniform_leaf_level(L, a * 2 ** L / (4.0 * 1.0 * eps)) != level
    assert _uniform_leaf_level(L, a * 2 ** L / (4.0 * (a * 0.5 + c) * eps)) != level
    _assert_uniform_leaves(o.leaves(), level)


def test_smax_of_the_depth_is_taken_again_every_step():
    """s_max of a flow variable is the largest finest magnitude at the start
    of each step.  A depth ramp h = 1 + a x (a = 3) on a flat closed basin
    with tiny gravity (so fluxes change it by less than 1e-5) and heavy
    rain: the first step refines to the closed-form level for
    s_max = 1 + a (1 - 2^-(L+1)); the rain then adds R dt = 10 m to every
    cell (details unchanged), s_max grows to the largest level-4 average
    plus 10 and the second step's tree is one level coarser.  An s_max
    kept from the first step, or the guard value, gives other levels."""
    L, a = 7, 3.0
    smax1 = 1.0 + a * (1.0 - 2.0 ** -(L + 1))
    eps = a * 2 ** L / (4.0 * smax1 * (3.0 * 4 ** 3))   # ratio 192: level 4
    p = W.base_params(L, 1.0, eps, g=1e-12, dt_max=1.0, rain_rate=10.0)
    x, _ = W.cell_centres(L, 1.0)
    h = 1.0 + a * x
    zero = np.zeros_like(h)
    o = O.Oracle(p, h, zero, zero.copy(), zero.copy())
    assert o.scalars()["dt"] == 1.0
    assert o.step()
    level1 = _uniform_leaf_level(L, a * 2 ** L / (4.0 * smax1 * eps))
    assert level1 == 4
    _assert_uniform_leaves(o.leaves(), level1)
    assert o.scalars()["smax_h"] == smax1
    # after the step: piecewise constant on level 4, plus the rain
    smax2 = 1.0 + a * (1.0 - 2.0 ** -5) + 10.0
    assert o.step()
    assert o.scalars()["smax_h"] == pytest.approx(smax2, rel=1e-6)
    level2 = _uniform_leaf_level(L, a * 2 ** L / (4.0 * smax2 * eps))
    assert level2 == 3
    _assert_uniform_leaves(o.leaves(), level2)
    # the normaliser of the first step, or the guard, would keep level 4 or more
    assert _uniform_leaf_level(L, a * 2 ** L / (4.0 * smax1 * eps)) != level2
    assert _uniform_leaf_level(L, a * 2 ** L / (4.0 * 1.0 * eps)) != level2


def test_eps_zero_gives_all_finest_leaves_and_constant_gives_root():
    L = 4
    w = W.lake_at_rest(L, 0.8, 3, eps=0.0)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    o.step()
    start = (4 ** L - 1) // 3
    assert np.array_equal(o.leaves(), np.arange(start, start + 4 ** L))
    # constant field, no bed: every detail is zero, the root is the only leaf
    p = W.base_params(L, 1.0, 1e-3)
    one = np.ones((1 << L, 1 << L))
    zero = np.zeros_like(one)
    o2 = O.Oracle(p, one, zero, zero, zero)
    o2.step()
    assert list(o2.leaves()) == [0]


def test_threshold_is_inclusive():
    """Algorithm 1 flags d_norm >= 2^(n-L) eps: a detail exactly on the
    threshold is significant."""
    L = 2
    p = W.base_params(L, 1.0, 0.25)
    # bed with a single x-jump inside the finest level-1 cell (0,0):
    # z of children (0,0),(1,0),(0,1),(1,1) = 0, 0.5, 0, 0.5 gives
    # |d_beta| = 0.25 on level 1 -> normalised 0.25, threshold 2^-1*0.25.
    z = np.zeros((4, 4))
    z[:, 1] = 0.5
    z[:, 3] = 0.5
    # level 1 threshold = 0.125 < 0.25: significant; level 0: details of the
    # level-1 averages (0.25 everywhere) are zero -> not significant.
    zero = np.zeros_like(z)
    o = O.Oracle(p, np.ones_like(z), zero, zero, z)
    o.phase_encode()
    raw = o.flags("raw")
    assert raw[0] == 0 and all(raw[1:5] == 1)
    # now put the detail exactly on the threshold of level 1: eps such that
    # 2^(1-2) eps = 0.25  ->  eps = 0.5
    p2 = dict(p, eps=0.5)
    o2 = O.Oracle(p2, np.ones_like(z), zero, zero, z)
    o2.phase_encode()
    assert all(o2.flags("raw")[1:5] == 1)
    p3 = dict(p, eps=0.5000001)
    o3 = O.Oracle(p3, np.ones_like(z), zero, zero, z)
    o3.phase_encode()
    assert all(o3.flags("raw")[1:5] == 0)


# --------------------------------------------------------------------------
# Regularisation (refine the face neighbours of significant cells)
# --------------------------------------------------------------------------
def _brute_regularise(L, raw):
    sig = np.zeros_like(raw)
    for n in range(L):
        s = 1 << n
        for j in range(s):
            for i in range(s):
                f = 0
                for di, dj in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
                    ii, jj = i + di, j + dj
                    if 0 <= ii < s and 0 <= jj < s:
                        f |= raw[O.zindex(n, ii, jj)]
                sig[O.zindex(n, i, j)] = 1 if f else 0
    return sig


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_regularisation_matches_brute_force(seed):
    L = 5
    rng = np.random.default_rng(seed)
    raw = (rng.uniform(size=(4 ** L - 1) // 3) < 0.08).astype(np.uint8)
    assert np.array_equal(O.regularise_flags(L, raw), _brute_regularise(L, raw))


def test_regularisation_single_cell_plus_shape_clipped_at_edge():
    L = 3
    n = 2
    raw = np.zeros((4 ** L - 1) // 3, dtype=np.uint8)
    raw[O.zindex(n, 0, 2)] = 1          # west edge of level 2
    sig = O.regularise_flags(L, raw)
    want = {(0, 2), (1, 2), (0, 1), (0, 3)}
    for j in range(4):
        for i in range(4):
            assert sig[O.zindex(n, i, j)] == (1 if (i, j) in want else 0)
    assert sig.sum() == 4


# --------------------------------------------------------------------------
# Depth-first leaf list (Algorithm 2) against the paper's L = 2 example
# --------------------------------------------------------------------------
def test_dft_worked_example_l2():
    g = golden("traversal_l2_example.txt")
    L = 2
    sig = np.zeros((4 ** L - 1) // 3, dtype=np.uint8)
    for k in map(int, g["significant"].split()):
        sig[k] = 1
    leaves = O.dft_from_flags(L, sig)
    want = [int(t) for t in g["leaves"].split()]
    assert list(leaves) == want
    assert len(leaves) == 10
    # each finest thread t_m stops at the leaf that contains its target cell
    ptt = [int(t) for t in g["ptt"].split()]
    first = [0] * 16
    for lf in leaves:
        n = 0 if lf == 0 else (1 if lf < 5 else 2)
        m = lf - (4 ** n - 1) // 3
        span = 4 ** (L - n)
        for t in range(m * span, (m + 1) * span):
            first[t] = lf
    assert first == ptt


def test_dft_leaves_tile_the_domain():
    L = 6
    rng = np.random.default_rng(5)
    sig = (rng.uniform(size=(4 ** L - 1) // 3) < 0.7).astype(np.uint8)
    leaves = O.dft_from_flags(L, sig)
    covered = 0
    prev_first = -1
    for lf in leaves:
        n = 0
        while (4 ** (n + 1) - 1) // 3 <= lf:
            n += 1
        m = lf - (4 ** n - 1) // 3
        first = m * 4 ** (L - n)
        assert first > prev_first          # ascending first-descendant order
        prev_first = first
        covered += 4 ** (L - n)
        # every ancestor is significant, the leaf itself is not (unless finest)
        for a in range(n):
            anc = (4 ** a - 1) // 3 + (m >> (2 * (n - a)))
            assert sig[anc] == 1
        if n < L:
            assert sig[lf] == 0
    assert covered == 4 ** L
