"""Helpers shared by the GPU parity tests: Morton permutations between the
oracle's row-major fields and the device's Morton arrays, leaf-list checks
and the tie band of the significance test.  Test code only."""
import numpy as np


def compact1by1(x):
    x = np.asarray(x, dtype=np.uint64) & np.uint64(0x5555555555555555)
    for s, m in ((1, 0x3333333333333333), (2, 0x0F0F0F0F0F0F0F0F),
                 (4, 0x00FF00FF00FF00FF), (8, 0x0000FFFF0000FFFF),
                 (16, 0x00000000FFFFFFFF)):
        x = (x | (x >> np.uint64(s))) & np.uint64(m)
    return x


def morton_to_rowmajor(L):
    """Index array r such that fine_morton[m] == field.ravel()[r[m]]."""
    m = np.arange(1 << (2 * L), dtype=np.uint64)
    i = compact1by1(m)
    j = compact1by1(m >> np.uint64(1))
    return (j * np.uint64(1 << L) + i).astype(np.int64)


def level_of(idx):
    idx = np.asarray(idx, dtype=np.int64)
    n = np.zeros_like(idx)
    off = 1
    k = 1
    while True:
        more = idx >= off
        if not more.any():
            break
        n += more
        k *= 4
        off += k
    return n


def check_leaf_list(L, leaves, sig):
    """Leaves tile the domain, come in ascending first-descendant order, every
    ancestor is significant and the leaf itself is not (unless finest)."""
    leaves = np.asarray(leaves, dtype=np.int64)
    n = level_of(leaves)
    off = ((4 ** n) - 1) // 3
    m = leaves - off
    first = m << (2 * (L - n))
    assert np.all(np.diff(first) > 0), "leaves not in ascending order"
    assert int(np.sum(4 ** (L - n))) == 4 ** L, "leaves do not tile the domain"
    coarse = n < L
    assert np.all(sig[leaves[coarse]] == 0), "a coarse leaf is significant"
    for a in range(L):
        sel = n > a
        anc = (4 ** a - 1) // 3 + (m[sel] >> (2 * (n[sel] - a)))
        assert np.all(sig[anc] == 1), "a leaf has an insignificant ancestor"


def tie_band_cells(L, eps, smax, details, rel=1e-12):
    """Coarse cells whose normalised detail of some variable lies within rel
    of the threshold 2^(n-L) eps (details: list of (3, Nc) arrays, smax: the
    matching s_max values)."""
    nc = details[0].shape[1]
    n = level_of(np.arange(nc))
    thr = eps * np.ldexp(1.0, (n - L).astype(np.int64))
    band = np.zeros(nc, dtype=bool)
    for d, s in zip(details, smax):
        dn = np.max(np.abs(d), axis=0) / s
        band |= np.abs(dn - thr) <= rel * np.maximum(thr, 1e-300)
    return np.nonzero(band)[0]


def part1by1(x):
    x = np.asarray(x, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    for s, m in ((16, 0x0000FFFF0000FFFF), (8, 0x00FF00FF00FF00FF),
                 (4, 0x0F0F0F0F0F0F0F0F), (2, 0x3333333333333333),
                 (1, 0x5555555555555555)):
        x = (x | (x << np.uint64(s))) & np.uint64(m)
    return x


def oracle_tie_band(o, rel=1e-12):
    """Tie band of the oracle's last encoding: coarse cells whose normalised
    detail of h, qx, qy or the bed lies within rel of 2^(n-L) eps, with the
    s_max values that encoding used."""
    sc = o.scalars()
    names = ("h", "qx", "qy", "z")
    smax = [sc["smax_" + v] for v in names]
    return tie_band_cells(o.L, float(o.params["eps"]), smax,
                          [o.details(v) for v in names], rel)


def band_region(L, ties):
    """Finest cells (Morton order) whose leaf can change when the flags of
    the tie cells flip: the descendants of each tie cell and of its face
    neighbours on its level (regularisation spreads a flag to those)."""
    mark = np.zeros((1 << (2 * L)) + 1, dtype=np.int64)
    ties = np.asarray(ties, dtype=np.int64)
    if ties.size == 0:
        return np.zeros(1 << (2 * L), dtype=bool)
    n = level_of(ties)
    m = (ties - ((4 ** n) - 1) // 3).astype(np.uint64)
    i = compact1by1(m).astype(np.int64)
    j = compact1by1(m >> np.uint64(1)).astype(np.int64)
    side = np.int64(1) << n
    for di, dj in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < side) & (jj >= 0) & (jj < side)
        code = (part1by1(ii[ok]) | (part1by1(jj[ok]) << np.uint64(1))).astype(np.int64)
        sh = 2 * (L - n[ok])
        np.add.at(mark, code << sh, 1)
        np.add.at(mark, (code + 1) << sh, -1)
    return np.cumsum(mark[:-1]) > 0


def leaf_of_finest(L, leaves):
    """For every finest cell (Morton order) the leaf that contains it."""
    leaves = np.asarray(leaves, dtype=np.int64)
    reps = np.int64(4) ** (L - level_of(leaves))
    out = np.repeat(leaves, reps)
    assert out.size == 1 << (2 * L), "leaves do not tile the domain"
    return out


def compare_leaf_lists(L, got, want, ties, log=print):
    """Leaf lists must be identical outside the tie band: cells whose
    normalised detail sits within 1e-12 of the threshold are listed, and
    only the finest cells they can affect may carry different leaves.
    Returns the number of tie cells."""
    got = np.asarray(got)
    want = np.asarray(want)
    ties = np.asarray(ties)
    if ties.size:
        log(f"  tie band: {ties.size} cells within 1e-12 of the threshold: "
            f"{ties[:20].tolist()}{' ...' if ties.size > 20 else ''}")
    else:
        log("  tie band: none")
    if np.array_equal(got, want):
        return int(ties.size)
    assert ties.size, "leaf lists differ and no cell lies in the tie band"
    region = band_region(L, ties)
    a, b = leaf_of_finest(L, got), leaf_of_finest(L, want)
    outside = (a != b) & ~region
    assert not outside.any(), (
        f"leaf lists differ outside the tie band at {int(outside.sum())} finest cells")
    log(f"  leaf lists differ only inside the tie band "
        f"({int((a != b).sum())} finest cells)")
    return int(ties.size)


def check_block_first(L, stored, canon):
    """Layout of a plan's block-first leaf list against the depth-first
    list of the same leaves: first every aligned 64-cell block whose finest
    cells are all leaves, in ascending order, each in Morton order; then
    the other leaves in depth-first order.  Returns the number of whole
    blocks."""
    off = (4 ** L - 1) // 3
    canon = np.asarray(canon, dtype=np.int64)
    stored = np.asarray(stored, dtype=np.int64)
    assert stored.size == canon.size
    fin = canon[canon >= off] - off
    blk, cnt = np.unique(fin >> 6, return_counts=True)
    full = blk[cnt == 64]
    nb = int(full.size)
    head = (off + (full[:, None] << 6) + np.arange(64)[None, :]).ravel()
    assert np.array_equal(stored[:64 * nb], head)
    in_full = np.zeros(canon.size, dtype=bool)
    f = canon >= off
    in_full[f] = np.isin((canon[f] - off) >> 6, full)
    assert np.array_equal(stored[64 * nb:], canon[~in_full])
    return nb
