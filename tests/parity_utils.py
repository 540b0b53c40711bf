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
