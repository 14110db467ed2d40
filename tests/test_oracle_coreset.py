"""Pins of the coreset oracle (Sec. 3.1) against brute force, closed forms and
library routines; none re-types the oracle's own slicing."""
import itertools

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import coreset as OC


def _field(shape, seed):
    return np.random.default_rng(seed).random(shape, dtype=np.float32)


def test_interval_brute_force_and_partition():
    f = _field((2, 3, 4, 70), 1)
    m = OC.feature_interval(f, 0.25, 0.75)
    for idx in itertools.product(*map(range, f.shape)):
        v = float(f[idx])
        assert m[idx] == (0.25 < v <= 0.75)  # both bounds exact in fp32
    # half-open ranges tile the real line: every voxel in exactly one
    parts = [OC.feature_interval(f, a, b) for a, b in
             [(-np.inf, 0.3), (0.3, 0.6), (0.6, np.inf)]]
    assert np.array_equal(sum(p.astype(int) for p in parts), np.ones(f.shape, int))
    assert OC.feature_interval(f, -np.inf, np.inf).all()


def test_isosurface_brute_force():
    """Voxel-centric enumeration: a voxel is kept iff one of the (up to 8)
    cells having it as a corner has corners on both sides of the level."""
    f = _field((2, 4, 5, 6), 2)
    lvl = 0.5
    m = OC.feature_isosurface(f, lvl)
    T, Z, Y, X = f.shape
    for t, z, y, x in itertools.product(range(T), range(Z), range(Y), range(X)):
        want = False
        for cz, cy, cx in itertools.product((z - 1, z), (y - 1, y), (x - 1, x)):
            if not (0 <= cz < Z - 1 and 0 <= cy < Y - 1 and 0 <= cx < X - 1):
                continue
            vals = [f[t, cz + a, cy + b, cx + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)]
            if any(v >= lvl for v in vals) and any(v < lvl for v in vals):
                want = True
        assert m[t, z, y, x] == want, (t, z, y, x)


def test_isosurface_linear_ramp_closed_form():
    """v = x: the level 3.5 crosses only the cells between x = 3 and x = 4, so
    the feature is exactly the two voxel planes x = 3 and x = 4; a level on a
    voxel value (v = 3) crosses the cells [2, 3] only."""
    X = 9
    f = np.broadcast_to(np.arange(X, dtype=np.float32), (2, 3, 4, X)).copy()
    m = OC.feature_isosurface(f, 3.5)
    assert np.array_equal(np.nonzero(m.any(axis=(0, 1, 2)))[0], [3, 4])
    assert m[..., 3].all() and m[..., 4].all()
    m = OC.feature_isosurface(f, 3.0)
    assert np.array_equal(np.nonzero(m.any(axis=(0, 1, 2)))[0], [2, 3])
    # a constant field has no isosurface
    assert not OC.feature_isosurface(np.zeros((1, 3, 3, 3), np.float32), 0.0).any()


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_dilation_is_scipy_cube_dilation_per_frame(r):
    rng = np.random.default_rng(3 + r)
    m = rng.random((3, 9, 11, 70)) < 0.01
    got = OC.dilate(m, r)
    cube = np.ones((1, 2 * r + 1, 2 * r + 1, 2 * r + 1), bool)  # no reach across frames
    want = ndi.binary_dilation(m, structure=cube) if r else m
    assert np.array_equal(got, want)


@pytest.mark.parametrize("r", [4, 8])
def test_dilation_radius_beyond_the_volume(r):
    """A radius at or above a dimension fills that dimension (scipy, cube)."""
    m = np.zeros((2, 3, 5, 70), bool)
    m[0, 1, 2, 30] = True
    got = OC.dilate(m, r)
    cube = np.ones((1, 2 * r + 1, 2 * r + 1, 2 * r + 1), bool)
    assert np.array_equal(got, ndi.binary_dilation(m, structure=cube))
    assert got[0, :, :, 30 - r:31 + r].all()
    assert not got[1].any()


def test_dilation_of_a_single_voxel_is_a_clipped_cube():
    m = np.zeros((2, 6, 6, 6), bool)
    m[1, 0, 2, 5] = True
    d = OC.dilate(m, 2)
    assert not d[0].any()
    z, y, x = np.nonzero(d[1])
    assert (z.min(), z.max(), y.min(), y.max(), x.min(), x.max()) == (0, 2, 0, 4, 3, 5)
    assert d[1].sum() == 3 * 5 * 3


def test_boxes_are_tight_and_fbb_contains_every_box():
    rng = np.random.default_rng(5)
    m = rng.random((4, 7, 8, 90)) < 0.002
    m[2] = False  # an empty frame
    b = OC.feature_boxes(m)
    T, Z, Y, X = m.shape
    for k in range(T):
        if not m[k].any():
            assert list(b[k]) == [X, Y, Z, -1, -1, -1]
            continue
        x0, y0, z0, x1, y1, z1 = b[k]
        inside = np.zeros_like(m[k])
        inside[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1] = True
        assert not (m[k] & ~inside).any()  # contains the feature
        # tight: every face of the box touches a feature voxel
        assert m[k, z0].any() and m[k, z1].any() and m[k, :, y0].any() and m[k, :, y1].any()
        assert m[k, :, :, x0].any() and m[k, :, :, x1].any()
    fbb = b[T]
    ne = [k for k in range(T) if m[k].any()]
    assert list(fbb[:3]) == list(b[ne, :3].min(axis=0))
    assert list(fbb[3:]) == list(b[ne, 3:].max(axis=0))
    assert list(OC.feature_boxes(np.zeros((2, 3, 3, 3), bool))[2]) == [3, 3, 3, -1, -1, -1]


def test_morton_bit_closed_form():
    assert OC.morton_bit(1, 0, 0) == 1 and OC.morton_bit(0, 1, 0) == 2
    assert OC.morton_bit(0, 0, 1) == 4 and OC.morton_bit(2, 0, 0) == 8
    assert OC.morton_bit(0, 2, 0) == 16 and OC.morton_bit(0, 0, 2) == 32
    assert OC.morton_bit(3, 3, 3) == 63
    assert sorted(OC.morton_bit(*p) for p in itertools.product(range(4), repeat=3)) == \
        list(range(64))


def test_occupancy_grid_single_voxels_and_popcount():
    T, Z, Y, X = 2, 6, 7, 9
    m = np.zeros((T, Z, Y, X), bool)
    for (t, z, y, x) in [(0, 0, 0, 0), (0, 5, 6, 8), (1, 3, 2, 1), (1, 4, 4, 4)]:
        m[t, z, y, x] = True
    occ = OC.occupancy_grid(m)
    assert occ.shape == (T, 2, 2, 3)
    assert occ[0, 0, 0, 0] == 1
    assert occ[0, 1, 1, 2] == np.uint64(1) << np.uint64(OC.morton_bit(0, 2, 1))
    assert occ[1, 0, 0, 0] == np.uint64(1) << np.uint64(OC.morton_bit(1, 2, 3))
    assert occ[1, 1, 1, 1] == 1
    rng = np.random.default_rng(9)
    m = rng.random((3, 10, 13, 70)) < 0.2
    occ = OC.occupancy_grid(m)
    pop = sum(bin(int(w)).count("1") for w in occ.ravel())
    assert pop == int(m.sum())


def test_coreset_ids_and_row_packing():
    rng = np.random.default_rng(11)
    m = rng.random((2, 3, 5, 130)) < 0.1
    ids = OC.coreset_ids(m)
    t, z, y, x = np.nonzero(m)
    lin = ((t * 3 + z) * 5 + y) * 130 + x
    assert np.array_equal(ids, np.sort(lin).astype(np.uint64))
    w = OC.pack_rows(m)
    assert w.shape == (2, 3, 5, 3)
    assert int(w[t[0], z[0], y[0], x[0] // 64]) >> int(x[0] % 64) & 1 == 1
    assert (w[..., 2] >> np.uint64(2)).max() == 0  # padding bits of the last word are zero
    assert np.array_equal(OC.unpack_rows(w, m.shape), m)
