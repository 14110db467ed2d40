"""Pins of the oracle's spatial-hash comparison index (the alternative the
paper contrasts F-Hash with; the hash itself is this repository's definition,
so these check the construction and its use, not a published value):

- a level of at most 2^b vertices keeps the F-Hash equation (row = vertex id);
- a hashed level has 2^b rows, every row in range, and the vertices of the x
  axis (y = z = t = 0, x's multiplier is 1) land on row x mod 2^b;
- pigeonhole: a level of V > 2^b vertices uses at most 2^b rows, so some
  vertices share one;
- the encoding through the hashed rows equals the encoding of the dense box
  whose table holds, per vertex, the row that vertex hashes to (tied
  embeddings), i.e. the map is used exactly where the F-Hash slot would be.
"""
import numpy as np

import oracle as O

RES = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]


def test_small_levels_keep_the_fhash_equation():
    g = O.Grid(RES, 2, hash_bits=9)
    assert g.counts == [128, 512, 512, 512]
    np.testing.assert_array_equal(g.maps[0], np.arange(128))


def test_hashed_rows_range_axis_and_pigeonhole():
    g = O.Grid(RES, 2, hash_bits=9)
    for l in (1, 2, 3):
        m = g.maps[l]
        nv = int(np.prod(RES[l]))
        assert m.shape == (nv,) and m.min() >= 0 and m.max() < 512
        Rx = RES[l][0]
        np.testing.assert_array_equal(m[:Rx], np.arange(Rx) % 512)
        assert len(np.unique(m)) <= 512 < nv
    # a level with more rows available than vertices is not hashed
    g2 = O.Grid(RES, 2, hash_bits=20)
    for l in range(4):
        np.testing.assert_array_equal(g2.maps[l], np.arange(int(np.prod(RES[l]))))


def test_encoding_equals_dense_box_with_tied_embeddings():
    rng = np.random.default_rng(8)
    gh = O.Grid(RES, 2, hash_bits=9)
    gd = O.Grid(RES, 2)
    tab_h = rng.uniform(-1, 1, (gh.total_slots, 2))
    tab_d = np.zeros((gd.total_slots, 2))
    for l in range(4):
        tab_d[gd.slot_offset[l]: gd.slot_offset[l + 1]] = tab_h[gh.slot_offset[l] + gh.maps[l]]
    pos = rng.uniform(0, 1, (300, 4)).astype(np.float32)
    eh, _ = O.encode_fwd(gh, pos, tab_h)
    ed, _ = O.encode_fwd(gd, pos, tab_d)
    np.testing.assert_array_equal(eh, ed)
