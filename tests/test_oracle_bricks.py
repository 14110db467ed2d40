"""Pins of the oracle's brick linearisation of the active-vertex index
(Sec. 3.2.3: linearisations other than the F-Hash equation's may build the
hash): the rank order against a sort by brick key, the same active set as the
F-Hash order, brick locality, and the encoding and its adjoint invariant under
the row permutation between the two orders."""
import numpy as np
import pytest

import oracle as O


def _tiny_masks(rng, k):
    for _ in range(k):
        S = [int(v) for v in rng.integers(3, 12, 3)] + [int(rng.integers(2, 6))]
        m = (rng.random((S[3], S[2], S[1], S[0])) < rng.uniform(0.01, 0.2)).astype(np.uint8)
        R = [int(rng.integers(2, 9)) for _ in range(3)] + [int(rng.integers(2, 6))]
        yield R, m


def test_brick_ranks_equal_a_sort_by_brick_key():
    rng = np.random.default_rng(11)
    for R, m in _tiny_masks(rng, 60):
        rows, n_rows = O.level_slots(R, m)
        bricks, n_bricks = O.level_slots(R, m, O.LAYOUT_BRICKS)
        assert n_rows == n_bricks
        act = np.flatnonzero(rows >= 0)
        np.testing.assert_array_equal(np.flatnonzero(bricks >= 0), act)
        Rx, Ry, Rz, Rt = R
        x = act % Rx
        y = (act // Rx) % Ry
        z = (act // (Rx * Ry)) % Rz
        t = act // (Rx * Ry * Rz)
        inner = (x & 1) | (y & 1) << 1 | (z & 1) << 2 | (t & 1) << 3
        order = np.lexsort((inner, x >> 1, y >> 1, z >> 1, t >> 1))
        want = np.empty(act.size, np.int64)
        want[order] = np.arange(act.size)
        np.testing.assert_array_equal(bricks[act], want)


def test_aligned_cells_own_one_brick():
    # every vertex active, even resolutions: the 16 corners of a cell whose origin
    # is even in every axis are 16 consecutive slots starting at a multiple of 16
    R = [6, 4, 4, 4]
    m = np.ones((4, 4, 4, 6), np.uint8)
    bricks, n = O.level_slots(R, m, O.LAYOUT_BRICKS)
    assert n == int(np.prod(R))
    Rx, Ry, Rz, Rt = R
    for t in range(0, Rt - 1, 2):
        for z in range(0, Rz - 1, 2):
            for y in range(0, Ry - 1, 2):
                for x in range(0, Rx - 1, 2):
                    s = sorted(bricks[((t + dt) * Rz + z + dz) * Ry * Rx + (y + dy) * Rx + x + dx]
                               for dt in (0, 1) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1))
                    assert s == list(range(s[0], s[0] + 16)) and s[0] % 16 == 0


@pytest.mark.parametrize("F", [1, 2])
def test_encoding_and_adjoint_invariant_under_the_row_permutation(F):
    rng = np.random.default_rng(3)
    S = [11, 9, 7, 4]
    m = np.zeros((S[3], S[2], S[1], S[0]), np.uint8)
    m[rng.random(m.shape) < 0.08] = 1
    res = np.array([[3, 3, 3, 2], [6, 5, 4, 3], [11, 9, 7, 4]])
    gr = O.Grid(res, F, m)
    gb = O.Grid(res, F, m, layout=O.LAYOUT_BRICKS)
    assert gr.total_slots == gb.total_slots
    # row p of the rows-ordered table moves to row perm[p] of the brick-ordered one
    perm = np.full(gr.total_slots, -1, np.int64)
    for l in range(len(res)):
        a, b = gr.maps[l], gb.maps[l]
        on = a >= 0
        perm[gr.slot_offset[l] + a[on]] = gb.slot_offset[l] + b[on]
    assert (np.sort(perm) == np.arange(gr.total_slots)).all()
    table_r = rng.uniform(-1, 1, (gr.total_slots, F))
    table_b = np.empty_like(table_r)
    table_b[perm] = table_r
    pos = rng.random((500, 4)).astype(np.float32)
    er, _ = O.encode_fwd(gr, pos, table_r)
    eb, _ = O.encode_fwd(gb, pos, table_b)
    np.testing.assert_array_equal(er, eb)
    d_enc = rng.standard_normal(er.shape)
    dr, _ = O.encode_bwd(gr, pos, d_enc)
    db, _ = O.encode_bwd(gb, pos, d_enc)
    np.testing.assert_array_equal(db[perm], dr)
