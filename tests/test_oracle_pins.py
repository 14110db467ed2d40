"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these tests re-types an oracle formula: each checks the oracle against
an independent fact (a value printed in the paper, a closed form, an invariant,
brute force on a tiny input with exact rational arithmetic, a library routine).
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O


# ----------------------------------------------------------------------------- RNG
def test_philox_known_answers(golden_dir):
    kat = json.load(open(os.path.join(golden_dir, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(O.philox4x32_10(ctr, key)) == out


def test_sample_ids_range_and_mapping():
    # M = 1 maps every draw to 0; ids are the high word of r*M (so < M).
    assert (O.sample_ids(7, 3, 1000, 1) == 0).all()
    M = 1000003
    ids = O.sample_ids(11, 5, 200000, M)
    assert ids.max() < M
    # uniformity: chi-square over 50 equal bins, 49 dof (p ~ 1e-6 bound ~ 100)
    h = np.bincount((ids * 50 // M).astype(np.int64), minlength=50)
    exp = ids.size / 50
    assert ((h - exp) ** 2 / exp).sum() < 110
    # different steps give different streams; same step reproduces
    assert not np.array_equal(ids[:100], O.sample_ids(11, 6, 100, M))
    assert np.array_equal(ids[:100], O.sample_ids(11, 5, 100, M))


def test_sample_ids_from_philox_words():
    # draw i of step s: r = out1:out0 of Philox(ctr=(i, 0, s, 0), key=(seed, 0)),
    # id = floor(r * M / 2^64), checked with Python big integers.
    seed, step, M = 1234, 9, 987654321
    ids = O.sample_ids(seed, step, 5, M)
    for i in range(5):
        o = O.philox4x32_10([i, 0, step, 0], [seed, 0])
        r = (int(o[1]) << 32) | int(o[0])
        assert int(ids[i]) == (r * M) >> 64


def test_sample_batch_positions_and_labels():
    rng = np.random.default_rng(0)
    field = rng.random((3, 4, 5, 6), dtype=np.float32)  # T, Sz, Sy, Sx
    pos, tgt = O.sample_batch(42, 1, 500, field)
    ids = O.sample_ids(42, 1, 500, field.size)
    t, z, y, x = np.unravel_index(ids.astype(np.int64), field.shape)
    np.testing.assert_array_equal(pos[:, 0], x.astype(np.float32) / np.float32(5))
    np.testing.assert_array_equal(pos[:, 3], t.astype(np.float32) / np.float32(2))
    np.testing.assert_array_equal(tgt, field[t, z, y, x])
    coreset = np.array([3, 17, 64, 100], np.uint64)
    pos2, tgt2 = O.sample_batch(42, 2, 50, field, coreset)
    assert set(tgt2.tolist()) <= set(field.ravel()[coreset.astype(np.int64)].tolist())


# ----------------------------------------------------------------------------- resolutions
def test_table3_parameter_counts(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "table3_parameter_counts.json")))
    F = g["n_features"]
    h = g["mlp_hidden"]
    for c in g["cases"]:
        S = list(c["fbb_xyz"]) + [c["key_frames"]]
        res = O.fold_resolutions(S, g["fold"])
        enc = F * sum(int(np.prod(r)) for r in res)
        width = [len(res) * F] + h + [1]
        total = enc + O.mlp_num_params(width)
        assert abs(total / 2 ** 20 - c["params_mebi"]) <= c["tolerance_mebi"], (c, total / 2 ** 20)
        frac = 100.0 * np.prod(c["fbb_xyz"]) / np.prod(c["frame_xyz"])
        assert abs(frac - c["fbb_fraction_percent"]) < 0.005
    for c in g["fbb_fraction_only"]:
        frac = 100.0 * np.prod(c["fbb_xyz"]) / np.prod(c["frame_xyz"])
        assert abs(frac - c["fbb_fraction_percent"]) < 0.005


def test_fold_policy_hand_example():
    # Hand-evaluated from the level equations with f = 2: L_x = ceil(log2 5) = 3,
    # L_y = ceil(log2 3) = 2, L_z = ceil(log2 2) = 1 -> L_s = 3; each dimension
    # divides by f (rounding up) while above f, else pads with 2.
    res = O.fold_resolutions([5, 3, 2, 2], 2)
    assert res.tolist() == [[5, 3, 2, 2], [3, 2, 2, 2], [2, 2, 2, 2]]
    # fold 4 on 200: L = ceil(log4 200) = 4; 200 -> 50 -> 13 -> 4 (4 <= f is kept as
    # computed by the ceiling, the tail pads only below)
    res = O.fold_resolutions([200, 16, 16, 10], 4)
    assert res[:, 0].tolist() == [200, 50, 13, 4]
    assert res[:, 3].tolist() == [10, 3, 2, 2]
    assert O.fold_num_levels(200, 2) == 8 and O.fold_num_levels(256, 2) == 8
    assert O.fold_num_levels(257, 2) == 9


def test_geometric_policy_endpoints_and_clamp():
    res = O.geometric_resolutions(16, 16, 512, 4, 100, [480, 720, 120, 100])
    assert res[0].tolist() == [16, 16, 16, 4]
    assert res[-1].tolist() == [480, 512, 120, 100]  # clamped to the native size
    assert (np.diff(res, axis=0) >= 0).all()
    res = O.geometric_resolutions(4, 4, 32, 2, 8, [32, 32, 32, 8])
    assert res.tolist() == [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]


# ----------------------------------------------------------------------------- index
def _cells_rational(i, S, R):
    p = Fraction(i, S - 1)
    return {c for c in range(R - 1) if Fraction(c, R - 1) <= p <= Fraction(c + 1, R - 1)}


def test_voxel_cells_closed_box_rule():
    rng = np.random.default_rng(1)
    for _ in range(400):
        S = int(rng.integers(2, 40))
        R = int(rng.integers(2, 40))
        i = int(rng.integers(0, S))
        lo, hi = O.voxel_cells(i, S, R)
        assert set(range(lo, hi + 1)) == _cells_rational(i, S, R)


def _bruteforce_slots(res, mask):
    """Active vertices by exhaustive rational geometry, ranked in F-Hash order."""
    T, Sz, Sy, Sx = mask.shape
    S = (Sx, Sy, Sz, T)
    pts = np.argwhere(mask)  # (n, z, y, x)
    cells = set()
    for (n, k, j, i) in pts:
        per = [_cells_rational(int(v), S[d], int(res[d])) for d, v in enumerate((i, j, k, n))]
        cells.update(itertools.product(*per))
    Rx, Ry, Rz, Rt = [int(r) for r in res]
    active = np.zeros((Rt, Rz, Ry, Rx), bool)
    for (cx, cy, cz, ct) in cells:
        active[ct:ct + 2, cz:cz + 2, cy:cy + 2, cx:cx + 2] = True
    flat = active.ravel()
    slots = np.full(flat.size, -1, np.int64)
    slots[flat] = np.arange(flat.sum())
    return slots


def test_index_bruteforce_tiny_grids():
    rng = np.random.default_rng(2)
    for trial in range(25):
        S = rng.integers(2, 7, size=4)
        mask = (rng.random((S[3], S[2], S[1], S[0])) < rng.uniform(0.02, 0.4)).astype(np.uint8)
        res = rng.integers(2, 6, size=4)
        got, cnt = O.level_slots(res, mask)
        exp = _bruteforce_slots(res, mask)
        np.testing.assert_array_equal(got, exp)
        assert cnt == int((exp >= 0).sum())


def test_index_dense_is_the_fhash_equation():
    res = [3, 4, 2, 5]
    slots, cnt = O.level_slots(res, None)
    assert cnt == 3 * 4 * 2 * 5
    Rx, Ry, Rz, Rt = res
    for t, z, y, x in itertools.product(range(Rt), range(Rz), range(Ry), range(Rx)):
        lin = t * Rx * Ry * Rz + z * Rx * Ry + y * Rx + x  # Sec. 3.2.3
        assert slots[lin] == lin
    # an all-ones mask activates every vertex: same map
    full = np.ones((6, 5, 5, 5), np.uint8)
    s2, c2 = O.level_slots(res, full)
    np.testing.assert_array_equal(s2, slots)


def test_index_is_minimal_perfect_hash():
    rng = np.random.default_rng(3)
    mask = (rng.random((8, 32, 32, 32)) < 0.05).astype(np.uint8)
    for res in ([4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8], [7, 13, 5, 4]):
        slots, cnt = O.level_slots(res, mask)
        act = slots[slots >= 0]
        # injective, no waste: active slots are exactly 0..count-1, increasing in lin order
        np.testing.assert_array_equal(act, np.arange(cnt))


def test_training_samples_hit_active_corners():
    """Every masked voxel, located as a sample, sees active corners wherever its
    weight is not negligible (the coreset trains only existing slots)."""
    rng = np.random.default_rng(4)
    mask = (rng.random((5, 12, 11, 10)) < 0.08).astype(np.uint8)
    res = np.array([[4, 4, 3, 2], [7, 6, 5, 3], [10, 11, 12, 5]])
    g = O.Grid(res, 1, mask)
    T, Sz, Sy, Sx = mask.shape
    pts = np.argwhere(mask)
    pos = np.stack([pts[:, 3] / np.float32(Sx - 1), pts[:, 2] / np.float32(Sy - 1),
                    pts[:, 1] / np.float32(Sz - 1), pts[:, 0] / np.float32(T - 1)],
                   axis=1).astype(np.float32)
    pos = np.stack([pts[:, 3].astype(np.float32) / np.float32(Sx - 1),
                    pts[:, 2].astype(np.float32) / np.float32(Sy - 1),
                    pts[:, 1].astype(np.float32) / np.float32(Sz - 1),
                    pts[:, 0].astype(np.float32) / np.float32(T - 1)], axis=1)
    slots, w = O.corners(g, pos)
    assert not ((slots < 0) & (w > 1e-4)).any()


# ----------------------------------------------------------------------------- encoding
def test_locate_special_values():
    assert O.locate(0.0, 9) == (0, 0.0)
    assert O.locate(1.0, 9) == (7, 1.0)
    assert O.locate(0.5, 9) == (4, 0.0)
    assert O.locate(-3.0, 9) == (0, 0.0)
    assert O.locate(7.0, 9) == (7, 1.0)
    assert O.locate(float("nan"), 9) == (0, 0.0)
    c, f = O.locate(0.3, 11)
    assert c == 3 and abs(f - (np.float32(0.3) * np.float32(10) - 3)) == 0.0


def _dense_grid(res, F):
    return O.Grid(np.asarray(res, np.int64).reshape(-1, 4), F, None)


def test_weights_partition_of_unity():
    g = _dense_grid([[5, 4, 3, 6], [9, 9, 9, 2]], 1)
    pos = np.random.default_rng(5).random((300, 4), dtype=np.float32)
    slots, w = O.corners(g, pos)
    np.testing.assert_allclose(w.sum(-1), 1.0, rtol=0, atol=1e-12)
    assert (w >= 0).all()


def _multilinear(coef, x, y, z, t):
    # g = sum over subsets A of {x,y,z,t} of c_A prod_{d in A} d
    v = 0.0
    for m in range(16):
        term = coef[m]
        for d, q in enumerate((x, y, z, t)):
            if (m >> d) & 1:
                term = term * q
        v = v + term
    return v


def test_multilinear_field_reproduced_exactly():
    res = np.array([[5, 7, 4, 3], [9, 6, 8, 5]])
    F = 2
    g = _dense_grid(res, F)
    rng = np.random.default_rng(6)
    coefs = rng.normal(size=(F, 16))
    table = np.zeros((g.total_slots, F))
    for l, r in enumerate(res):
        Rx, Ry, Rz, Rt = r
        t, z, y, x = np.meshgrid(np.arange(Rt), np.arange(Rz), np.arange(Ry), np.arange(Rx),
                                 indexing="ij")
        for k in range(F):
            vals = _multilinear(coefs[k], x / (Rx - 1), y / (Ry - 1), z / (Rz - 1), t / (Rt - 1))
            table[g.slot_offset[l]:g.slot_offset[l + 1], k] = vals.ravel()
    pos = rng.random((400, 4), dtype=np.float32)
    enc, _ = O.encode_fwd(g, pos, table)
    for l, r in enumerate(res):
        # the located position (FP32 cell + exact fraction) is what is interpolated
        q = []
        for d in range(4):
            u = np.array([sum(O.locate(float(p), int(r[d]))) for p in pos[:, d]])
            q.append(u / (r[d] - 1))
        for k in range(F):
            exp = _multilinear(coefs[k], *q)
            np.testing.assert_allclose(enc[:, l * F + k], exp, rtol=0, atol=1e-12)


def test_vertex_reproduction():
    res = [[9, 5, 3, 17]]  # R-1 powers of two: vertex positions exact in FP32
    g = _dense_grid(res, 1)
    table = np.random.default_rng(7).normal(size=(g.total_slots, 1))
    Rx, Ry, Rz, Rt = res[0]
    pts = np.array([[x, y, z, t] for x in range(Rx) for y in range(Ry) for z in range(Rz)
                    for t in (0, 5, Rt - 1)])
    pos = (pts / (np.array(res[0]) - 1)).astype(np.float32)
    enc, _ = O.encode_fwd(g, pos, table)
    lin = ((pts[:, 3] * Rz + pts[:, 2]) * Ry + pts[:, 1]) * Rx + pts[:, 0]
    np.testing.assert_allclose(enc[:, 0], table[lin, 0], rtol=0, atol=1e-14)


def test_single_cell_is_textbook_quadrilinear():
    g = _dense_grid([[2, 2, 2, 2]], 1)
    E = np.random.default_rng(8).normal(size=(16, 1))
    pos = np.random.default_rng(9).random((50, 4), dtype=np.float32)
    enc, _ = O.encode_fwd(g, pos, E)
    p = pos.astype(np.float64)
    V = E[:, 0].reshape(2, 2, 2, 2)  # [t][z][y][x]
    for s in range(50):
        x, y, z, t = p[s]
        wx, wy, wz, wt = [np.array([1 - q, q]) for q in (x, y, z, t)]
        exp = np.einsum("tzyx,t,z,y,x->", V, wt, wz, wy, wx)
        assert abs(enc[s, 0] - exp) < 1e-12


def test_encoding_linear_in_tables_and_adjoint():
    rng = np.random.default_rng(10)
    mask = (rng.random((6, 9, 8, 7)) < 0.15).astype(np.uint8)
    res = np.array([[3, 3, 3, 2], [5, 4, 6, 3], [7, 8, 9, 6]])
    g = O.Grid(res, 2, mask)
    pos = rng.random((700, 4), dtype=np.float32)
    E1 = rng.normal(size=(g.total_slots, 2))
    E2 = rng.normal(size=(g.total_slots, 2))
    e1, _ = O.encode_fwd(g, pos, E1)
    e2, _ = O.encode_fwd(g, pos, E2)
    e12, _ = O.encode_fwd(g, pos, 2.0 * E1 - 3.0 * E2)
    np.testing.assert_allclose(e12, 2.0 * e1 - 3.0 * e2, rtol=0, atol=1e-12)
    G = rng.normal(size=e1.shape)
    dE, mag = O.encode_bwd(g, pos, G)
    lhs = float((e1 * G).sum())
    rhs = float((E1 * dE).sum())
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    assert (mag >= np.abs(dE) - 1e-15).all()


def test_inactive_corners_contribute_zero():
    mask = np.zeros((2, 9, 9, 9), np.uint8)
    mask[0, 0, 0, 0] = 1  # one corner voxel: only the cell at the origin is active
    g = O.Grid(np.array([[5, 5, 5, 2]]), 1, mask)
    assert g.total_slots == 16
    table = np.ones((16, 1))
    far = np.array([[0.9, 0.9, 0.9, 0.5]], np.float32)
    enc, _ = O.encode_fwd(g, far, table)
    assert enc[0, 0] == 0.0
    near = np.array([[0.1, 0.1, 0.1, 0.5]], np.float32)
    enc, _ = O.encode_fwd(g, near, table)
    assert abs(enc[0, 0] - 1.0) < 1e-12  # partition of unity inside the active cell


# ----------------------------------------------------------------------------- MLP
def _numpy_mlp(width, params, x):
    h = x
    off = 0
    for k in range(len(width) - 1):
        i, o = width[k], width[k + 1]
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        h = h @ W.T + b
        if k < len(width) - 2:
            h = np.maximum(h, 0.0)
    return h


def test_mlp_matches_numpy_layers():
    width = [8, 32, 32, 1]
    rng = np.random.default_rng(11)
    P = O.mlp_num_params(width)
    assert P == 8 * 32 + 32 + 32 * 32 + 32 + 32 + 1
    params = rng.normal(size=P) * 0.3
    x = rng.normal(size=(64, 8))
    y, acts, ymag = O.mlp_fwd(width, params, x)
    np.testing.assert_allclose(y, _numpy_mlp(width, params, x), rtol=1e-13, atol=1e-13)
    assert (ymag >= np.abs(y) - 1e-12).all()


def test_mlp_gradients_central_differences():
    width = [6, 16, 16, 1]
    rng = np.random.default_rng(12)
    P = O.mlp_num_params(width)
    params = rng.normal(size=P) * 0.5
    x = rng.normal(size=(5, 6))
    dy = rng.normal(size=(5, 1))
    y, acts, _ = O.mlp_fwd(width, params, x)
    dp, dx, dpm, dxm = O.mlp_bwd(width, params, acts, dy, 5)

    def loss(p, xx):
        return float((_numpy_mlp(width, p, xx) * dy).sum())

    for j in rng.choice(P, 40, replace=False):
        h = 1e-6 * max(1.0, abs(params[j]))
        e = np.zeros(P)
        e[j] = h
        fd = (loss(params + e, x) - loss(params - e, x)) / (2 * h)
        assert abs(fd - dp[j]) <= 1e-6 * max(1.0, abs(fd)), j
    for s in range(5):
        for i in range(6):
            h = 1e-6
            e = np.zeros_like(x)
            e[s, i] = h
            fd = (loss(params, x + e) - loss(params, x - e)) / (2 * h)
            assert abs(fd - dx[s, i]) <= 1e-6 * max(1.0, abs(fd))
    assert (dpm >= np.abs(dp) - 1e-12).all()


def test_table_gradients_central_differences():
    """d(MSE(MLP(enc(E))))/dE by the oracle's adjoints vs central differences."""
    rng = np.random.default_rng(13)
    mask = (rng.random((4, 7, 7, 7)) < 0.3).astype(np.uint8)
    res = np.array([[3, 3, 3, 2], [5, 6, 4, 3]])
    g = O.Grid(res, 2, mask)
    width = [4, 16, 16, 1]
    params = rng.normal(size=O.mlp_num_params(width)) * 0.5
    pos = rng.random((30, 4), dtype=np.float32)
    v = rng.random(30)
    E = rng.normal(size=(g.total_slots, 2)) * 0.5

    def loss(EE):
        enc, _ = O.encode_fwd(g, pos, EE)
        y, _, _ = O.mlp_fwd(width, params, enc)
        return O.mse(y[:, 0], v)[0]

    enc, _ = O.encode_fwd(g, pos, E)
    y, acts, _ = O.mlp_fwd(width, params, enc)
    L0, dy = O.mse(y[:, 0], v)
    _, denc, _, _ = O.mlp_bwd(width, params, acts, dy.reshape(-1, 1), 30)
    dE, _ = O.encode_bwd(g, pos, denc)
    for j in rng.choice(E.size, 30, replace=False):
        h = 1e-6
        e = np.zeros(E.size)
        e[j] = h
        fd = (loss(E + e.reshape(E.shape)) - loss(E - e.reshape(E.shape))) / (2 * h)
        assert abs(fd - dE.ravel()[j]) <= 1e-6 * max(1e-3, abs(fd)), j


# ----------------------------------------------------------------------------- loss/adam
def test_mse_and_psnr_closed_forms():
    y = np.array([0.0, 1.0, 0.5, 0.25])
    v = np.array([0.1, 0.8, 0.5, 0.0])
    L, dy = O.mse(y, v)
    assert abs(L - (0.01 + 0.04 + 0.0 + 0.0625) / 4) < 1e-15
    np.testing.assert_allclose(dy, 2 * (y - v) / 4, rtol=0, atol=1e-15)
    assert abs(O.psnr(0.01) - 20.0) < 1e-12
    assert abs(O.psnr(1e-4) - 40.0) < 1e-12


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(14)
    p0 = rng.normal(size=1000)
    g = rng.normal(size=1000) * np.logspace(-10, 1, 1000)
    g[::7] = 0.0
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    lr, eps = 0.01, 1e-8
    O.adam(p, g, m, v, lr, 0.9, 0.999, eps, 1)
    # step 1: m_hat = g, v_hat = g^2  ->  dp = -lr g / (|g| + eps)
    np.testing.assert_allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_matches_torch_optim_float64():
    rng = np.random.default_rng(15)
    p0 = rng.normal(size=257)
    grads = [rng.normal(size=257) * s for s in (1.0, 0.1, 3.0, 0.0, 0.5)]
    p, m, v = p0.copy(), np.zeros(257), np.zeros(257)
    for k, g in enumerate(grads, 1):
        O.adam(p, g, m, v, 0.01, 0.9, 0.999, 1e-8, k)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        opt.zero_grad()
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_one_by_one_vertex_activity_matches_enumeration():
    from paper_2507_03836_amd import synth
    rng = np.random.default_rng(16)
    for trial in range(10):
        S = rng.integers(2, 80, size=4)
        S[3] = rng.integers(2, 7)
        mask = (rng.random((S[3], S[2], S[1], S[0])) < rng.uniform(0.001, 0.2)).astype(np.uint8)
        res = [int(rng.integers(2, 40)) for _ in range(3)] + [int(rng.integers(2, 8))]
        bits = synth.pack_mask_rows(mask)
        slots, _ = O.level_slots(res, mask)
        Rx, Ry, Rz, Rt = res
        for q in rng.choice(len(slots), min(50, len(slots)), replace=False):
            v = [q % Rx, (q // Rx) % Ry, (q // (Rx * Ry)) % Rz, q // (Rx * Ry * Rz)]
            assert O.vertex_active_bits(res, bits, list(S), v) == (slots[q] >= 0)
