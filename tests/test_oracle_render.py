"""Pins of the oracle renderer (Sec. 3.3) by closed forms and geometry."""
import math

import numpy as np

import oracle as O
from paper_2507_03836_amd import synth


def _const_model(v0, F=2):
    """Decoder with zero weights and output bias v0: every sample's value is v0."""
    res = np.array([[3, 3, 3, 2], [5, 5, 5, 3]])
    g = O.Grid(res, F, None)
    width = [2 * F, 16, 16, 1]
    params = np.zeros(O.mlp_num_params(width))
    params[-1] = v0
    return g, np.zeros((g.total_slots, F)), width, params


def test_empty_occupancy_is_transparent():
    g, tab, width, params = _const_model(0.8)
    mask = np.zeros((3, 9, 8, 7), np.uint8)
    view = synth.orbit_view([7, 8, 9, 3], 0.3, 0.2, 24, 20)
    rgba, amb, ev = O.render(g, tab, width, params, mask, view, 1.0, synth.transfer_function(),
                             24, 20)
    assert ev == 0 and (rgba == 0).all()


def test_constant_field_closed_form():
    tf = synth.transfer_function()
    i = 200
    v0 = i / 255.0  # a transfer-function node: colour and opacity are the table entry
    c = tf[i].astype(np.float64)
    a0 = c[3]
    g, tab, width, params = _const_model(v0)
    mask = np.ones((3, 20, 20, 20), np.uint8)
    W, H = 40, 30
    view = synth.orbit_view([20, 20, 20, 3], 0.7, 0.3, W, H)
    rgba, amb, ev = O.render(g, tab, width, params, mask, view, 1.5, tf, W, H, ds=0.5)
    nstar = math.ceil(math.log(1 - 0.99) / math.log(1 - a0))
    A = rgba[..., 3]
    hit = A > 0
    assert hit.sum() > 0.3 * W * H
    # A after n identical samples is 1 - (1 - a0)^n; termination at the first n with A >= 0.99
    n = np.round(np.log(1 - A[hit]) / np.log(1 - a0))
    np.testing.assert_allclose(A[hit], 1 - (1 - a0) ** n, rtol=0, atol=1e-12)
    assert n.max() == nstar and (A[hit] <= 1 - (1 - a0) ** nstar + 1e-12).all()
    assert (A[hit] >= 0.99).sum() > 0
    # colour = c_rgb * A (front-to-back of a constant colour)
    for k in range(3):
        np.testing.assert_allclose(rgba[..., k][hit], c[k] * A[hit], rtol=1e-12, atol=1e-14)


def test_occupancy_of_a_single_voxel():
    mask = np.zeros((4, 6, 7, 8), np.uint8)
    vx, vy, vz, vt = 3, 2, 4, 2
    mask[vt, vz, vy, vx] = 1
    rng = np.random.default_rng(0)
    for _ in range(3000):
        p = rng.uniform(-0.5, [7.5, 6.5, 5.5]).astype(np.float32)
        t = np.float32(rng.uniform(0, 3))
        # the voxel is a corner of the cells whose floor coordinate is v-1 or v,
        # and of the timesteps t with floor(t) = vt or ceil(t) = vt
        inside = all(v - 1 <= min(max(math.floor(q), 0), S - 2) <= v
                     for q, v, S in zip(p, (vx, vy, vz), (8, 7, 6)))
        tin = math.floor(t) == vt or math.ceil(t) == vt
        assert O.occupied(mask, p, t) == (inside and tin)


def _axis_view(eye, W, H, fovy_deg):
    """Camera looking along -z (right = +x, up = +y)."""
    th = math.tan(math.radians(fovy_deg) / 2.0)
    return np.array([*eye, 0, 0, -1, 1, 0, 0, 0, 1, 0, th, W / H], np.float32)


def test_axis_aligned_camera_path_lengths():
    """Camera above the box [0, Sx-1] x [0, Sy-1] x [0, Sz-1] looking straight
    down, off-centre in x and y; every voxel occupied; a constant value whose
    transfer-function opacity a0 is small enough that no ray terminates.  A ray
    entering through the top face and leaving through the bottom face travels
    (Sz - 1) |d| / |d_z| (d = fwd + u right + v up), so it composites
    n = ceil(len/ds - 1/2) lattice samples and A = 1 - (1 - a0)^n; a ray whose
    footprint between the two faces lies outside the box's x-y rectangle is
    transparent.  Pins the pixel -> (u, v) map (centre pixel straight down,
    v up at the top row), the box bounds S - 1 and the lattice count."""
    Sx, Sy, Sz, T = 21, 17, 13, 3
    W, H, fovy, ds = 81, 61, 70.0, 0.5
    tf = synth.transfer_function()
    i = 49
    a0 = float(tf[i, 3])
    assert 0.01 < a0 < 0.03
    g, tab, width, params = _const_model(i / 255.0)
    mask = np.ones((T, Sz, Sy, Sx), np.uint8)
    ex, ey, ez = (Sx - 1) / 2 + 1.25, (Sy - 1) / 2 - 0.75, Sz - 1 + 30.0
    view = _axis_view((ex, ey, ez), W, H, fovy)
    rgba, amb, ev = O.render(g, tab, width, params, mask, view, 1.0, tf, W, H, ds=ds)
    A = rgba[..., 3]
    th = math.tan(math.radians(fovy) / 2.0)
    through = miss = 0
    for py in range(H):
        for px in range(W):
            u = (2 * (px + 0.5) / W - 1) * th * (W / H)
            v = (1 - 2 * (py + 0.5) / H) * th
            h1, h2 = ez - (Sz - 1), ez          # z distances to the top and bottom faces
            xt, yt, xb, yb = ex + u * h1, ey + v * h1, ex + u * h2, ey + v * h2
            m = 1e-3
            inside = lambda x, y: m < x < Sx - 1 - m and m < y < Sy - 1 - m
            if inside(xt, yt) and inside(xb, yb):
                length = (Sz - 1) * math.sqrt(u * u + v * v + 1.0)
                q = length / ds - 0.5
                if min(q - math.floor(q), math.ceil(q) - q) < 2e-3:
                    continue  # lattice count decided by rounding
                n = math.ceil(q)
                assert abs(A[py, px] - (1 - (1 - a0) ** n)) <= 1e-12, (px, py, n, A[py, px])
                for k in range(3):
                    assert abs(rgba[py, px, k] - tf[i, k] * A[py, px]) <= 1e-12
                through += 1
            elif ((xt < -m and xb < -m) or (xt > Sx - 1 + m and xb > Sx - 1 + m) or
                  (yt < -m and yb < -m) or (yt > Sy - 1 + m and yb > Sy - 1 + m)):
                assert A[py, px] == 0.0, (px, py)
                miss += 1
    assert through > 150 and miss > 150
    # the centre pixel looks straight down: (Sz - 1) / ds samples
    cy, cx = (H - 1) // 2, (W - 1) // 2
    assert abs(A[cy, cx] - (1 - (1 - a0) ** ((Sz - 1) / ds))) <= 1e-12
    # the image is not mirror-symmetric: the eye is off-centre (+x, -y), so the
    # box (up = +y at the top row) shows more rows above the centre than below
    # and more columns left of it than right
    hit = A > 0
    rows, cols = np.nonzero(hit.any(axis=1))[0], np.nonzero(hit.any(axis=0))[0]
    assert cy - rows.min() > rows.max() - cy
    assert cx - cols.min() > cols.max() - cx


def test_voxel_positions_pin():
    """Positions of linear voxel ids: the id decomposes as numpy.unravel_index
    over [T][Sz][Sy][Sx]; each coordinate is the correctly rounded FP32 quotient
    i / (S - 1) (within half an ulp of the exact rational, exact at both ends);
    ids beyond 2^32 at the 432^3 x 60 shape."""
    dims = (7, 5, 3, 4)
    N = int(np.prod(dims))
    ids = np.arange(N, dtype=np.uint64)
    pos = O.voxel_positions(ids, dims)
    n, k, j, i = np.unravel_index(np.arange(N), (dims[3], dims[2], dims[1], dims[0]))
    for d, c in enumerate((i, j, k, n)):
        exact = c / (dims[d] - 1)
        err = np.abs(pos[:, d].astype(np.float64) - exact)
        assert (err <= 2.0 ** -24 * exact + 1e-300).all()
        assert (np.rint(pos[:, d].astype(np.float64) * (dims[d] - 1)) == c).all()
    assert (pos[0] == 0).all() and (pos[-1] == 1).all()
    big = (432, 432, 432, 60)
    Nb = 432 ** 3 * 60
    assert Nb > 1 << 32
    lin = np.array([Nb - 1, Nb - 432, Nb - 432 * 432 * 432, 1 << 32], np.uint64)
    p = O.voxel_positions(lin, big)
    np.testing.assert_array_equal(p[0], [1, 1, 1, 1])
    np.testing.assert_array_equal(p[1], [0, 1, 1, 1])
    np.testing.assert_array_equal(p[2], [0, 0, 0, 1])
    n, k, j, i = np.unravel_index(1 << 32, (60, 432, 432, 432))
    want = [np.float32(c) / np.float32(S - 1) for c, S in zip((i, j, k, n), big)]
    np.testing.assert_array_equal(p[3], want)


def test_pixel_stats_of_the_constant_field():
    """The per-pixel statistics the GPU image bound is built from: composited
    sample count (A = 1 - (1 - a0)^n), sum of output magnitudes (n |v0| for the
    constant decoder, whose output is its bias) and the opacity margin."""
    tf = synth.transfer_function()
    i = 200
    v0 = i / 255.0
    a0 = float(tf[i, 3])
    g, tab, width, params = _const_model(v0)
    mask = np.ones((3, 20, 20, 20), np.uint8)
    view = synth.orbit_view([20, 20, 20, 3], 0.7, 0.3, 24, 18)
    rgba, amb, ev, pix = O.render(g, tab, width, params, mask, view, 1.5, tf, 24, 18,
                                  pixel_stats=True)
    n = pix[..., 0]
    np.testing.assert_allclose(rgba[..., 3], 1 - (1 - a0) ** n, rtol=0, atol=1e-12)
    np.testing.assert_allclose(pix[..., 1], n * v0, rtol=1e-12)
    assert n.sum() == ev
    hit = n > 0
    np.testing.assert_allclose(pix[..., 2][hit],
                               np.min(np.abs(1 - (1 - a0) ** np.arange(1, n.max() + 1)[None]
                                             - float(np.float32(0.99))) + np.where(
                                   np.arange(1, n.max() + 1)[None] <= n[hit][:, None], 0, 9),
                                   axis=1), rtol=0, atol=1e-12)
    assert (pix[..., 2][~hit] == 1.0).all()
