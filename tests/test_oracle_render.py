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
