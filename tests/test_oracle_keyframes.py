"""Pins of the oracle's key-frame time axis and frame-aware sampler (Sec. 3.2.2)
by closed forms, the oracle's own cell location and the C sampler."""
import numpy as np

import oracle as O


def test_key_frames_sit_on_temporal_vertices():
    for T, frames in ((60, [0, 7, 13, 20, 26, 33, 39, 46, 52, 59]), (100, [0, 4, 50, 51, 99]),
                      (9, [2, 5, 6])):
        K = len(frames)
        tau = O.key_frame_times(T, frames)
        for k, f in enumerate(frames):
            c, frac = O.locate(float(tau[f]), K)
            assert (c, frac) in ((k, 0.0), (k - 1, 1.0)), (T, k, c, frac)
        assert (np.diff(tau) >= 0).all()
        assert tau[frames[0]] == 0 and tau[frames[-1]] == 1
        assert (tau[: frames[0] + 1] == 0).all() and (tau[frames[-1]:] == 1).all()
        # strictly between its neighbouring key frames' times
        for k in range(K - 1):
            mid = tau[frames[k] + 1: frames[k + 1]]
            assert (mid > tau[frames[k]]).all() and (mid < tau[frames[k + 1]]).all()


def test_evenly_spaced_key_frames_reduce_to_the_frame_axis():
    # every 11th of 100 frames (99 = 9 x 11): tau(n) = n / 99 for every frame
    T, K = 100, 10
    tau = O.key_frame_times(T, list(range(0, 100, 11)))
    np.testing.assert_array_equal(tau, (np.arange(T) / 99.0).astype(np.float32))


def test_midpoints_between_key_frames():
    frames = [0, 10, 30, 31, 51]
    tau = O.key_frame_times(52, frames)
    assert tau[5] == np.float32(0.5 / 4) and tau[20] == np.float32(1.5 / 4)
    assert tau[41] == np.float32(3.5 / 4)


def test_frame_sampler_reduces_to_the_sampler_and_maps_boxes():
    rng = np.random.default_rng(3)
    field = rng.random((5, 6, 7, 8), dtype=np.float32)          # T, Sz, Sy, Sx
    cs = np.sort(rng.choice(field.size, 300, replace=False)).astype(np.uint64)
    p0, t0 = O.sample_batch(11, 2, 400, field, cs)
    p1, t1 = O.sample_batch_frames(11, 2, 400, field, cs)
    np.testing.assert_array_equal(p0, p1)
    np.testing.assert_array_equal(t0, t1)
    frame_t = O.key_frame_times(5, [0, 2, 4])
    box = [1, 2, 0, 6, 5, 5]
    lin = cs[(cs % 8 >= 1) & (cs % 8 <= 6) & ((cs // 8) % 7 >= 2) & ((cs // 8) % 7 <= 5)]
    p2, t2 = O.sample_batch_frames(11, 3, 500, field, lin, frame_t, box)
    ids = lin[O.sample_ids(11, 3, 500, lin.size).astype(np.int64)].astype(np.int64)
    t, z, y, x = np.unravel_index(ids, field.shape)
    lo, hi = np.array(box[:3]), np.array(box[3:])
    for d, c in enumerate((x, y, z)):
        assert (p2[:, d] >= 0).all() and (p2[:, d] <= 1).all()
        np.testing.assert_array_equal(np.rint(p2[:, d] * (hi[d] - lo[d])) + lo[d], c)
    np.testing.assert_array_equal(p2[:, 3], frame_t[t])
    np.testing.assert_array_equal(t2, field.ravel()[ids])
