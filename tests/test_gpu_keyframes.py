"""Key-frame training (Sec. 3.2.2) and the dense FBB mode (Sec. 3.1-3.2.1) on
the device against the oracle:

- fhash_coreset_frames equals the oracle's coreset of the listed frames, bit
  for bit;
- fhash_sample with a frame-time table (fhash_key_frame_times) and an FBB box
  equals the oracle's frame-aware sampler bit for bit;
- a render at frames that were not trained (between key frames) through the
  step API with the render state's model time matches the oracle's render at
  that time coordinate within the derived image bound;
- a model over the dense FBB with fold-policy levels (fhash_fold_resolutions,
  finest temporal level = the key frames) trains one fused step equal to the
  oracle within the FP32 tolerance.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import coreset as OC
from paper_2507_03836_amd import synth

from workloads import coreset_ids, render_bound, tiny_volume

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-12
KEY = [0, 3, 5, 7]   # key frames of the 8-frame tiny volume


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


def _dims(mask):
    T, Sz, Sy, Sx = mask.shape
    return [Sx, Sy, Sz, T]


@pytest.mark.parametrize("case", range(5))
def test_coreset_frames_bit_exact(fl, case):
    rng = np.random.default_rng(40 + case)
    if case == 0:
        f, m = tiny_volume()
        frames = KEY
    else:
        T = int(rng.integers(2, 9))
        shape = (T, int(rng.integers(2, 9)), int(rng.integers(2, 40)), int(rng.integers(2, 200)))
        m = (rng.random(shape) < rng.uniform(0.0, 0.3)).astype(np.uint8)
        if case == 1:
            m[0] = 0  # an empty frame among the listed ones
        k = int(rng.integers(1, T + 1))
        frames = sorted(rng.choice(T, k, replace=False).tolist())
    dims = _dims(m)
    bits = torch.from_numpy(synth.pack_mask_rows(m).view(np.int64)).cuda()
    ids = fl.fhash_coreset_frames(bits, dims, frames)
    sub = np.zeros_like(m)
    sub[frames] = m[frames]
    want = coreset_ids(sub)
    got = ids.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, want)


def test_sampler_with_frame_times_and_box_bit_exact(fl):
    f, mask = tiny_volume()
    dims = _dims(mask)
    T = dims[3]
    frame_t = fl.fhash_key_frame_times(T, KEY)
    np.testing.assert_array_equal(frame_t, O.key_frame_times(T, KEY))
    box = OC.feature_boxes(mask)[T].tolist()
    cs = coreset_ids(mask)
    n = 5000 + 3
    fd = torch.from_numpy(f).cuda()
    csd = torch.from_numpy(cs.view(np.int64)).cuda()
    ftd = torch.from_numpy(frame_t).cuda()
    for kw_box in (None, box):
        pos = torch.empty(n, 4, device="cuda")
        tgt = torch.empty(n, device="cuda")
        fl.fhash_sample(77, 5, n, csd, cs.size, dims, fd, pos, tgt, frame_t=ftd, box=kw_box)
        pr, tr = O.sample_batch_frames(77, 5, n, f, cs, O.key_frame_times(T, KEY), kw_box)
        np.testing.assert_array_equal(pos.cpu().numpy(), pr)
        np.testing.assert_array_equal(tgt.cpu().numpy(), tr)


def test_render_between_key_frames_matches_oracle(fl):
    """A model over key frames, rendered at frames it was not trained on: the
    model's time coordinate is the frame time of t (the render state's t01),
    the occupancy that of the volume at t."""
    f, mask = tiny_volume()
    dims = _dims(mask)
    T = dims[3]
    res = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 4]]   # finest temporal level = 4 key frames
    g = O.Grid(np.array(res), 2, mask)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    idx, _, _dir, _ = fl.fhash_build_index(fl.grid_desc(res, 2), bits, dims)
    rng = np.random.default_rng(2)
    table = rng.uniform(-1, 1, (g.total_slots, 2)).astype(np.float32)
    width = [6, 32, 32, 1]
    params = synth.mlp_init(width, seed=3)
    params[-1] = 0.5
    tf = synth.transfer_function()
    tab_d, prm_d, tf_d = (torch.from_numpy(x).cuda() for x in (table, params, tf))
    mlp = fl.mlp_desc(width)
    frame_t = O.key_frame_times(T, KEY)
    W, H = 40, 30
    for t in (4.0, 6.5, 1.25):
        lo, hi = int(np.floor(t)), int(np.ceil(t))
        t01 = np.float32(frame_t[lo] + (t - lo) * (frame_t[hi] - frame_t[lo]))
        view = synth.orbit_view(dims, 0.8 + t, 0.3, W, H)
        ws = torch.empty(fl.fhash_render_state_bytes(W, H, dims), dtype=torch.uint8,
                         device="cuda")
        rgba = torch.empty(H, W, 4, device="cuda")
        opts = fl.render_opts()
        st = fl.fhash_render_begin(fl.view_struct(view), t, W, H, bits, dims, ws, rgba)
        assert abs(st.t01 - t / (T - 1)) <= 1e-7
        st.t01 = float(t01)
        pos = torch.empty(W * H * 64, 4, device="cuda")
        y = torch.empty(W * H * 64, device="cuda")
        while st.n_alive > 0:
            pace = fl.fhash_render_pace(W * H, st.n_alive, opts.arm_max)
            ns = fl.fhash_render_march(st, opts, pace, pos, W * H * 64)
            if ns:
                assert bool((pos[:ns, 3] == float(t01)).all())
                fl.fhash_fused_fwd(idx, mlp, pos[:ns], ns, tab_d, prm_d, y)
            fl.fhash_render_composite(st, y, tf_d, opts, rgba)
        ref, amb, ev, pix = O.render(g, table.astype(np.float64), width,
                                     params.astype(np.float64), mask, view, t, tf, W, H,
                                     pixel_stats=True, t01=float(t01))
        bound, amb = render_bound(pix, tf)
        err = np.abs(rgba.cpu().numpy() - ref)
        assert (err <= bound).all(), (t, float((err - bound).max()))
        assert ref[..., 3].max() > 0.3


def test_dense_fbb_fold_model_trains_like_the_oracle(fl):
    f, mask = tiny_volume()
    dims = _dims(mask)
    T = dims[3]
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    box = fl.fhash_feature_boxes(bits, dims).cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(box, OC.feature_boxes(mask))
    fbb = box[T].tolist()
    size = [fbb[3] - fbb[0] + 1, fbb[4] - fbb[1] + 1, fbb[5] - fbb[2] + 1, len(KEY)]
    res = fl.fhash_fold_resolutions(size, 2)
    assert res == O.fold_resolutions(size, 2)[::-1].tolist()
    F = 2
    idx, counts = fl.fhash_dense_index(fl.grid_desc(res, F))
    g = O.Grid(np.array(res), F, None)
    assert counts == g.counts
    width = [len(res) * F, 32, 32, 1]
    params = synth.mlp_init(width, seed=8)
    rng = np.random.default_rng(9)
    table = rng.uniform(-1, 1, (g.total_slots, F)).astype(np.float32)
    frame_t = fl.fhash_key_frame_times(T, KEY)
    sub = np.zeros_like(mask)
    sub[KEY] = mask[KEY]
    cs = fl.fhash_coreset_frames(bits, dims, KEY)
    n = 4096
    pos = torch.empty(n, 4, device="cuda")
    tgt = torch.empty(n, device="cuda")
    fl.fhash_sample(2001, 1, n, cs, cs.numel(), dims, torch.from_numpy(f).cuda(), pos, tgt,
                    frame_t=torch.from_numpy(frame_t).cuda(), box=fbb)
    pr, tr = O.sample_batch_frames(2001, 1, n, f, coreset_ids(sub), O.key_frame_times(T, KEY),
                                   fbb)
    np.testing.assert_array_equal(pos.cpu().numpy(), pr)
    # every key-frame sample sits on a vertex of the finest temporal level
    c = np.array([O.locate(float(v), len(KEY)) for v in pr[:64, 3]])
    assert (np.isin(c[:, 1], [0.0, 1.0])).all()
    enc, emag = O.encode_fwd(g, pr, table.astype(np.float64))
    y, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    L, dy = O.mse(y[:, 0], tr.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tr)) / n
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                         x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pr, denc)
    _, dtm = O.encode_bwd(g, pr, dencm)
    dt = torch.zeros(g.total_slots, F, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl.fhash_fused_train(idx, fl.mlp_desc(width), pos, tgt, n, torch.from_numpy(table).cuda(),
                         torch.from_numpy(params).cuda(), dt, dp, loss)
    assert (np.abs(dt.cpu().numpy() - dt_ref) <= RTOL * dtm + ATOL).all()
    assert (np.abs(dp.cpu().numpy() - dp_ref) <= RTOL * dpm + ATOL).all()
    assert abs(loss.item() - L * n) <= 1e-4 * L * n
