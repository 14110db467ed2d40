"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Integer outputs (index, sampler ids/positions) must match bit-exactly.  FP32
outputs must satisfy |gpu - oracle| <= 1e-5 * mag + atol, where mag is the
oracle's sum of term magnitudes (the scale of any FP32 evaluation order's
rounding error) and atol = 1e-12.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import coreset_ids, tiny_volume

pytestmark = pytest.mark.gpu

RTOL = 1e-5
ATOL = 1e-12


def _lib():
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return _lib()


def _assert_close(gpu, ref, mag, what, rtol=RTOL, atol=ATOL):
    gpu = np.asarray(gpu, np.float64)
    err = np.abs(gpu - ref)
    tol = rtol * mag + atol
    bad = err > tol
    if bad.any():
        i = np.argmax(err - tol)
        raise AssertionError(f"{what}: {bad.sum()} / {bad.size} outside tolerance; worst at {i}: "
                             f"gpu={gpu.ravel()[i]!r} ref={ref.ravel()[i]!r} "
                             f"mag={mag.ravel()[i]!r}")


TINY_RES = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]


@pytest.fixture(scope="module")
def tiny():
    f, mask = tiny_volume()
    return f, mask


def _dims(mask):
    T, Sz, Sy, Sx = mask.shape
    return [Sx, Sy, Sz, T]


def _build(fl, res, F, mask):
    grid = fl.grid_desc(res, F)
    if mask is None:
        return fl.fhash_build_index(grid, None, [2, 2, 2, 2])
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    return fl.fhash_build_index(grid, bits, _dims(mask))


def _decode_dir(idx, dir_t, res):
    """Vertex -> slot maps from the directory (row-padded bitmap + rank words,
    entries of one x word adjacent over y)."""
    d = dir_t.cpu().numpy().view(np.uint64)
    maps = []
    for l, (Rx, Ry, Rz, Rt) in enumerate(res):
        Wv = (Rx + 63) // 64
        off = int(idx.dir_offset[l])
        # stored ((t*Rz + z)*Wv + word)*Ry + y: bring it to row-major (t, z, y), word
        ent = d[off: off + Rt * Rz * Ry * Wv].reshape(Rt * Rz, Wv, Ry, 2)
        ent = ent.transpose(0, 2, 1, 3).reshape(Rt * Rz * Ry, Wv, 2)
        bits, rank = ent[..., 0], ent[..., 1]
        x = np.arange(Rx)
        w, b = x // 64, (x % 64).astype(np.uint64)
        word = bits[:, w]
        act = ((word >> b) & np.uint64(1)).astype(bool)
        below = word & ((np.uint64(1) << b) - np.uint64(1))
        pc = np.array([[bin(int(v)).count("1") for v in row] for row in below], np.int64)
        slot = rank[:, w].astype(np.int64) + pc
        slot[~act] = -1
        maps.append(slot.ravel())
    return maps


# ----------------------------------------------------------------------------- index
def test_index_tiny_bit_exact(fl, tiny):
    f, mask = tiny
    idx, counts, dir_t, _ = _build(fl, TINY_RES, 2, mask)
    g = O.Grid(np.array(TINY_RES), 2, mask)
    assert counts == g.counts
    got = _decode_dir(idx, dir_t, TINY_RES)
    for l in range(len(TINY_RES)):
        np.testing.assert_array_equal(got[l], g.maps[l], err_msg=f"level {l}")
    assert [int(idx.slot_offset[l]) for l in range(5)] == g.slot_offset.tolist()


@pytest.mark.parametrize("trial", range(12))
def test_index_random_grids_bit_exact(fl, trial):
    rng = np.random.default_rng(100 + trial)
    S = rng.integers(2, 90, size=4)
    S[3] = rng.integers(2, 9)
    mask = (rng.random((S[3], S[2], S[1], S[0])) < rng.uniform(0.001, 0.3)).astype(np.uint8)
    L = int(rng.integers(1, 5))
    res = [[int(rng.integers(2, 70)) for _ in range(3)] + [int(rng.integers(2, 10))]
           for _ in range(L)]
    if trial == 0:
        mask[:] = 0  # empty feature region: no active vertex anywhere
    if trial == 1:
        res = [[65, 129, 3, 2]]  # x-pairs straddling directory words
    L = len(res)
    idx, counts, dir_t, _ = _build(fl, res, 1, mask)
    g = O.Grid(np.array(res), 1, mask)
    assert counts == g.counts
    got = _decode_dir(idx, dir_t, res)
    for l in range(L):
        np.testing.assert_array_equal(got[l], g.maps[l], err_msg=f"level {l}")


def test_dense_index_counts(fl):
    idx, counts, _, _ = _build(fl, TINY_RES, 2, None)
    assert idx.active == 0
    assert counts == [int(np.prod(r)) for r in TINY_RES]


# ----------------------------------------------------------------------------- encoding
def _probe_positions(n, seed):
    p = synth.probe_points(n, seed)
    p[:8] = [[0, 0, 0, 0], [1, 1, 1, 1], [0.5, 0.5, 0.5, 0.5], [-0.2, 1.3, 0.3, 2.0],
             [np.nan, 0.1, 0.2, 0.3], [1 / 3, 2 / 3, 1 / 7, 3 / 7], [0.999999, 1e-7, 0.25, 0.75],
             [0.125, 0.0625, 0.03125, 1.0]]
    return p.astype(np.float32)


@pytest.mark.parametrize("active", [True, False])
@pytest.mark.parametrize("F", [1, 2, 4, 8])
def test_encode_fwd_bwd(fl, tiny, active, F):
    f, mask = tiny
    m = mask if active else None
    idx, counts, dir_t, _ = _build(fl, TINY_RES, F, m)
    g = O.Grid(np.array(TINY_RES), F, m)
    rows = g.total_slots
    rng = np.random.default_rng(F)
    table = rng.uniform(-1, 1, size=(rows, F)).astype(np.float32)
    n = 3000 + 77  # ragged tail
    pos = _probe_positions(n, 7 + F)
    ref, mag = O.encode_fwd(g, pos, table.astype(np.float64))
    pos_d = torch.from_numpy(pos).cuda()
    tab_d = torch.from_numpy(table).cuda()
    enc = torch.full((n, len(TINY_RES) * F), np.nan, device="cuda")
    fl.fhash_encode_fwd(idx, pos_d, n, tab_d, enc)
    _assert_close(enc.cpu().numpy(), ref, mag, "encode_fwd")
    # backward
    d_enc = rng.normal(size=(n, len(TINY_RES) * F)).astype(np.float32)
    dref, dmag = O.encode_bwd(g, pos, d_enc.astype(np.float64))
    d_tab = torch.zeros(rows, F, device="cuda")
    fl.fhash_encode_bwd(idx, pos_d, n, torch.from_numpy(d_enc).cuda(), d_tab)
    _assert_close(d_tab.cpu().numpy(), dref, dmag, "encode_bwd")


def test_encode_f16_table(fl, tiny):
    f, mask = tiny
    idx, counts, dir_t, _ = _build(fl, TINY_RES, 2, mask)
    g = O.Grid(np.array(TINY_RES), 2, mask)
    table = np.random.default_rng(3).uniform(-1, 1, size=(g.total_slots, 2)).astype(np.float16)
    pos = _probe_positions(2000, 3)
    ref, mag = O.encode_fwd(g, pos, table.astype(np.float64))
    enc = torch.empty(2000, 8, device="cuda")
    fl.fhash_encode_fwd(idx, torch.from_numpy(pos).cuda(), 2000, torch.from_numpy(table).cuda(),
                        enc)
    _assert_close(enc.cpu().numpy(), ref, mag, "encode_fwd f16")


def test_encode_empty_batch_and_empty_table(fl):
    mask = np.zeros((2, 5, 5, 5), np.uint8)
    idx, counts, dir_t, _ = _build(fl, [[3, 3, 3, 2]], 2, mask)
    assert counts == [0]
    enc = torch.full((10, 2), 7.0, device="cuda")
    pos = torch.rand(10, 4, device="cuda")
    fl.fhash_encode_fwd(idx, pos, 10, torch.zeros(1, 2, device="cuda"), enc)
    assert (enc == 0).all()
    fl.fhash_encode_fwd(idx, pos, 0, torch.zeros(1, 2, device="cuda"), enc)


# ----------------------------------------------------------------------------- MLP
@pytest.mark.parametrize("width", [[8, 32, 32, 1], [32, 64, 64, 1], [32, 64, 64, 64, 1],
                                   [5, 32, 1], [20, 64, 64, 1]])
def test_mlp_fwd_bwd(fl, width):
    rng = np.random.default_rng(len(width) * 100 + width[0])
    P = O.mlp_num_params(width)
    params = np.concatenate([
        np.concatenate([rng.uniform(-1, 1, width[k + 1] * width[k]) / np.sqrt(width[k]),
                        rng.uniform(-0.1, 0.1, width[k + 1])]) for k in range(len(width) - 1)
    ]).astype(np.float32)
    n = 1000 + 13
    x = rng.normal(size=(n, width[0])).astype(np.float32)
    dy = rng.normal(size=(n, 1)).astype(np.float32)
    y_ref, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), x.astype(np.float64))
    mlp = fl.mlp_desc(width)
    prm = torch.from_numpy(params).cuda()
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(n, device="cuda")
    fl.fhash_mlp_fwd(mlp, prm, xd, n, y)
    _assert_close(y.cpu().numpy(), y_ref[:, 0], ymag[:, 0], "mlp_fwd")
    dp_ref, dx_ref, dpm, dxm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy.astype(np.float64), n)
    dp = torch.zeros(P, device="cuda")
    dx = torch.empty(n, width[0], device="cuda")
    fl.fhash_mlp_bwd(mlp, prm, xd, torch.from_numpy(dy[:, 0].copy()).cuda(), n, dp, dx)
    _assert_close(dp.cpu().numpy(), dp_ref, dpm, "mlp_bwd dparams")
    _assert_close(dx.cpu().numpy(), dx_ref, dxm, "mlp_bwd dx")


# ----------------------------------------------------------------------------- fused
def _mlp_params(width, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([
        np.concatenate([rng.uniform(-1, 1, width[k + 1] * width[k]) / np.sqrt(width[k]),
                        rng.uniform(-0.1, 0.1, width[k + 1])]) for k in range(len(width) - 1)
    ]).astype(np.float32)


@pytest.mark.parametrize("F,hidden", [(2, [32, 32]), (1, [64, 64]), (4, [64, 64, 64])])
def test_fused_paths(fl, tiny, F, hidden):
    f, mask = tiny
    idx, counts, dir_t, _ = _build(fl, TINY_RES, F, mask)
    g = O.Grid(np.array(TINY_RES), F, mask)
    width = [len(TINY_RES) * F] + hidden + [1]
    rng = np.random.default_rng(F)
    table = rng.uniform(-1, 1, size=(g.total_slots, F)).astype(np.float32)
    params = _mlp_params(width, F + 10)
    n = 2048 + 5
    pos = _probe_positions(n, 20 + F)
    tgt = rng.random(n).astype(np.float32)
    enc, emag = O.encode_fwd(g, pos, table.astype(np.float64))
    y_ref, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    mlp = fl.mlp_desc(width)
    pos_d, tab_d = torch.from_numpy(pos).cuda(), torch.from_numpy(table).cuda()
    prm = torch.from_numpy(params).cuda()
    y = torch.empty(n, device="cuda")
    fl.fhash_fused_fwd(idx, mlp, pos_d, n, tab_d, prm, y)
    _assert_close(y.cpu().numpy(), y_ref[:, 0], ymag[:, 0], "fused_fwd")
    # backward with a given dy
    dy = rng.normal(size=n).astype(np.float32)
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy.astype(np.float64).reshape(-1, 1), n, x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    dt = torch.zeros(g.total_slots, F, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    fl.fhash_fused_bwd(idx, mlp, pos_d, n, tab_d, prm, torch.from_numpy(dy).cuda(), dt, dp)
    _assert_close(dp.cpu().numpy(), dp_ref, dpm, "fused_bwd dparams")
    _assert_close(dt.cpu().numpy(), dt_ref, dtm, "fused_bwd dtable")
    # forward + MSE + backward
    L_ref, dy_ref = O.mse(y_ref[:, 0], tgt.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tgt)) / n
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy_ref.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                         x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    dt.zero_()
    dp.zero_()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl.fhash_fused_train(idx, mlp, pos_d, torch.from_numpy(tgt).cuda(), n, tab_d, prm, dt, dp,
                         loss)
    _assert_close(dp.cpu().numpy(), dp_ref, dpm, "fused_train dparams")
    _assert_close(dt.cpu().numpy(), dt_ref, dtm, "fused_train dtable")
    lmag = float(((ymag[:, 0] + np.abs(tgt)) * np.abs(y_ref[:, 0] - tgt)).sum()) * 2
    assert abs(loss.item() - L_ref * n) <= RTOL * lmag + ATOL


# ----------------------------------------------------------------------------- optimiser
def test_adam_step(fl):
    rng = np.random.default_rng(5)
    n = 100003
    p = rng.normal(size=n).astype(np.float32)
    g = (rng.normal(size=n) * np.logspace(-6, 1, n)).astype(np.float32)
    g[::11] = 0.0
    m = (rng.normal(size=n) * 0.01).astype(np.float32)
    v = (rng.random(n) * 1e-4).astype(np.float32)
    step = 7
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    O.adam(pr, g.astype(np.float64), mr, vr, 0.01, 0.9, 0.999, 1e-8, step)
    pd, gd, md, vd = [torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v)]
    sh = torch.empty(n, dtype=torch.float16, device="cuda")
    o = fl.AdamDesc()
    o.lr, o.beta1, o.beta2, o.eps, o.step, o.grad_scale = 0.01, 0.9, 0.999, 1e-8, step, 1.0
    fl.fhash_step(o, pd, gd, md, vd, shadow=sh)
    _assert_close(md.cpu().numpy(), mr, np.abs(mr) + 0.1 * np.abs(g), "adam m")
    _assert_close(vd.cpu().numpy(), vr, np.abs(vr), "adam v")
    _assert_close(pd.cpu().numpy(), pr, np.abs(pr) * 0.1 + 0.01, "adam p")
    assert (gd == 0).all()
    np.testing.assert_array_equal(sh.cpu().numpy(), pd.cpu().numpy().astype(np.float16))
    # overflow flag: update skipped, grads still zeroed
    gd.copy_(torch.from_numpy(g))
    before = pd.clone()
    flag = torch.ones(1, dtype=torch.int32, device="cuda")
    fl.fhash_step(o, pd, gd, md, vd, found_inf=flag)
    assert torch.equal(before, pd) and (gd == 0).all()


# ----------------------------------------------------------------------------- touched segments
@pytest.mark.parametrize("path", ["fused_train", "fused_bwd", "encode_bwd"])
def test_touched_segment_flags_are_exact(fl, tiny, path):
    """Flags are set exactly for the segments (16 floats) holding a slot that an
    active corner of some sample wrote, at or after float `begin` (from the
    oracle's corner slots)."""
    f, mask = tiny
    F = 2
    idx, counts, dir_t, _ = _build(fl, TINY_RES, F, mask)
    g = O.Grid(np.array(TINY_RES), F, mask)
    rows = g.total_slots
    begin = int(g.slot_offset[2]) * F // 16 * 16 - 16
    nseg = (rows * F + 15) // 16
    flags = torch.zeros(nseg, dtype=torch.uint8, device="cuda")
    t = fl.touch_desc(flags, begin, rows * F)
    n = 777
    pos = _probe_positions(n, 91)
    pos_d = torch.from_numpy(pos).cuda()
    width = [8, 32, 32, 1]
    prm = torch.from_numpy(_mlp_params(width, 3)).cuda()
    tab = torch.from_numpy(np.random.default_rng(4).uniform(-1, 1, (rows, F))
                           .astype(np.float32)).cuda()
    dt = torch.zeros(rows, F, device="cuda")
    dp = torch.zeros(prm.numel(), device="cuda")
    mlp = fl.mlp_desc(width)
    if path == "fused_train":
        tgt = torch.rand(n, device="cuda")
        fl.fhash_fused_train(idx, mlp, pos_d, tgt, n, tab, prm, dt, dp, touch=t)
    elif path == "fused_bwd":
        dy = torch.randn(n, device="cuda")
        fl.fhash_fused_bwd(idx, mlp, pos_d, n, tab, prm, dy, dt, dp, touch=t)
    else:
        de = torch.randn(n, len(TINY_RES) * F, device="cuda")
        fl.fhash_encode_bwd(idx, pos_d, n, de, dt, touch=t)
    slots, _ = O.corners(g, pos)
    sl = slots[slots >= 0] * F
    exp = np.zeros(nseg, bool)
    exp[np.unique(sl[sl >= begin] // 16)] = True
    got = flags.cpu().numpy() != 0
    assert np.array_equal(got, exp), (int((got != exp).sum()), int(exp.sum()))
    # every nonzero gradient float at or after begin lies in a flagged segment
    nz = np.flatnonzero(dt.cpu().numpy().ravel() != 0)
    nz = nz[nz >= begin]
    assert got[nz // 16].all()


def test_tracked_adam_equals_untracked(fl):
    """A tracked step (gradient read only in flagged segments of [begin, end),
    always read outside) gives bit for bit the untracked step when the gradient
    is zero in every unflagged segment; it resets the gradient and the flags."""
    rng = np.random.default_rng(8)
    n = 4 * 65536 + 3
    begin, end = 16 * 1000, n - 4093
    nseg = (end + 15) // 16
    seg_on = rng.random(nseg) < 0.1
    g = (rng.normal(size=n) * np.logspace(-6, 1, n)).astype(np.float32)
    fidx = np.arange(n)
    in_range = (fidx >= begin) & (fidx < end)
    off = in_range & ~seg_on[np.minimum(fidx // 16, nseg - 1)]
    g[off] = 0.0
    g[::13] = 0.0
    p = rng.normal(size=n).astype(np.float32)
    m = (rng.normal(size=n) * 0.01).astype(np.float32)
    v = (rng.random(n) * 1e-4).astype(np.float32)
    o = fl.AdamDesc()
    o.lr, o.beta1, o.beta2, o.eps, o.step, o.grad_scale = 0.01, 0.9, 0.999, 1e-8, 3, 0.5
    outs = []
    for tracked in (False, True):
        pd, gd, md, vd = [torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v)]
        sh = torch.empty(n, dtype=torch.float16, device="cuda")
        touch = None
        if tracked:
            flags = torch.from_numpy(seg_on.astype(np.uint8)).cuda()
            flags[: begin // 16] = 1   # outside the range: must stay untouched
            touch = fl.touch_desc(flags, begin, end)
        fl.fhash_step(o, pd, gd, md, vd, shadow=sh, touch=touch)
        assert (gd == 0).all()
        if tracked:
            fc = flags.cpu().numpy()
            assert (fc[begin // 16:] == 0).all() and (fc[: begin // 16] == 1).all()
        outs.append([x.cpu() for x in (pd, md, vd, sh)])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_check_finite_and_cast(fl):
    x = torch.randn(10007, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    fl.fhash_check_finite(x, flag)
    assert flag.item() == 0
    x[5000] = float("inf")
    fl.fhash_check_finite(x, flag)
    assert flag.item() == 1
    y = torch.randn(1001, device="cuda")
    b = torch.empty(1001, dtype=torch.bfloat16, device="cuda")
    fl.fhash_cast(y, b)
    assert torch.equal(b, y.to(torch.bfloat16))


# ----------------------------------------------------------------------------- sampler / reductions
@pytest.mark.parametrize("use_coreset", [True, False])
def test_sampler_bit_exact(fl, tiny, use_coreset):
    f, mask = tiny
    cs = coreset_ids(mask) if use_coreset else None
    n = 4096 + 3
    pos_r, tgt_r = O.sample_batch(2001, 17, n, f, cs)
    fd = torch.from_numpy(f).cuda()
    csd = torch.from_numpy(cs.view(np.int64)).cuda() if use_coreset else None
    M = cs.size if use_coreset else f.size
    pos = torch.empty(n, 4, device="cuda")
    tgt = torch.empty(n, device="cuda")
    fl.fhash_sample(2001, 17, n, csd, M, _dims(mask), fd, pos, tgt)
    np.testing.assert_array_equal(pos.cpu().numpy(), pos_r)
    np.testing.assert_array_equal(tgt.cpu().numpy(), tgt_r)


def test_sq_err_sum(fl):
    rng = np.random.default_rng(9)
    y = rng.random(123457).astype(np.float32)
    v = rng.random(123457).astype(np.float32)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl.fhash_sq_err_sum(torch.from_numpy(y).cuda(), torch.from_numpy(v).cuda(), y.size, out)
    ref = float(((y.astype(np.float64) - v) ** 2).sum())
    assert abs(out.item() - ref) <= 1e-12 * ref


# ----------------------------------------------------------------------------- one training step
def _step1_bounds(g, gmag, lr, eps):
    """Interval of the oracle's first Adam update over g +- tolerance."""
    tol = RTOL * gmag + ATOL
    lo, hi = g - tol, g + tol

    def d(q):
        return -lr * q / (np.abs(q) + eps)
    a, b = d(lo), d(hi)
    return np.minimum(a, b), np.maximum(a, b)


def test_one_training_step_tiny(fl, tiny):
    """Tiny workload: 4096 uniformly sampled voxels, fused MSE fwd+bwd, one Adam
    step; replayed by the oracle on the identical Philox batch."""
    from paper_2507_03836_amd.model import FHashConfig, FHashModel
    f, mask = tiny
    cfg = FHashConfig(res=TINY_RES, n_features=2, hidden=32, n_hidden=2)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    g = O.Grid(np.array(TINY_RES), 2, mask)
    table0 = synth.table_init(g.total_slots, 2)
    mlp0 = synth.mlp_init(cfg.width)
    model = FHashModel(cfg, bits, _dims(mask), table_init=torch.from_numpy(table0),
                       mlp_init=torch.from_numpy(mlp0))
    n = 4096
    pos = torch.empty(n, 4, device="cuda")
    tgt = torch.empty(n, device="cuda")
    fd = torch.from_numpy(f).cuda()
    fl.fhash_sample(2001, 1, n, None, f.size, _dims(mask), fd, pos, tgt)
    model.train_step(pos, tgt)
    # oracle replay
    pos_r, tgt_r = O.sample_batch(2001, 1, n, f)
    np.testing.assert_array_equal(pos.cpu().numpy(), pos_r)
    enc, emag = O.encode_fwd(g, pos_r, table0.astype(np.float64))
    y, acts, ymag = O.mlp_fwd(cfg.width, mlp0.astype(np.float64), enc, x_mag=emag)
    L, dy = O.mse(y[:, 0], tgt_r.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tgt_r)) / n
    dp, denc, dpm, dencm = O.mlp_bwd(cfg.width, mlp0.astype(np.float64), acts, dy.reshape(-1, 1),
                                     n, dy_mag=dym.reshape(-1, 1), x_mag=emag)
    dt, _ = O.encode_bwd(g, pos_r, denc)
    _, dtm = O.encode_bwd(g, pos_r, dencm)
    lr, eps = cfg.lr, cfg.eps
    for name, p0, gr, gm, got in (
            ("table", table0.ravel(), dt.ravel(), dtm.ravel(), model.table.cpu().numpy()),
            ("mlp", mlp0, dp, dpm, model.mlp_params.cpu().numpy())):
        lo, hi = _step1_bounds(gr, gm, lr, eps)
        delta = got.astype(np.float64) - p0.astype(np.float64)
        # FP32 rounding of the update and of p + update
        slack = 2.4e-7 * (np.abs(p0) + np.maximum(np.abs(lo), np.abs(hi))) + 1e-12
        bad = (delta < lo - slack) | (delta > hi + slack)
        assert not bad.any(), (name, int(bad.sum()), np.argwhere(bad)[:5].ravel())
    assert (model.grads == 0).all()
    assert abs(model.loss_sum.item() - L * n) <= 1e-4 * L * n


# ----------------------------------------------------------------------------- sort + merged scatter
def _morton_keys(pos):
    q = np.minimum((pos.astype(np.float32) * np.float32(256.0)).astype(np.int64), 255)
    q = np.maximum(q, 0)
    key = np.zeros(len(pos), np.int64)
    for d in range(4):
        for b in range(8):
            key |= ((q[:, d] >> b) & 1) << (4 * b + d)
    return key


def test_sort_samples_is_a_morton_ordered_permutation(fl):
    n = 100003
    rng = np.random.default_rng(11)
    pos = rng.random((n, 4), dtype=np.float32)
    tgt = np.arange(n, dtype=np.float32)
    pd, td = torch.from_numpy(pos).cuda(), torch.from_numpy(tgt).cuda()
    fl.fhash_sort_samples(pd, td, n)
    ps, ts = pd.cpu().numpy(), td.cpu().numpy()
    idx = ts.astype(np.int64)
    np.testing.assert_array_equal(np.sort(idx), np.arange(n))  # a permutation
    np.testing.assert_array_equal(ps, pos[idx])                 # pairs kept together
    k = _morton_keys(ps)
    assert (np.diff(k) >= 0).all()
    # stable: equal keys keep their input order
    same = np.diff(k) == 0
    assert (np.diff(idx)[same] > 0).all()


@pytest.mark.parametrize("F,hidden", [(2, [32, 32]), (1, [64, 64]), (4, [64, 64, 64])])
def test_fused_train_sorted_merged_scatter(fl, tiny, F, hidden):
    """Sorted batch with FHASH_SAMPLES_SORTED: at the coarse levels a corner
    that every sample of a scatter pass hits on one slot is summed across the
    pass before one atomic (64 lanes of one level at F = 2 and 4, 32 at F = 1);
    the same gradients as the oracle up to FP32 summation order.  The batch
    ends in a ragged block (n = 16 k + 9)."""
    f, mask = tiny
    width = [len(TINY_RES) * F] + hidden + [1]
    idx, counts, dir_t, _ = _build(fl, TINY_RES, F, mask)
    g = O.Grid(np.array(TINY_RES), F, mask)
    rng = np.random.default_rng(21 + F)
    table = rng.uniform(-1, 1, size=(g.total_slots, F)).astype(np.float32)
    params = _mlp_params(width, 22 + F)
    n = 4096 + 9
    pos0, tgt0 = O.sample_batch(5, 3, n, f, coreset_ids(mask))
    pd, td = torch.from_numpy(pos0).cuda(), torch.from_numpy(tgt0).cuda()
    fl.fhash_sort_samples(pd, td, n)
    pos, tgt = pd.cpu().numpy(), td.cpu().numpy()
    enc, emag = O.encode_fwd(g, pos, table.astype(np.float64))
    y, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    L, dy = O.mse(y[:, 0], tgt.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tgt)) / n
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                         x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    dt = torch.zeros(g.total_slots, F, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    mlp = fl.mlp_desc(width)
    fl.fhash_fused_train(idx, mlp, pd, td, n, torch.from_numpy(table).cuda(),
                         torch.from_numpy(params).cuda(), dt, dp, flags=fl.SAMPLES_SORTED)
    _assert_close(dt.cpu().numpy(), dt_ref, dtm, "sorted fused_train dtable")
    _assert_close(dp.cpu().numpy(), dp_ref, dpm, "sorted fused_train dparams")


COARSE_RES = [[4, 4, 4, 2], [8, 8, 8, 3], [24, 24, 24, 2], [32, 32, 32, 8]]


@pytest.mark.parametrize("sort", [True, False])
@pytest.mark.parametrize("F,hidden", [(2, [32, 32]), (1, [64, 64]), (4, [64, 64, 64])])
def test_fused_coarse_lds_scatter(fl, tiny, F, hidden, sort):
    """FHASH_COARSE_LDS: the levels with at most one cell per sample (here
    levels 0-2 of 4) leave the fused kernel through the workspace and are
    summed per chunk of 2048 samples in LDS before their atomics.  Level 2's
    vertex box (24^3 x 2 vertices) does not fit the LDS image for a chunk of
    unsorted draws, nor at F = 4, so those chunks take the direct path; the
    batch ends in a ragged chunk.  fused_train and fused_bwd against the FP64
    oracle at the FP32 tolerance."""
    f, mask = tiny
    width = [len(COARSE_RES) * F] + hidden + [1]
    idx, counts, dir_t, _ = _build(fl, COARSE_RES, F, mask)
    g = O.Grid(np.array(COARSE_RES), F, mask)
    rng = np.random.default_rng(41 + F)
    table = rng.uniform(-1, 1, size=(g.total_slots, F)).astype(np.float32)
    params = _mlp_params(width, 42 + F)
    n = 8 * 2048 + 9
    pos0, tgt0 = O.sample_batch(7, 2, n, f, coreset_ids(mask))
    pd, td = torch.from_numpy(pos0).cuda(), torch.from_numpy(tgt0).cuda()
    if sort:
        fl.fhash_sort_samples(pd, td, n)
    pos, tgt = pd.cpu().numpy(), td.cpu().numpy()
    enc, emag = O.encode_fwd(g, pos, table.astype(np.float64))
    y, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    L, dy = O.mse(y[:, 0], tgt.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tgt)) / n
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                         x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    mlp = fl.mlp_desc(width)
    tab_d, prm = torch.from_numpy(table).cuda(), torch.from_numpy(params).cuda()
    dt = torch.zeros(g.total_slots, F, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl.fhash_fused_train(idx, mlp, pd, td, n, tab_d, prm, dt, dp, loss, flags=fl.COARSE_LDS)
    _assert_close(dt.cpu().numpy(), dt_ref, dtm, "coarse-LDS fused_train dtable")
    _assert_close(dp.cpu().numpy(), dp_ref, dpm, "coarse-LDS fused_train dparams")
    lmag = float(((ymag[:, 0] + np.abs(tgt)) * np.abs(y[:, 0] - tgt)).sum()) * 2
    assert abs(loss.item() - L * n) <= RTOL * lmag + ATOL
    # the same through fhash_fused_bwd with a given output gradient
    dyg = rng.normal(size=n).astype(np.float32)
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dyg.astype(np.float64).reshape(-1, 1), n, x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    dt.zero_()
    dp.zero_()
    fl.fhash_fused_bwd(idx, mlp, pd, n, tab_d, prm, torch.from_numpy(dyg).cuda(), dt, dp,
                       flags=fl.COARSE_LDS)
    _assert_close(dt.cpu().numpy(), dt_ref, dtm, "coarse-LDS fused_bwd dtable")
    _assert_close(dp.cpu().numpy(), dp_ref, dpm, "coarse-LDS fused_bwd dparams")
