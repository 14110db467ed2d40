"""GPU parity at the encoding width the production workloads run: 16 levels x
2 features = 32 decoder inputs (two 16-feature blocks of the fused kernels),
decoders 32-64-64-1 and 32-64-64-64-1, also ragged (12 levels x 2 = 24 inputs,
padded to 32) and F = 4 (8 levels x 4).  The level grids are small enough for
the FP64 oracle to enumerate every level, and the finest levels span more than
64 vertices in x so vertex pairs straddle directory words.

Every fused entry point (forward, backward with a given dy, forward + MSE +
backward, the merged scatter of sorted batches, FP16 table reads and
the FP16-MFMA inference decoder) is compared element by element with the
oracle at |gpu - oracle| <= 1e-5 * mag + 1e-12 (mag = the oracle's sum of term
magnitudes); the FP16 decoder against its layer-by-layer rounding bound.  The
deferred Adam is compared with the dense update bit for bit at this width.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import coreset_ids, tiny_volume

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-12
U16 = 2.0 ** -11


def _wide_res(L, rmax=(70, 24, 20, 8)):
    """L levels, geometric from 2 to rmax per dimension (x beyond 64 vertices)."""
    out = []
    for l in range(L):
        out.append([max(2, int(np.floor(2.0 * (r / 2.0) ** (l / (L - 1)) + 0.5))) for r in rmax])
    return out


WIDE16 = _wide_res(16)
WIDE12 = _wide_res(12)
WIDE8 = _wide_res(8)


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


@pytest.fixture(scope="module")
def vol():
    return tiny_volume()


def _dims(mask):
    T, Sz, Sy, Sx = mask.shape
    return [Sx, Sy, Sz, T]


def _close(gpu, ref, mag, what):
    gpu = np.asarray(gpu, np.float64)
    err = np.abs(gpu - ref)
    tol = RTOL * mag + ATOL
    bad = err > tol
    if bad.any():
        i = int(np.argmax(err - tol))
        raise AssertionError(f"{what}: {int(bad.sum())} / {bad.size} outside tolerance; worst at "
                             f"{i}: gpu={gpu.ravel()[i]!r} ref={ref.ravel()[i]!r} "
                             f"mag={mag.ravel()[i]!r}")


def _params(width, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([
        np.concatenate([rng.uniform(-1, 1, width[k + 1] * width[k]) / np.sqrt(width[k]),
                        rng.uniform(-0.1, 0.1, width[k + 1])]) for k in range(len(width) - 1)
    ]).astype(np.float32)


def _positions(n, seed):
    p = synth.probe_points(n, seed)
    p[:6] = [[0, 0, 0, 0], [1, 1, 1, 1], [0.5, 0.5, 0.5, 0.5], [63.5 / 69, 0.3, 0.7, 0.2],
             [64 / 69, 1 / 23, 0.5, 1 / 7], [np.nan, 1.2, -0.1, 0.5]]
    return p.astype(np.float32)


def _setup(fl, vol, res, F, tdt):
    f, mask = vol
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    idx, counts, dir_t, _ = fl.fhash_build_index(fl.grid_desc(res, F), bits, _dims(mask))
    g = O.Grid(np.array(res), F, mask)
    assert counts == g.counts
    rng = np.random.default_rng(len(res) * 10 + F)
    table = rng.uniform(-1, 1, size=(g.total_slots, F)).astype(np.float32)
    if tdt == "f16":
        table = table.astype(np.float16)
    return idx, dir_t, g, table


CASES = [  # (levels, F, hidden layers, table dtype)
    (WIDE16, 2, [64, 64], "f32"),       # the 480x720x120x100 training kernel's shape
    (WIDE16, 2, [64, 64, 64], "f32"),   # the 432^3 x 60 training kernel's shape
    (WIDE16, 2, [64, 64, 64], "f16"),   # its mixed-precision table reads
    (WIDE12, 2, [64, 64], "f32"),       # 24 inputs padded to 32
    (WIDE8, 4, [64, 64], "f32"),        # F = 4 at 32 inputs
    (WIDE16, 2, [32, 32], "f32"),
]


@pytest.mark.parametrize("res,F,hidden,tdt", CASES,
                         ids=[f"L{len(c[0])}F{c[1]}H{len(c[2])}x{c[2][0]}-{c[3]}" for c in CASES])
def test_fused_wide_against_oracle(fl, vol, res, F, hidden, tdt):
    idx, dir_t, g, table = _setup(fl, vol, res, F, tdt)
    L = len(res)
    width = [L * F] + hidden + [1]
    params = _params(width, 100 + L + F + len(hidden))
    n = 4096 + 37  # several waves of 16-sample blocks and a ragged tail
    pos = _positions(n, 50 + L)
    rng = np.random.default_rng(L + F)
    tgt = rng.random(n).astype(np.float32)
    tab64 = table.astype(np.float64)
    enc, emag = O.encode_fwd(g, pos, tab64)
    y_ref, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    mlp = fl.mlp_desc(width)
    pos_d, tab_d = torch.from_numpy(pos).cuda(), torch.from_numpy(table).cuda()
    prm = torch.from_numpy(params).cuda()
    # forward
    y = torch.full((n,), np.nan, device="cuda")
    fl.fhash_fused_fwd(idx, mlp, pos_d, n, tab_d, prm, y)
    _close(y.cpu().numpy(), y_ref[:, 0], ymag[:, 0], "fused_fwd")
    # backward with a given dy
    dy = rng.normal(size=n).astype(np.float32)
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy.astype(np.float64).reshape(-1, 1), n, x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    dt = torch.zeros(g.total_slots, F, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    fl.fhash_fused_bwd(idx, mlp, pos_d, n, tab_d, prm, torch.from_numpy(dy).cuda(), dt, dp)
    _close(dp.cpu().numpy(), dp_ref, dpm, "fused_bwd d_params")
    _close(dt.cpu().numpy(), dt_ref, dtm, "fused_bwd d_table")
    # the second 16-feature block (levels 8..15 at F = 2) really received gradient
    hi = int(g.slot_offset[16 // F]) if L * F > 16 else None
    if hi is not None:
        assert np.abs(dt.cpu().numpy()[hi:]).sum() > 0
    # forward + MSE + backward
    L_ref, dy_ref = O.mse(y_ref[:, 0], tgt.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tgt)) / n
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy_ref.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                         x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    for flags in (0, fl.SAMPLES_SORTED):
        dt.zero_()
        dp.zero_()
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        fl.fhash_fused_train(idx, mlp, pos_d, torch.from_numpy(tgt).cuda(), n, tab_d, prm, dt,
                             dp, loss, flags=flags)
        _close(dp.cpu().numpy(), dp_ref, dpm, f"fused_train d_params (flags {flags})")
        _close(dt.cpu().numpy(), dt_ref, dtm, f"fused_train d_table (flags {flags})")
        lmag = float(((ymag[:, 0] + np.abs(tgt)) * np.abs(y_ref[:, 0] - tgt)).sum()) * 2
        assert abs(loss.item() - L_ref * n) <= RTOL * lmag + ATOL


def test_fused_train_wide_sorted_batch(fl, vol):
    """Coreset draws sorted by fhash_sort_samples, then the merge of equal
    slots ahead of the atomics, at 32 inputs and three hidden layers."""
    f, mask = vol
    idx, dir_t, g, table = _setup(fl, vol, WIDE16, 2, "f32")
    width = [32, 64, 64, 64, 1]
    params = _params(width, 77)
    n = 8192 + 5
    pos0, tgt0 = O.sample_batch(9, 4, n, f, coreset_ids(mask))
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
    dt = torch.zeros(g.total_slots, 2, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    fl.fhash_fused_train(idx, fl.mlp_desc(width), pd, td, n, torch.from_numpy(table).cuda(),
                         torch.from_numpy(params).cuda(), dt, dp, flags=fl.SAMPLES_SORTED)
    _close(dt.cpu().numpy(), dt_ref, dtm, "sorted fused_train d_table")
    _close(dp.cpu().numpy(), dp_ref, dpm, "sorted fused_train d_params")


@pytest.mark.parametrize("hidden", [[64, 64], [64, 64, 64]])
def test_fp16_decoder_wide_within_rounding_bound(fl, vol, hidden):
    """The FP16-MFMA inference decoder at 32 inputs (the serving kernel's shape)
    against the FP64 oracle, inside the bound built layer by layer from binary16
    rounding of every weight and hidden-layer input, FP32 accumulation and the
    1-Lipschitz ReLU; FP16 table reads as served."""
    idx, dir_t, g, table = _setup(fl, vol, WIDE16, 2, "f16")
    width = [32] + hidden + [1]
    params = synth.mlp_init(width, seed=43)
    n = 1 << 14
    pos = synth.probe_points(n, 4003).astype(np.float32)
    pd = torch.from_numpy(pos).cuda()
    tab_d, prm_d = torch.from_numpy(table).cuda(), torch.from_numpy(params).cuda()
    y16 = torch.empty(n, device="cuda")
    y32 = torch.empty(n, device="cuda")
    fl.fhash_fused_fwd(idx, fl.mlp_desc(width, fl.F16), pd, n, tab_d, prm_d, y16)
    fl.fhash_fused_fwd(idx, fl.mlp_desc(width), pd, n, tab_d, prm_d, y32)
    enc, emag = O.encode_fwd(g, pos, table.astype(np.float64))
    y64, _, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    _close(y32.cpu().numpy(), y64[:, 0], ymag[:, 0], "FP32 decoder, FP16 table")
    e = RTOL * emag + ATOL
    m = np.abs(enc) + e
    off = 0
    for k in range(len(width) - 1):
        W = params[off: off + width[k + 1] * width[k]].astype(np.float64).reshape(width[k + 1],
                                                                                 width[k])
        b = params[off + width[k + 1] * width[k]: off + width[k + 1] * (width[k] + 1)]
        off += width[k + 1] * (width[k] + 1)
        aW, ab = np.abs(W), np.abs(b.astype(np.float64))
        mag_next = m @ aW.T + ab
        if k < len(width) - 2:
            e = (e * (1 + 2 * U16) + 2 * U16 * m + 2.0 ** -25) @ aW.T + \
                2.0 ** -25 * m.sum(axis=1, keepdims=True) + RTOL * mag_next
        else:
            e = e @ aW.T + RTOL * mag_next
        m = mag_next + e
    err = np.abs(y16.cpu().numpy().astype(np.float64) - y64[:, 0])
    assert (err <= e[:, 0] + ATOL).all(), float((err - e[:, 0]).max())
    assert not torch.equal(y16, y32)


def test_lazy_equals_dense_wide(fl, vol):
    """Deferred Adam against the dense update at 16 levels x 2 features and the
    32-64-64-64-1 decoder: every forward value between steps and every
    parameter, moment and gradient after the flush equal bit for bit."""
    from paper_2507_03836_amd.model import FHashConfig, FHashModel
    f, mask = vol
    dims = _dims(mask)
    cfg = FHashConfig(res=WIDE16, n_features=2, hidden=64, n_hidden=3)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    probe = FHashModel(cfg, bits, dims, track_touched=False)
    rows = probe.rows
    del probe
    rng = np.random.default_rng(81)
    table0 = torch.from_numpy(rng.uniform(-0.3, 0.3, (rows, 2)).astype(np.float32))
    mlp0 = torch.from_numpy(synth.mlp_init(cfg.width, seed=82))
    mk = lambda **a: FHashModel(cfg, bits, dims, table_init=table0, mlp_init=mlp0, **a)
    dense = mk(track_touched=False)
    lazy = mk(lazy=True)
    # defer from level 6 on (a dense prefix, as at the production shapes)
    begin = int(lazy.index.slot_offset[6]) * 2 // 16 * 16
    lazy.lazy = fl.LazyState(begin, lazy.mlp_off, 64)

    def same(a, b, what):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), what

    def fresh(m):
        lz = m.lazy
        b, e = lz.desc.begin, lz.desc.end
        nseg = (e - b + 15) // 16
        stamp = lz.ws[: nseg * 8].view(torch.int32).view(nseg, 2)[:, 1]
        keep = torch.ones(m.grads.numel(), dtype=torch.bool, device=m.grads.device)
        keep[b:e] = (stamp == lz.steps + 1).repeat_interleave(16)[: e - b]
        return torch.where(keep, m.grads, torch.zeros_like(m.grads))

    gen = torch.Generator().manual_seed(83)
    for s in range(10):
        pos = torch.rand(700, 4, generator=gen).cuda()
        tgt = torch.rand(700, generator=gen).cuda()
        same(lazy.forward(pos), dense.forward(pos), f"forward, step {s}")
        lazy.fwd_bwd(pos, tgt)
        dense.grads.copy_(fresh(lazy))
        assert dense.optimizer_step() and lazy.optimizer_step()
        if s == 5:
            lazy.flush()
    lazy.flush()
    n = dense.n_params
    for name in ("params", "m", "v", "grads"):
        same(getattr(lazy, name)[:n], getattr(dense, name)[:n], name)


def test_corner_rows_match_oracle_corners(fl, vol):
    """fhash_corner_rows (the instrumentation behind the benchmark's
    compulsory-line count): table rows equal the oracle's corner slots (corner
    c = x-bit | row << 1), directory entries follow the documented layout
    ((t Rz + z) ceil(Rx/64) + x // 64) Ry + y of the oracle's cell."""
    idx, dir_t, g, _ = _setup(fl, vol, WIDE16, 2, "f32")
    n = 1000
    pos = _positions(n, 61)
    d_dir, d_slot = fl.fhash_corner_rows(idx, torch.from_numpy(pos).cuda(), n)
    slots, _ = O.corners(g, pos)
    got = d_slot.cpu().numpy().reshape(n, 16, 8, 2)
    want = slots.reshape(n, 16, 8, 2)  # c = e + 2 r
    np.testing.assert_array_equal(got, want)
    dd = d_dir.cpu().numpy()
    for s in range(0, n, 37):
        for l, (Rx, Ry, Rz, Rt) in enumerate(WIDE16):
            cell = [O.locate(float(pos[s, d]), WIDE16[l][d])[0] for d in range(4)]
            Wv = (Rx + 63) // 64
            for r in range(8):
                y, z, t = cell[1] + (r & 1), cell[2] + ((r >> 1) & 1), cell[3] + (r >> 2)
                w0 = int(idx.dir_offset[l]) + ((t * Rz + z) * Wv + cell[0] // 64) * Ry + y
                assert dd[s, l, r, 0] == w0
                assert dd[s, l, r, 1] == (w0 + Ry if cell[0] % 64 == 63 else -1)
