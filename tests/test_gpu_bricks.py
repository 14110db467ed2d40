"""The active-vertex index in brick order (2 x 2 x 2 x 2 vertex bricks, Sec.
3.2.3 allows linearisations other than the F-Hash equation's) on the device
against the oracle's brick ranking: the directory bit for bit (tiny and random
grids, odd resolutions, x pairs straddling bricks and words), the fused
kernels at 16 levels x 2 features element by element within the FP32
tolerance, the deferred Adam against the dense update bit for bit, and the
instrumentation's directory entries at the documented brick layout."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import tiny_volume

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-12
WIDE16 = None  # filled from test_gpu_parity_wide's grid rule below


def _wide_res(L, rmax=(70, 24, 20, 8)):
    return [[max(2, int(np.floor(2.0 * (r / 2.0) ** (l / (L - 1)) + 0.5))) for r in rmax]
            for l in range(L)]


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


def _popcount(v):
    v = v.astype(np.uint64)
    c = np.zeros(v.shape, np.int64)
    for k in range(64):
        c += ((v >> np.uint64(k)) & np.uint64(1)).astype(np.int64)
    return c


def _brick_entry(R, x, y, z, t):
    """(entry index within the level, bit) of vertices, per the header's layout."""
    Rx, Ry, Rz, Rt = R
    By, Bz = (Ry + 1) // 2, (Rz + 1) // 2
    Wb = ((Rx + 1) // 2 + 3) // 4
    inner = (x & 1) | (y & 1) << 1 | (z & 1) << 2 | (t & 1) << 3
    bit = (x >> 1) * 16 + inner
    btz = (t >> 1) * Bz + (z >> 1)
    return (btz * Wb + (bit >> 6)) * By + (y >> 1), bit & 63


def _decode_bricks(idx, dir_t, res):
    d = dir_t.cpu().numpy().view(np.uint64).reshape(-1, 2)
    maps = []
    for l, R in enumerate(res):
        Rx, Ry, Rz, Rt = R
        t, z, y, x = np.meshgrid(np.arange(Rt), np.arange(Rz), np.arange(Ry), np.arange(Rx),
                                 indexing="ij")
        e, b = _brick_entry(R, x.ravel(), y.ravel(), z.ravel(), t.ravel())
        ent = d[int(idx.dir_offset[l]) + e]
        bits, rank = ent[:, 0], ent[:, 1]
        bu = b.astype(np.uint64)
        act = ((bits >> bu) & np.uint64(1)).astype(bool)
        below = np.where(b == 0, np.uint64(0), bits & ((np.uint64(1) << bu) - np.uint64(1)))
        slot = rank.astype(np.int64) + _popcount(below)
        slot[~act] = -1
        maps.append(slot)
    return maps


def _build(fl, res, F, mask):
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    return fl.fhash_build_index(fl.grid_desc(res, F, fl.LAYOUT_BRICKS), bits, _dims(mask))


@pytest.mark.parametrize("trial", range(10))
def test_brick_index_bit_exact(fl, trial):
    if trial == 0:
        f, mask = tiny_volume()
        res = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]
    else:
        rng = np.random.default_rng(300 + trial)
        S = rng.integers(2, 90, size=4)
        S[3] = rng.integers(2, 9)
        mask = (rng.random((S[3], S[2], S[1], S[0])) < rng.uniform(0.001, 0.3)).astype(np.uint8)
        res = [[int(rng.integers(2, 70)) for _ in range(3)] + [int(rng.integers(2, 10))]
               for _ in range(int(rng.integers(1, 5)))]
        if trial == 1:
            res = [[67, 129, 3, 2], [9, 5, 7, 3]]  # odd edges, x pairs across words
        if trial == 2:
            mask[:] = 0
    idx, counts, dir_t, _ = _build(fl, res, 1, mask)
    g = O.Grid(np.array(res), 1, mask, layout=O.LAYOUT_BRICKS)
    assert counts == g.counts
    got = _decode_bricks(idx, dir_t, res)
    for l in range(len(res)):
        np.testing.assert_array_equal(got[l], g.maps[l], err_msg=f"level {l}")


def test_brick_layout_rejected_where_not_built(fl):
    with pytest.raises(fl.FHashError):
        fl.fhash_dense_index(fl.grid_desc([[4, 4, 4, 2]], 2, fl.LAYOUT_BRICKS))


def _close(gpu, ref, mag, what):
    bad = np.abs(gpu - ref) > RTOL * mag + ATOL
    assert not bad.any(), (what, int(bad.sum()), float(np.abs(gpu - ref).max()))


@pytest.mark.parametrize("F,L,hidden,tdt", [(2, 16, [64, 64, 64], "f32"),
                                            (2, 16, [64, 64, 64], "f16"),
                                            (4, 8, [64, 64], "f32")])
def test_brick_fused_against_oracle(fl, F, L, hidden, tdt):
    f, mask = tiny_volume()
    res = _wide_res(L)
    idx, counts, dir_t, _ = _build(fl, res, F, mask)
    g = O.Grid(np.array(res), F, mask, layout=O.LAYOUT_BRICKS)
    assert counts == g.counts
    rng = np.random.default_rng(L * 7 + F)
    table = rng.uniform(-1, 1, (g.total_slots, F)).astype(np.float32)
    if tdt == "f16":
        table = table.astype(np.float16)
    width = [L * F] + hidden + [1]
    params = synth.mlp_init(width, seed=L + F)
    n = 4096 + 37
    pos = rng.random((n, 4)).astype(np.float32)
    tgt = rng.random(n).astype(np.float32)
    enc, emag = O.encode_fwd(g, pos, table.astype(np.float64))
    y_ref, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    mlp = fl.mlp_desc(width)
    pos_d, tab_d, prm = (torch.from_numpy(a).cuda() for a in (pos, table, params))
    y = torch.full((n,), np.nan, device="cuda")
    fl.fhash_fused_fwd(idx, mlp, pos_d, n, tab_d, prm, y)
    _close(y.cpu().numpy(), y_ref[:, 0], ymag[:, 0], "fused_fwd")
    L_ref, dy_ref = O.mse(y_ref[:, 0], tgt.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tgt)) / n
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy_ref.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                         x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    dt = torch.zeros(g.total_slots, F, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl.fhash_fused_train(idx, mlp, pos_d, torch.from_numpy(tgt).cuda(), n, tab_d, prm, dt, dp,
                         loss)
    _close(dp.cpu().numpy(), dp_ref, dpm, "fused_train d_params")
    _close(dt.cpu().numpy(), dt_ref, dtm, "fused_train d_table")


def test_brick_lazy_equals_dense(fl):
    """Deferred Adam on a brick-ordered index against the dense update: every
    forward value between steps and every parameter, moment and gradient
    after the flush equal bit for bit."""
    from paper_2507_03836_amd.model import FHashConfig, FHashModel
    f, mask = tiny_volume()
    dims = _dims(mask)
    cfg = FHashConfig(res=_wide_res(16), n_features=2, hidden=64, n_hidden=3, layout=1)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    probe = FHashModel(cfg, bits, dims, track_touched=False)
    rows = probe.rows
    assert probe.grid.layout == fl.LAYOUT_BRICKS
    del probe
    rng = np.random.default_rng(91)
    table0 = torch.from_numpy(rng.uniform(-0.3, 0.3, (rows, 2)).astype(np.float32))
    mlp0 = torch.from_numpy(synth.mlp_init(cfg.width, seed=92))
    mk = lambda **a: FHashModel(cfg, bits, dims, table_init=table0, mlp_init=mlp0, **a)
    dense = mk(track_touched=False)
    lazy = mk(lazy=True)
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

    gen = torch.Generator().manual_seed(93)
    for s in range(8):
        pos = torch.rand(700, 4, generator=gen).cuda()
        tgt = torch.rand(700, generator=gen).cuda()
        same(lazy.forward(pos), dense.forward(pos), f"forward, step {s}")
        lazy.fwd_bwd(pos, tgt)
        dense.grads.copy_(fresh(lazy))
        assert dense.optimizer_step() and lazy.optimizer_step()
    lazy.flush()
    n = dense.n_params
    for name in ("params", "m", "v", "grads"):
        same(getattr(lazy, name)[:n], getattr(dense, name)[:n], name)


def _pair_axis(c):
    for a in range(4):
        if c[a] % 2 == 0:
            return a
    return 0


def _pair_offsets(r, a):
    """Offsets (x, y, z, t) of the first corner of pair r along axis a: the
    other axes, in increasing order, take bits 0, 1, 2 of r."""
    o, k = [0, 0, 0, 0], 0
    for d in range(4):
        if d != a:
            o[d] = (r >> k) & 1
            k += 1
    return o


def test_brick_corner_rows(fl):
    """fhash_corner_rows on a brick-ordered index: the 16 rows of every sample
    and level are the oracle's corner slots (as a set: the corners are taken
    as 8 pairs along the first axis with an even cell index); the directory
    entries follow the documented brick layout for the pair's first corner
    (and its x neighbour's when the pair runs along x)."""
    f, mask = tiny_volume()
    res = _wide_res(16)
    idx, counts, dir_t, _ = _build(fl, res, 2, mask)
    g = O.Grid(np.array(res), 2, mask, layout=O.LAYOUT_BRICKS)
    n = 600
    pos = np.random.default_rng(5).random((n, 4)).astype(np.float32)
    d_dir, d_slot = fl.fhash_corner_rows(idx, torch.from_numpy(pos).cuda(), n)
    slots, _ = O.corners(g, pos)
    got = np.sort(d_slot.cpu().numpy().reshape(n, 16, 16), axis=2)
    np.testing.assert_array_equal(got, np.sort(slots.reshape(n, 16, 16), axis=2))
    dd = d_dir.cpu().numpy()
    for s in range(0, n, 29):
        for l, R in enumerate(res):
            cell = [O.locate(float(pos[s, d]), R[d])[0] for d in range(4)]
            a = _pair_axis(cell)
            for r in range(8):
                o = _pair_offsets(r, a)
                x, y, z, t = (cell[d] + o[d] for d in range(4))
                e0, _ = _brick_entry(R, x, y, z, t)
                e1, _ = _brick_entry(R, x + 1, y, z, t)
                off = int(idx.dir_offset[l])
                assert dd[s, l, r, 0] == off + e0
                assert dd[s, l, r, 1] == (off + e1 if a == 0 and e1 != e0 else -1)
