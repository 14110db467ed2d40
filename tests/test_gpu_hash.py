"""The spatial-hash comparison index (fhash_hash_index) on the GPU kernels,
against the FP64 oracle on the same hashed rows (oracle.Grid(hash_bits=b)):
row offsets exact, the encoding, the fused training gradients (where colliding
vertices sum into one row) and the decoder gradient within the FP32 tolerance,
and the deferred Adam on a hashed table equal to the dense update bit for bit
(the two slots of a row pair are then not neighbours)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import coreset_ids, tiny_volume

pytestmark = pytest.mark.gpu

TINY_RES = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]
BITS = 9  # levels 1-3 hash into 512 rows
RTOL, ATOL = 1e-5, 1e-12


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


def _close(gpu, ref, mag, what):
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    tol = RTOL * mag + ATOL
    assert (err <= tol).all(), (what, float((err - tol).max()))


def _params(width, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([
        np.concatenate([rng.uniform(-1, 1, width[k + 1] * width[k]) / np.sqrt(width[k]),
                        rng.uniform(-0.1, 0.1, width[k + 1])]) for k in range(len(width) - 1)
    ]).astype(np.float32)


def test_hash_index_rows(fl):
    idx, rows = fl.fhash_hash_index(fl.grid_desc(TINY_RES, 2), BITS)
    g = O.Grid(np.array(TINY_RES), 2, hash_bits=BITS)
    assert rows == g.counts and idx.hash_bits == BITS and idx.active == 0
    assert [idx.slot_offset[l] for l in range(5)] == list(g.slot_offset)
    with pytest.raises(fl.FHashError):
        fl.fhash_hash_index(fl.grid_desc(TINY_RES, 2), 3)


@pytest.mark.parametrize("F", [2, 4])
def test_encode_and_fused_train_against_oracle(fl, F):
    f, mask = tiny_volume()
    idx, _ = fl.fhash_hash_index(fl.grid_desc(TINY_RES, F), BITS)
    g = O.Grid(np.array(TINY_RES), F, hash_bits=BITS)
    rng = np.random.default_rng(30 + F)
    table = rng.uniform(-1, 1, (g.total_slots, F)).astype(np.float32)
    n = 3000 + 7
    pos = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    tgt = rng.uniform(0, 1, n).astype(np.float32)
    pd, td = torch.from_numpy(pos).cuda(), torch.from_numpy(tgt).cuda()
    tab = torch.from_numpy(table).cuda()
    enc = torch.empty(n, 4 * F, device="cuda")
    fl.fhash_encode_fwd(idx, pd, n, tab, enc)
    e_ref, e_mag = O.encode_fwd(g, pos, table.astype(np.float64))
    _close(enc.cpu().numpy(), e_ref, e_mag, "hashed encode")
    width = [4 * F, 32, 32, 1]
    params = _params(width, 40 + F)
    y, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), e_ref, x_mag=e_mag)
    L, dy = O.mse(y[:, 0], tgt.astype(np.float64))
    dym = 2.0 * (ymag[:, 0] + np.abs(tgt)) / n
    dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                         dy.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                         x_mag=e_mag)
    dt_ref, _ = O.encode_bwd(g, pos, denc)
    _, dtm = O.encode_bwd(g, pos, dencm)
    dt = torch.zeros(g.total_slots, F, device="cuda")
    dp = torch.zeros(len(params), device="cuda")
    fl.fhash_fused_train(idx, fl.mlp_desc(width), pd, td, n, tab,
                         torch.from_numpy(params).cuda(), dt, dp)
    _close(dt.cpu().numpy(), dt_ref, dtm, "hashed fused_train d_table")
    _close(dp.cpu().numpy(), dp_ref, dpm, "hashed fused_train d_params")
    # collisions really happen at this size: some row receives several vertices
    used = np.concatenate([g.maps[l] for l in (2, 3)])
    assert len(np.unique(used)) < used.size


def test_lazy_adam_on_hashed_table_equals_dense(fl):
    from paper_2507_03836_amd.model import FHashConfig, FHashModel
    f, mask = tiny_volume()
    T, Sz, Sy, Sx = mask.shape
    dims = [Sx, Sy, Sz, T]
    cfg = FHashConfig(res=TINY_RES, n_features=2, hidden=32, n_hidden=2)
    g = O.Grid(np.array(TINY_RES), 2, hash_bits=BITS)
    rng = np.random.default_rng(77)
    table0 = torch.from_numpy(rng.uniform(-0.3, 0.3, (g.total_slots, 2)).astype(np.float32))
    mlp0 = torch.from_numpy(synth.mlp_init(cfg.width, seed=78))
    mk = lambda **a: FHashModel(cfg, None, dims, table_init=table0, mlp_init=mlp0,
                                hash_bits=BITS, **a)
    dense, lazy = mk(track_touched=False), mk(lazy=True)
    gen = torch.Generator().manual_seed(11)
    for s in range(10):
        pos = torch.rand(60, 4, generator=gen).cuda()
        tgt = torch.rand(60, generator=gen).cuda()
        assert torch.equal(lazy.forward(pos), dense.forward(pos)), s
        lazy.fwd_bwd(pos, tgt)
        lz = lazy.lazy
        b, e = lz.desc.begin, lz.desc.end
        nseg = (e - b + 15) // 16
        stamp = lz.ws[: nseg * 8].view(torch.int32).view(nseg, 2)[:, 1]
        fresh = torch.ones(lazy.grads.numel(), dtype=torch.bool, device="cuda")
        fresh[b:e] = (stamp == lz.steps + 1).repeat_interleave(16)[: e - b]
        dense.grads.copy_(torch.where(fresh, lazy.grads, torch.zeros_like(lazy.grads)))
        dense.optimizer_step()
        lazy.optimizer_step()
    lazy.flush()
    n = dense.n_params
    for name in ("params", "m", "v", "grads"):
        assert torch.equal(getattr(lazy, name)[:n].view(torch.int32),
                           getattr(dense, name)[:n].view(torch.int32)), name
