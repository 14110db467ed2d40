"""GPU checks at the production training shape (480 x 720 x 120 x 100, 16 levels,
batch 2^18, the launch configuration bench.py times), where the oracle cannot
enumerate whole levels: properties that hold at any size, plus sampled outputs
the oracle computes one by one.

- the rank directory is an exact exclusive prefix sum of its own bit words and
  sums to the reported per-level counts (so slots are a bijection onto
  0..count-1 in F-Hash order);
- sampled vertices are active exactly when the oracle's one-by-one decision
  (closed-box cells, corner rule) says so;
- the fused forward over a full 2^18 batch reproduces, for sampled samples, the
  oracle's value computed from vertex coordinates alone: every touched active
  vertex's row holds h(vertex id), so a wrong slot would read a wrong h.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

pytestmark = pytest.mark.gpu

DIMS = [480, 720, 120, 100]


def _popcount64(x: torch.Tensor) -> torch.Tensor:
    """Population count of int64 words (logical shifts emulated with masks)."""
    m1, m2, m4 = 0x5555555555555555, 0x3333333333333333, 0x0F0F0F0F0F0F0F0F
    sh = lambda v, k: (v >> k) & ((1 << (64 - k)) - 1)
    to_s = lambda c: c - (1 << 64) if c >= 1 << 63 else c
    x = x - (sh(x, 1) & to_s(m1))
    x = (x & to_s(m2)) + (sh(x, 2) & to_s(m2))
    x = (x + sh(x, 4)) & to_s(m4)
    return (sh(x * 0x0101010101010101, 56)) & 0xFF


@pytest.fixture(scope="module")
def prod():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd.model import geometric_resolutions
    fl.lib()
    gen = synth.production_volume_gpu(DIMS, seed=1002)
    res = geometric_resolutions(16, 16, 512, 4, 100, DIMS)
    grid = fl.grid_desc(res, 2)
    idx, counts, dir_t, ws = fl.fhash_build_index(grid, gen["bits"], DIMS)
    del ws
    return dict(fl=fl, gen=gen, res=res, idx=idx, counts=counts, dir=dir_t)


def test_directory_is_exact_prefix_sum(prod):
    idx, dir_t, res, counts = prod["idx"], prod["dir"], prod["res"], prod["counts"]
    for l, (Rx, Ry, Rz, Rt) in enumerate(res):
        lo, hi = int(idx.dir_offset[l]), int(idx.dir_offset[l + 1])
        Wv = (Rx + 63) // 64
        # stored ((t*Rz + z)*Wv + word)*Ry + y; ranks follow row-major (t, z, y, word)
        rm = dir_t[lo:hi].view(Rt * Rz, Wv, Ry, 2).permute(0, 2, 1, 3).reshape(-1, 2)
        run = 0
        for s in range(0, hi - lo, 1 << 24):
            e = min(s + (1 << 24), hi - lo)
            ent = rm[s:e]
            pc = _popcount64(ent[:, 0])
            rank = ent[:, 1]
            assert int(rank[0]) == run
            assert torch.equal(rank[1:], rank[:-1] + pc[:-1])
            run = int(rank[-1]) + int(pc[-1])
        assert run == counts[l], (l, run, counts[l])
        assert int(idx.slot_offset[l + 1] - idx.slot_offset[l]) == counts[l]


def _entry(res, v):
    """Directory entry of vertex v = (x, y, z, t): ((t*Rz + z)*Wv + x//64)*Ry + y."""
    Rx, Ry, Rz, Rt = res
    Wv = (Rx + 63) // 64
    return ((v[3] * Rz + v[2]) * Wv + v[0] // 64) * Ry + v[1]


def _vertex_bit(dir_np_level, res, v):
    word = int(dir_np_level[_entry(res, v), 0])
    return (word >> (v[0] % 64)) & 1


def test_sampled_vertex_activity_matches_oracle(prod):
    idx, dir_t, res = prod["idx"], prod["dir"], prod["res"]
    bits = prod["gen"]["bits"].cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(7)
    for l, r in enumerate(res):
        lo, hi = int(idx.dir_offset[l]), int(idx.dir_offset[l + 1])
        dl = dir_t[lo:hi].cpu().numpy().view(np.uint64)
        n_check = 12 if l < 6 else 40
        for _ in range(n_check):
            v = [int(rng.integers(0, r[d])) for d in range(4)]
            exp = O.vertex_active_bits(r, bits, DIMS, v)
            assert _vertex_bit(dl, r, v) == int(exp), (l, v)


def _h(lin):
    return np.sin(0.6180339887 * lin.astype(np.float64) + 0.25) * 0.5


def test_fused_forward_sampled_against_oracle(prod):
    fl, gen, res, idx, dir_t = prod["fl"], prod["gen"], prod["res"], prod["idx"], prod["dir"]
    B = 1 << 18
    width = [32, 64, 64, 1]
    params = synth.mlp_init(width, seed=9)
    pos = torch.empty(B, 4, device="cuda")
    tgt = torch.empty(B, device="cuda")
    fl.fhash_sample(2002, 7, B, gen["coreset"], gen["M"], DIMS, gen["field"], pos, tgt)
    pick = np.random.default_rng(3).choice(B, 48, replace=False)
    pos_np = pos[torch.from_numpy(pick).cuda()].cpu().numpy()
    dense = O.Grid(np.array(res), 2, None)          # slots = vertex linear ids
    lin, w = O.corners(dense, pos_np)               # [48][L][16]
    bits = gen["bits"].cpu().numpy().view(np.uint64)
    rows = int(idx.slot_offset[len(res)])
    table = torch.zeros(rows, 2, device="cuda")
    enc_ref = np.zeros((48, 32))
    enc_mag = np.zeros((48, 32))
    slot_list, val_list = [], []
    for l, r in enumerate(res):
        Rx, Ry, Rz, Rt = r
        lo, hi = int(idx.dir_offset[l]), int(idx.dir_offset[l + 1])
        dl = dir_t[lo:hi].cpu().numpy().view(np.uint64)
        Wv = (Rx + 63) // 64
        for s in range(48):
            for c in range(16):
                v_lin = int(lin[s, l, c] - dense.slot_offset[l])
                v = [v_lin % Rx, (v_lin // Rx) % Ry, (v_lin // (Rx * Ry)) % Rz,
                     v_lin // (Rx * Ry * Rz)]
                act = O.vertex_active_bits(r, bits, DIMS, v)
                hv = _h(np.array([v_lin + 1000003 * l]))[0]
                if act:
                    enc_ref[s, 2 * l] += w[s, l, c] * hv
                    enc_ref[s, 2 * l + 1] += w[s, l, c] * (0.5 - hv)
                    enc_mag[s, 2 * l] += w[s, l, c] * abs(hv)
                    enc_mag[s, 2 * l + 1] += w[s, l, c] * abs(0.5 - hv)
                    # the test (not the oracle) places h at the vertex's slot
                    ent = dl[_entry(r, v)]
                    below = int(ent[0]) & ((1 << (v[0] % 64)) - 1)
                    slot = int(idx.slot_offset[l]) + int(ent[1]) + bin(below).count("1")
                    slot_list.append(slot)
                    val_list.append((hv, 0.5 - hv))
    sl = torch.tensor(slot_list, device="cuda")
    table[sl] = torch.tensor(val_list, dtype=torch.float32, device="cuda")
    y = torch.empty(B, device="cuda")
    fl.fhash_fused_fwd(idx, fl.mlp_desc(width), pos, B, table.view(-1),
                       torch.from_numpy(params).cuda(), y)
    y_ref, _, ymag = O.mlp_fwd(width, params.astype(np.float64), enc_ref,
                               x_mag=enc_mag)
    got = y[torch.from_numpy(pick).cuda()].cpu().numpy().astype(np.float64)
    err = np.abs(got - y_ref[:, 0])
    assert (err <= 1e-5 * ymag[:, 0] + 1e-9).all(), float(err.max())
