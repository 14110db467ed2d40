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
  vertex's row holds h(vertex id), so a wrong slot would read a wrong h; the
  fused backward of the same launch, with dy nonzero only at the sampled
  samples, writes exactly the oracle's table gradient at their corner rows
  and the oracle's decoder gradient.
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
    from paper_2507_03836_amd import volume
    from paper_2507_03836_amd.model import geometric_resolutions
    fl.lib()
    gen = volume.production_volume(DIMS, seed=1002)
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


def test_fused_forward_backward_sampled_against_oracle(prod):
    from fullsize_util import sampled_fused_check
    sampled_fused_check(prod["fl"], prod["gen"], prod["res"], prod["idx"], prod["dir"], DIMS,
                        width=[32, 64, 64, 1], B=1 << 18, seed=2002)
