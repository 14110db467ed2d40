"""GPU checks at the mixed-precision / serving training shape: 432^3 x 60
voxels, 16 levels (spatial 16..512 clamped to 432, temporal 4..60), decoder
32-64-64-64-1, batch 2^20 (the launch configuration bench.py times for it).
The finest level has 432^3 x 60 = 4.84e9 box vertices (more than 2^32), so
vertex linear ids need 64 bits while the kernels index rows and directory
words in 32 bits: the sampled checks below put picked samples' corners at
that level through the full fused forward and backward."""
import numpy as np
import pytest
import torch

import oracle as O

from fullsize_util import sampled_fused_check

pytestmark = pytest.mark.gpu

DIMS = [432, 432, 432, 60]


@pytest.fixture(scope="module")
def prod():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import volume
    from paper_2507_03836_amd.model import geometric_resolutions
    fl.lib()
    print("[fullsize432] generating the volume", flush=True)
    gen = volume.production_volume(DIMS, seed=1003)
    res = geometric_resolutions(16, 16, 512, 4, 60, DIMS)
    idx, counts, dir_t, ws = fl.fhash_build_index(fl.grid_desc(res, 2), gen["bits"], DIMS)
    del ws
    return dict(fl=fl, gen=gen, res=res, idx=idx, counts=counts, dir=dir_t)


def test_finest_level_exceeds_32_bit_vertex_ids(prod):
    Rx, Ry, Rz, Rt = prod["res"][-1]
    assert Rx * Ry * Rz * Rt > 1 << 32
    assert sum(prod["counts"]) == int(prod["idx"].slot_offset[16])


def test_sampled_directory_activity(prod):
    idx, dir_t, res = prod["idx"], prod["dir"], prod["res"]
    bits = prod["gen"]["bits"].cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(17)
    r = res[-1]
    Rx, Ry, Rz, Rt = r
    Wv = (Rx + 63) // 64
    lo = int(idx.dir_offset[15])
    dl = dir_t[lo:].view(torch.int64)
    for _ in range(64):
        v = [int(rng.integers(0, r[d])) for d in range(4)]
        e = ((v[3] * Rz + v[2]) * Wv + v[0] // 64) * Ry + v[1]
        word = int(dl[e, 0].item()) & ((1 << 64) - 1)
        assert ((word >> (v[0] % 64)) & 1) == int(O.vertex_active_bits(r, bits, DIMS, v)), v


def test_fused_forward_backward_sampled_against_oracle(prod):
    out = sampled_fused_check(prod["fl"], prod["gen"], prod["res"], prod["idx"], prod["dir"],
                              DIMS, width=[32, 64, 64, 64, 1], B=1 << 20, seed=2003)
    print(f"\n[fullsize432] {out['touched']} checked rows of {out['rows']}")
