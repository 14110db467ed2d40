"""Feature-based coreset selection of a volume (Sec. 3.1) through the C ABI.

A feature attribute field on the device goes through the method's own calls:
feature extraction (fhash_feature_mask), dilation inside each timestep
(fhash_dilate_mask) and the coreset id list (fhash_coreset).  The result is
the voxel mask the index is built from and the coreset the sampler draws
from.  `production_volume` composes this with the seeded synthetic field of the
production workloads (generator in `synth`, inputs only).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as fl
from . import synth


def select_coreset(attr: torch.Tensor, dims, lo: float, hi: float = float("inf"),
                   radius: int = 0, kind: int = fl.FEATURE_INTERVAL) -> dict:
    """Feature mask of `attr` (device float [T][Sz][Sy][Sx]) with bounds
    (lo, hi] (or the isosurface at lo), dilated by a cube of `radius`; returns
    dict(bits=int64 mask words [T][Sz][Sy][ceil(Sx/64)], coreset=int64 view of
    the increasing uint64 voxel ids, M=their count)."""
    Sx, Sy, Sz, T = (int(d) for d in dims)
    feat = fl.fhash_feature_mask(attr, dims, kind, lo, hi)
    if radius > 0:
        bits = fl.fhash_dilate_mask(feat, dims, radius)
        del feat
    else:
        bits = feat
    bits = bits.view(T, Sz, Sy, (Sx + 63) // 64)
    ids = fl.fhash_coreset(bits, dims)
    return dict(bits=bits, coreset=ids, M=int(ids.numel()))


def production_volume(shape_xyzt, seed: int, keep_field: bool = True) -> dict:
    """The production workload at `shape_xyzt` (Sx, Sy, Sz, T): the seeded
    synthetic field on the device and its coreset, feature = gradient
    magnitude above its 80th percentile, dilated by 2.

    Returns dict(field, bits, coreset, M, N, threshold)."""
    gen = synth.production_field_gpu(shape_xyzt, seed, keep_field=keep_field)
    sel = select_coreset(gen["grad"], shape_xyzt, gen["threshold"],
                         radius=synth.PRODUCTION_DILATION)
    del gen["grad"]
    torch.cuda.synchronize()
    return dict(field=gen["field"], bits=sel["bits"], coreset=sel["coreset"], M=sel["M"],
                N=gen["N"], threshold=gen["threshold"])


def tiny_volume_mask(field: np.ndarray) -> torch.Tensor:
    """Mask words of the tiny workload's feature (value > 0.1, dilated by 1),
    computed on the device from the host field."""
    T, Sz, Sy, Sx = field.shape
    f = torch.from_numpy(np.ascontiguousarray(field, np.float32)).cuda()
    return select_coreset(f, [Sx, Sy, Sz, T], synth.TINY_FEATURE_LO,
                          radius=synth.TINY_DILATION)["bits"]
