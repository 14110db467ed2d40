"""Feature-based coreset selection, plain numpy -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may use this module; the product path never does.  It shares no code with the
HIP library.  Every function follows Sec. 3.1 of the paper (feature
extraction, feature dilation and the occupancy grid, bounding boxes and
temporal fusion, time-step concatenation and the coreset union of Eq. (3)),
with the readings stated in each docstring.  Arrays are indexed [t][z][y][x]
(a voxel mask is a bool array of that shape).

Parity status: every function is pinned by tests/test_oracle_coreset.py against
brute-force enumeration on tiny inputs, closed forms and library routines
(scipy.ndimage dilation, numpy.flatnonzero).  The isosurface rule and the brick
layout of the occupancy grid are this repository's readings (the paper names
the feature types and Morton order without fixing either); they are pinned as
definitions, not against printed values.
"""
from __future__ import annotations

import numpy as np


def feature_interval(field: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Value-range feature (Sec. 3.1, feature extraction): voxel in the
    feature iff lo < v <= hi, compared in float32 like the field itself."""
    v = np.asarray(field, np.float32)
    return (v > np.float32(lo)) & (v <= np.float32(hi))


def feature_isosurface(field: np.ndarray, level: float) -> np.ndarray:
    """Isosurface feature (Sec. 3.1, feature extraction; reading): inside each
    timestep a spatial cell (its 8 corner voxels) is crossed by the level set
    v = level iff some corner has v >= level and some corner v < level; the
    feature is every corner voxel of a crossed cell."""
    v = np.asarray(field, np.float32)
    above = v >= np.float32(level)
    T, Z, Y, X = above.shape
    any_a = np.zeros((T, Z - 1, Y - 1, X - 1), bool)
    all_a = np.ones((T, Z - 1, Y - 1, X - 1), bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                c = above[:, dz:Z - 1 + dz, dy:Y - 1 + dy, dx:X - 1 + dx]
                any_a |= c
                all_a &= c
    crossed = any_a & ~all_a
    out = np.zeros_like(above)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                out[:, dz:Z - 1 + dz, dy:Y - 1 + dy, dx:X - 1 + dx] |= crossed
    return out


def dilate(mask: np.ndarray, r: int) -> np.ndarray:
    """Feature dilation (Sec. 3.1): add the neighbouring voxels of the feature
    so interpolation at its boundary has every corner.  Reading: a cube of
    radius r inside each timestep (the voxel is kept iff a feature voxel of
    the same timestep lies within r along each of x, y and z)."""
    m = np.asarray(mask, bool)
    T, Z, Y, X = m.shape
    out = np.zeros_like(m)
    # offsets of a whole dimension or more reach no voxel (and would wrap the slices)
    for dz in range(-min(r, Z - 1), min(r, Z - 1) + 1):
        for dy in range(-min(r, Y - 1), min(r, Y - 1) + 1):
            for dx in range(-min(r, X - 1), min(r, X - 1) + 1):
                src = m[:, max(dz, 0):Z + min(dz, 0), max(dy, 0):Y + min(dy, 0),
                        max(dx, 0):X + min(dx, 0)]
                out[:, max(-dz, 0):Z + min(-dz, 0), max(-dy, 0):Y + min(-dy, 0),
                    max(-dx, 0):X + min(-dx, 0)] |= src
    return out


def feature_boxes(mask: np.ndarray) -> np.ndarray:
    """Bounding box b_k of each timestep's feature and their temporal fusion,
    the FBB (Sec. 3.1): int array [T + 1][6] of inclusive voxel indices
    (xmin, ymin, zmin, xmax, ymax, zmax); row T is the smallest box that
    contains every b_k.  An empty frame (or an empty mask, row T) reads
    (X, Y, Z, -1, -1, -1)."""
    m = np.asarray(mask, bool)
    T, Z, Y, X = m.shape
    out = np.tile(np.array([X, Y, Z, -1, -1, -1], np.int64), (T + 1, 1))
    for k in range(T):
        z, y, x = np.nonzero(m[k])
        if x.size:
            out[k] = [x.min(), y.min(), z.min(), x.max(), y.max(), z.max()]
    t, z, y, x = np.nonzero(m)
    if x.size:
        out[T] = [x.min(), y.min(), z.min(), x.max(), y.max(), z.max()]
    return out


def morton_bit(lx: int, ly: int, lz: int) -> int:
    """Bit of voxel (lx, ly, lz) of a 4x4x4 brick in Morton (Z-order) order:
    the bits of x, y and z interleaved, x lowest."""
    m = 0
    for b in range(2):
        m |= ((lx >> b) & 1) << (3 * b)
        m |= ((ly >> b) & 1) << (3 * b + 1)
        m |= ((lz >> b) & 1) << (3 * b + 2)
    return m


def occupancy_grid(mask: np.ndarray) -> np.ndarray:
    """Occupancy grid stored as bits with Morton linearisation (Sec. 3.1).
    Reading: one 64-bit word per 4x4x4 brick, Morton order inside the brick,
    bricks in [t][bz][by][bx] order; voxels outside the volume are 0.
    Returns uint64 [T][ceil(Z/4)][ceil(Y/4)][ceil(X/4)]."""
    m = np.asarray(mask, bool)
    T, Z, Y, X = m.shape
    bz, by, bx = -(-Z // 4), -(-Y // 4), -(-X // 4)
    pad = np.zeros((T, 4 * bz, 4 * by, 4 * bx), bool)
    pad[:, :Z, :Y, :X] = m
    occ = np.zeros((T, bz, by, bx), np.uint64)
    for lz in range(4):
        for ly in range(4):
            for lx in range(4):
                bit = np.uint64(1) << np.uint64(morton_bit(lx, ly, lz))
                sel = pad[:, lz::4, ly::4, lx::4]
                occ[sel] |= bit
    return occ


def coreset_ids(mask: np.ndarray) -> np.ndarray:
    """Coreset of Eq. (3): the union over timesteps of the feature voxels with
    their timestep attached, as linear ids ((t Z + z) Y + y) X + x in
    increasing order."""
    return np.flatnonzero(np.asarray(mask, bool).ravel()).astype(np.uint64)


def pack_rows(mask: np.ndarray) -> np.ndarray:
    """Bool mask -> row-padded 64-voxel words [T][Z][Y][ceil(X/64)] (uint64),
    bit b of word w = voxel x = 64 w + b."""
    m = np.asarray(mask, bool)
    T, Z, Y, X = m.shape
    W = -(-X // 64)
    pad = np.zeros((T, Z, Y, 64 * W), bool)
    pad[..., :X] = m
    bits = pad.reshape(T, Z, Y, W, 64).astype(np.uint64)
    weights = np.uint64(1) << np.arange(64, dtype=np.uint64)
    return (bits * weights).sum(axis=-1, dtype=np.uint64)


def unpack_rows(words: np.ndarray, shape) -> np.ndarray:
    """Inverse of pack_rows for a mask of shape (T, Z, Y, X)."""
    T, Z, Y, X = shape
    w = np.asarray(words).view(np.uint64).reshape(T, Z, Y, -1)
    bits = (w[..., None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(T, Z, Y, -1)[..., :X].astype(bool)
