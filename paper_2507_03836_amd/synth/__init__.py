"""Seeded synthetic inputs shaped like the paper's time-varying volumes.

This module produces inputs only (fields, feature masks, coresets, initial
parameters, probe points); it holds none of the method's arithmetic and is the
one place that both the HIP path and the CPU oracle take their inputs from.

Workload recipe (shapes/distributions of the paper's datasets, which are not
available: scalar float32 fields normalised to [0,1], sparse moving features,
hundreds of voxels per side, tens to a hundred timesteps):

* tiny     : 32^3 x 8, 8 advected Gaussian blobs (centre U[0,1]^3, sigma
             U[0.05,0.15], amplitude U[0.5,1], velocity U[-0.05,0.05]^3 per
             step), clipped to [0,1]; mask = value > 0.1, dilated by 1.
* production: 64 blobs (sigma U[0.02,0.08], amplitude U[0.5,1], velocity
             U[-0.004,0.004]^3) + 0.25 * 3-octave 4D value noise, min-max
             normalised; mask = |grad| > 80th percentile, dilated by 2.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_HOST_LIB = os.path.join(_HERE, "libfhash_synth_host.so")

SEED_FIELD, SEED_SAMPLER, SEED_INIT, SEED_PROBE, SEED_ARRIVALS = 1000, 2000, 3000, 4000, 5000


def build_host(force: bool = True) -> str:
    if force or not os.path.exists(_HOST_LIB):
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", _HOST_LIB,
                        os.path.join(_HERE, "synth.c"), "-lm"], check=True)
    return _HOST_LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_HOST_LIB):
            build_host()
        L = C.CDLL(_HOST_LIB)
        P, I64, U64, D = C.c_void_p, C.c_int64, C.c_uint64, C.c_double
        L.sy_splitmix64.restype = U64
        L.sy_splitmix64.argtypes = [U64]
        L.sy_blob_params.restype = None
        L.sy_blob_params.argtypes = [U64, C.c_int, D, D, D, D, D, P]
        L.sy_value_noise4.restype = D
        L.sy_value_noise4.argtypes = [U64, D, D, D, D]
        L.sy_field.restype = None
        L.sy_field.argtypes = [P, P, C.c_int, D, U64, C.c_int, C.c_int, P]
        L.sy_grad_mag.restype = None
        L.sy_grad_mag.argtypes = [P, P, P]
        L.sy_quantile.restype = C.c_float
        L.sy_quantile.argtypes = [P, I64, D]
        L.sy_threshold.restype = None
        L.sy_threshold.argtypes = [P, I64, C.c_float, P]
        L.sy_dilate.restype = None
        L.sy_dilate.argtypes = [P, P, C.c_int, P]
        L.sy_coreset.restype = I64
        L.sy_coreset.argtypes = [P, I64, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def blob_params(seed, n_blobs, sig, amp, vmax):
    out = np.zeros((n_blobs, 8), np.float64)
    _L().sy_blob_params(seed, n_blobs, sig[0], sig[1], amp[0], amp[1], vmax, _p(out))
    return out


def field(shape_xyzt, blobs, turb_amp=0.0, noise_seed=0, clip01=True, normalise=False):
    Sx, Sy, Sz, T = shape_xyzt
    S = np.array(shape_xyzt, np.int64)
    out = np.zeros((T, Sz, Sy, Sx), np.float32)
    b = np.ascontiguousarray(blobs, np.float64)
    _L().sy_field(_p(S), _p(b), b.shape[0], turb_amp, noise_seed, int(clip01), int(normalise),
                  _p(out))
    return out


def grad_mag(f):
    f = np.ascontiguousarray(f, np.float32)
    T, Sz, Sy, Sx = f.shape
    S = np.array([Sx, Sy, Sz, T], np.int64)
    out = np.zeros_like(f)
    _L().sy_grad_mag(_p(S), _p(f), _p(out))
    return out


def quantile(v, q):
    v = np.ascontiguousarray(v, np.float32).ravel()
    return float(_L().sy_quantile(_p(v), v.size, q))


def threshold(v, thr):
    v = np.ascontiguousarray(v, np.float32)
    m = np.zeros(v.shape, np.uint8)
    _L().sy_threshold(_p(v), v.size, thr, _p(m))
    return m


def dilate(mask, r):
    m = np.ascontiguousarray(mask, np.uint8)
    T, Sz, Sy, Sx = m.shape
    S = np.array([Sx, Sy, Sz, T], np.int64)
    out = np.zeros_like(m)
    _L().sy_dilate(_p(S), _p(m), r, _p(out))
    return out


def coreset(mask):
    m = np.ascontiguousarray(mask, np.uint8).ravel()
    n = _L().sy_coreset(_p(m), m.size, None)
    ids = np.zeros(n, np.uint64)
    _L().sy_coreset(_p(m), m.size, _p(ids))
    return ids


def pack_mask_rows(mask) -> np.ndarray:
    """Byte mask [T][Sz][Sy][Sx] -> bit words [T][Sz][Sy][ceil(Sx/64)] (uint64),
    bit b of word w of a row = voxel x = 64*w + b; padding bits are zero."""
    m = np.ascontiguousarray(mask, np.uint8).astype(bool)
    T, Sz, Sy, Sx = m.shape
    W = (Sx + 63) // 64
    pad = np.zeros((T, Sz, Sy, W * 64), bool)
    pad[..., :Sx] = m
    by = np.packbits(pad.reshape(T, Sz, Sy, W * 8, 8), axis=-1, bitorder="little")
    return by.reshape(T, Sz, Sy, W * 8).view(np.uint64).reshape(T, Sz, Sy, W).copy()


# --------------------------------------------------------------------------- workloads
def tiny_volume(seed=SEED_FIELD + 1, shape=(32, 32, 32, 8), n_blobs=8):
    """The tiny parity workload: field, dilated feature mask (value > 0.1, r = 1)."""
    blobs = blob_params(seed, n_blobs, (0.05, 0.15), (0.5, 1.0), 0.05)
    f = field(shape, blobs, clip01=True)
    mask = dilate(threshold(f, 0.1), 1)
    return f, mask


def production_volume_host(shape, seed, n_blobs=64):
    """Host version of the production-shape generator (small shapes only)."""
    blobs = blob_params(seed, n_blobs, (0.02, 0.08), (0.5, 1.0), 0.004)
    f = field(shape, blobs, turb_amp=0.25, noise_seed=seed * 7919 + 17, clip01=False,
              normalise=True)
    g = grad_mag(f)
    thr = quantile(g, 0.8)
    mask = dilate(threshold(g, thr), 2)
    return f, mask


def table_init(n_slots, n_features, seed=SEED_INIT, scale=1e-4):
    """Uniform initialisation of every embedding (Sec. 3.2.4), U(-1e-4, 1e-4)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(n_slots, n_features)).astype(np.float32)


def mlp_init(width, seed=SEED_INIT + 1):
    """PyTorch nn.Linear default init: W, b ~ U(-1/sqrt(in), 1/sqrt(in)); packed
    per layer as W[out][in] then b[out]."""
    rng = np.random.default_rng(seed)
    parts = []
    for k in range(len(width) - 1):
        bound = 1.0 / np.sqrt(width[k])
        parts.append(rng.uniform(-bound, bound, size=width[k + 1] * width[k]))
        parts.append(rng.uniform(-bound, bound, size=width[k + 1]))
    return np.concatenate(parts).astype(np.float32)


def probe_points(n, seed=SEED_PROBE):
    """Continuous probe positions U[0,1)^4 (x, y, z, t)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 4), dtype=np.float64).astype(np.float32)
