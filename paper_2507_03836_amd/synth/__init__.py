"""Seeded synthetic inputs shaped like the paper's time-varying volumes.

This module produces inputs only (fields, the gradient-magnitude attribute
and the threshold value that define the feature, initial parameters, probe
points, cameras); it holds none of the method's arithmetic and is the one
place that both the HIP path and the CPU oracle take their inputs from.  The
feature masks and coresets are computed from these inputs by the method's own
code: the coreset-selection calls on the GPU, oracle/coreset.py in the tests.

Workload recipe (shapes/distributions of the paper's datasets, which are not
available: scalar float32 fields normalised to [0,1], sparse moving features,
hundreds of voxels per side, tens to a hundred timesteps):

* tiny     : 32^3 x 8, 8 advected Gaussian blobs (centre U[0,1]^3, sigma
             U[0.05,0.15], amplitude U[0.5,1], velocity U[-0.05,0.05]^3 per
             step), clipped to [0,1]; feature = value > 0.1, dilated by 1.
* production: 64 blobs (sigma U[0.02,0.08], amplitude U[0.5,1], velocity
             U[-0.004,0.004]^3) + 0.25 * 3-octave 4D value noise, min-max
             normalised; feature = |grad| > its 80th percentile, dilated by 2.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_HOST_LIB = os.path.join(_HERE, "libfhash_synth_host.so")
_GPU_LIB = os.path.join(_HERE, "libfhash_synth_gpu.so")

SEED_FIELD, SEED_SAMPLER, SEED_INIT, SEED_PROBE, SEED_ARRIVALS = 1000, 2000, 3000, 4000, 5000


def build_host(force: bool = True) -> str:
    if force or not os.path.exists(_HOST_LIB):
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", _HOST_LIB,
                        os.path.join(_HERE, "synth.c"), "-lm"], check=True)
    return _HOST_LIB


def build_gpu(force: bool = True) -> str:
    if force or not os.path.exists(_GPU_LIB):
        subprocess.run(["/opt/rocm/bin/hipcc", "-O3", "-fPIC", "-shared", "--offload-arch=gfx950",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-o", _GPU_LIB, os.path.join(_HERE, "synth_gpu.hip")], check=True,
                       capture_output=True)
    return _GPU_LIB


_lib = None
_glib = None


def _G():
    global _glib
    if _glib is None:
        if not os.path.exists(_GPU_LIB):
            raise ImportError(f"{_GPU_LIB} missing; run synth.build_gpu()")
        L = C.CDLL(_GPU_LIB)
        P, I64, U64, D = C.c_void_p, C.c_int64, C.c_uint64, C.c_double
        L.sy_gpu_field.argtypes = [P, P, C.c_int, D, U64, C.c_int, P, P]
        L.sy_gpu_normalise.argtypes = [P, I64, P, P]
        L.sy_gpu_grad_mag.argtypes = [P, P, P, P]
        L.sy_gpu_select.argtypes = [P, I64, I64, P, P, P]
        for n in ("sy_gpu_field", "sy_gpu_normalise", "sy_gpu_grad_mag", "sy_gpu_select"):
            getattr(L, n).restype = C.c_int
        _glib = L
    return _glib


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
TINY_FEATURE_LO, TINY_DILATION = 0.1, 1
PRODUCTION_QUANTILE, PRODUCTION_DILATION = 0.8, 2


def tiny_field(seed=SEED_FIELD + 1, shape=(32, 32, 32, 8), n_blobs=8):
    """The tiny parity workload's field; its feature is value > TINY_FEATURE_LO,
    dilated by TINY_DILATION."""
    blobs = blob_params(seed, n_blobs, (0.05, 0.15), (0.5, 1.0), 0.05)
    return field(shape, blobs, clip01=True)


def production_field_host(shape, seed, n_blobs=64):
    """Host version of the production-shape generator (small shapes only):
    field, gradient-magnitude attribute, and the feature threshold value (its
    PRODUCTION_QUANTILE order statistic); the feature is |grad| > threshold,
    dilated by PRODUCTION_DILATION."""
    blobs = blob_params(seed, n_blobs, (0.02, 0.08), (0.5, 1.0), 0.004)
    f = field(shape, blobs, turb_amp=0.25, noise_seed=seed * 7919 + 17, clip01=False,
              normalise=True)
    g = grad_mag(f)
    return f, g, quantile(g, PRODUCTION_QUANTILE)


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


def production_field_gpu(shape_xyzt, seed, n_blobs=64, quantile_q=PRODUCTION_QUANTILE,
                         keep_field=True):
    """Device version of production_field_host (same definitions) for large shapes.

    Returns dict(field=float32 [T][Sz][Sy][Sx] device tensor (or None),
    grad=its gradient magnitude (device), threshold=the quantile_q order
    statistic of grad, N=voxel count)."""
    import torch

    G = _G()
    Sx, Sy, Sz, T = shape_xyzt
    dims = np.array(shape_xyzt, np.int64)
    N = int(np.prod(dims))
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    blobs = torch.from_numpy(blob_params(seed, n_blobs, (0.02, 0.08), (0.5, 1.0), 0.004)).cuda()
    f = torch.empty((T, Sz, Sy, Sx), dtype=torch.float32, device="cuda")
    assert G.sy_gpu_field(_p(dims), C.c_void_p(blobs.data_ptr()), n_blobs, 0.25,
                          seed * 7919 + 17, 0, C.c_void_p(f.data_ptr()), st) == 0
    mm = torch.empty(2, dtype=torch.int32, device="cuda")
    assert G.sy_gpu_normalise(C.c_void_p(f.data_ptr()), N, C.c_void_p(mm.data_ptr()), st) == 0
    g = torch.empty_like(f)
    assert G.sy_gpu_grad_mag(_p(dims), C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr()), st) == 0
    hist = torch.empty(4096, dtype=torch.int64, device="cuda")
    thr = C.c_float()
    rank = min(int(np.floor(quantile_q * N)), N - 1)
    assert G.sy_gpu_select(C.c_void_p(g.data_ptr()), N, rank, C.c_void_p(hist.data_ptr()),
                           C.byref(thr), st) == 0
    if not keep_field:
        del f
        f = None
    torch.cuda.synchronize()
    return dict(field=f, grad=g, threshold=thr.value, N=N)


# --------------------------------------------------------------------------- render inputs
def orbit_view(dims, azimuth, elevation, W, H, fovy_deg=45.0, dist_factor=2.0):
    """Orbit camera around the volume box [0, S-1]^3 (voxel units): distance
    dist_factor x the box half-diagonal from its centre, looking at the centre,
    world z up.  Returns 14 float32: eye, fwd, right, up, tan(fovy/2), W/H
    (basis in FP64, rounded once)."""
    c = np.array([(dims[0] - 1) / 2.0, (dims[1] - 1) / 2.0, (dims[2] - 1) / 2.0])
    r = dist_factor * float(np.linalg.norm(c))
    ca, sa, ce, se = np.cos(azimuth), np.sin(azimuth), np.cos(elevation), np.sin(elevation)
    eye = c + r * np.array([ce * ca, ce * sa, se])
    fwd = c - eye
    fwd = fwd / np.sqrt((fwd * fwd).sum())
    wup = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, wup)
    right = right / np.sqrt((right * right).sum())
    up = np.cross(right, fwd)
    v = np.concatenate([eye, fwd, right, up, [np.tan(np.radians(fovy_deg) / 2.0), W / H]])
    return v.astype(np.float32)


def transfer_function():
    """Fixed 256-entry RGBA transfer function: a warm ramp in colour and an
    opacity ramp that is transparent below 0.15 and reaches 0.4 at 1."""
    v = np.arange(256) / 255.0
    r = np.clip(1.5 * v, 0, 1)
    g = np.clip(1.5 * v - 0.5, 0, 1)
    b = np.clip(0.6 - v, 0, 1)
    a = np.clip((v - 0.15) / 0.85, 0, 1) * 0.4
    return np.stack([r, g, b, a], axis=1).astype(np.float32)
