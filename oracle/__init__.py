"""F-Hash FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the F-Hash hot path
computes (oracle.c, FP64 C).  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product path
never does.  It shares no code with the HIP library: the two meet only through
the seeded input generators and through plain numpy arrays.

Parity status of each function is documented in oracle.h / the test-suite:
every routine here is pinned by tests that do not reuse its own formula.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAX_LEVELS = 32


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-o", _LIB_PATH, os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


P = C.c_void_p
I64 = C.c_int64
U64 = C.c_uint64


class OrGrid(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_features", C.c_int32),
                ("res", (C.c_int64 * 4) * MAX_LEVELS),
                ("slot_offset", C.c_int64 * (MAX_LEVELS + 1)),
                ("vtx_offset", C.c_int64 * (MAX_LEVELS + 1)),
                ("slot_map", P)]


def _declare(L):
    L.or_fold_num_levels.restype = C.c_int
    L.or_fold_num_levels.argtypes = [I64, I64]
    L.or_fold_resolutions.restype = C.c_int
    L.or_fold_resolutions.argtypes = [P, I64, C.c_int, P]
    L.or_geometric_resolutions.restype = C.c_int
    L.or_geometric_resolutions.argtypes = [C.c_int, I64, I64, I64, I64, P, P]
    L.or_voxel_cells.restype = None
    L.or_voxel_cells.argtypes = [I64, I64, I64, P, P]
    L.or_cell_activity.restype = None
    L.or_cell_activity.argtypes = [P, P, P, P]
    L.or_build_level_slots.restype = I64
    L.or_build_level_slots.argtypes = [P, P, P, P]
    L.or_build_level_slots_bricks.restype = I64
    L.or_build_level_slots_bricks.argtypes = [P, P, P, P]
    L.or_cell_active_bits.restype = C.c_int
    L.or_cell_active_bits.argtypes = [P, P, P, P]
    L.or_vertex_active_bits.restype = C.c_int
    L.or_vertex_active_bits.argtypes = [P, P, P, P]
    L.or_locate.restype = None
    L.or_locate.argtypes = [C.c_float, I64, P, P]
    L.or_corners.restype = None
    L.or_corners.argtypes = [P, P, I64, P, P]
    L.or_encode_fwd.restype = None
    L.or_encode_fwd.argtypes = [P, P, I64, P, P, P]
    L.or_encode_bwd.restype = None
    L.or_encode_bwd.argtypes = [P, P, I64, P, P, P]
    L.or_mlp_num_params.restype = I64
    L.or_mlp_num_params.argtypes = [C.c_int, P]
    L.or_mlp_fwd.restype = None
    L.or_mlp_fwd.argtypes = [C.c_int, P, P, P, I64, P, P, P, P]
    L.or_mlp_bwd.restype = None
    L.or_mlp_bwd.argtypes = [C.c_int, P, P, P, P, P, P, I64, P, P, P, P]
    L.or_mse.restype = C.c_double
    L.or_mse.argtypes = [P, P, I64, P]
    L.or_adam.restype = None
    L.or_adam.argtypes = [P, P, P, P, I64, C.c_double, C.c_double, C.c_double, C.c_double, I64]
    L.or_psnr.restype = C.c_double
    L.or_psnr.argtypes = [C.c_double]
    L.or_philox4x32_10.restype = None
    L.or_philox4x32_10.argtypes = [P, P, P]
    L.or_sample_ids.restype = None
    L.or_sample_ids.argtypes = [U64, U64, I64, U64, P]
    L.or_voxel_positions.restype = None
    L.or_voxel_positions.argtypes = [P, I64, P, P]
    L.or_occupied.restype = C.c_int
    L.or_occupied.argtypes = [P, P, P, C.c_float]
    L.or_render.restype = I64
    L.or_render.argtypes = [P, P, C.c_int, P, P, P, P, P, C.c_float, C.c_float, P, C.c_int,
                            C.c_int, C.c_float, C.c_float, C.c_int, P, P, P]
    L.or_sample_batch.restype = None
    L.or_sample_batch.argtypes = [U64, U64, I64, P, U64, P, P, P, P]


def _p(a):
    return None if a is None else a.ctypes.data_as(P)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------- resolutions
def fold_num_levels(S: int, f: int) -> int:
    return lib().or_fold_num_levels(S, f)


def fold_resolutions(S4, f: int) -> np.ndarray:
    """Paper fold policy; rows are paper levels 1..L_s (row 0 = finest)."""
    S = _c(S4, np.int64)
    out = np.zeros((MAX_LEVELS, 4), np.int64)
    L = lib().or_fold_resolutions(_p(S), f, MAX_LEVELS, _p(out))
    if L < 0:
        raise ValueError("too many levels")
    return out[:L].copy()


def geometric_resolutions(L, rmin_s, rmax_s, rmin_t, rmax_t, S4) -> np.ndarray:
    """Geometric policy; row 0 = coarsest level."""
    S = _c(S4, np.int64)
    out = np.zeros((MAX_LEVELS, 4), np.int64)
    if lib().or_geometric_resolutions(L, rmin_s, rmax_s, rmin_t, rmax_t, _p(S), _p(out)) < 0:
        raise ValueError("bad level count")
    return out[:L].copy()


# --------------------------------------------------------------------------- index
def voxel_cells(i, S, R):
    lo, hi = C.c_int64(), C.c_int64()
    lib().or_voxel_cells(i, S, R, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def cell_activity(res4, mask: np.ndarray) -> np.ndarray:
    """mask: uint8 [T][Sz][Sy][Sx]; returns uint8 [Rt-1][Rz-1][Ry-1][Rx-1]."""
    r = _c(res4, np.int64)
    m = _c(mask, np.uint8)
    S = np.array([m.shape[3], m.shape[2], m.shape[1], m.shape[0]], np.int64)
    out = np.zeros((r[3] - 1, r[2] - 1, r[1] - 1, r[0] - 1), np.uint8)
    lib().or_cell_activity(_p(r), _p(m), _p(S), _p(out))
    return out


LAYOUT_ROWS, LAYOUT_BRICKS = 0, 1


def level_slots(res4, mask, layout: int = LAYOUT_ROWS):
    """Slot map of one level (vertex -> slot within level, -1 inactive), count.
    layout: rank in the F-Hash equation's order, or in 2^4-vertex bricks."""
    r = _c(res4, np.int64)
    nv = int(np.prod(r))
    out = np.zeros(nv, np.int64)
    fn = lib().or_build_level_slots_bricks if layout == LAYOUT_BRICKS else \
        lib().or_build_level_slots
    if mask is None:
        S = np.zeros(4, np.int64)
        cnt = fn(_p(r), None, _p(S), _p(out))
    else:
        m = _c(mask, np.uint8)
        S = np.array([m.shape[3], m.shape[2], m.shape[1], m.shape[0]], np.int64)
        cnt = fn(_p(r), _p(m), _p(S), _p(out))
    if cnt < 0:
        raise RuntimeError("brick ranking lost a vertex")
    return out, int(cnt)


def vertex_active_bits(res4, bits, dims, v):
    """Activity of vertex v = (x, y, z, t) of a level, from a row-padded bit mask
    (uint64 [T][Sz][Sy][ceil(Sx/64)]); dims = (Sx, Sy, Sz, T)."""
    r = _c(res4, np.int64)
    b = _c(bits, np.uint64)
    S = _c(dims, np.int64)
    vv = _c(v, np.int64)
    return bool(lib().or_vertex_active_bits(_p(r), _p(b), _p(S), _p(vv)))


HASH_PRIMES = (1, 2654435761, 805459861, 3674653429)


def spatial_hash_slots(res4, bits: int):
    """Comparison index (not the method; parity unpinned as values, pinned by
    properties in tests/test_oracle_hash.py): the row of every vertex of a level
    under the 4D spatial hash of multiresolution hash encodings, written from
    its definition: with the F-Hash order lin = ((t Rz + z) Ry + y) Rx + x, row
    = (x*1 XOR y*2654435761 XOR z*805459861 XOR t*3674653429) mod 2^32 mod
    2^bits, products taken mod 2^32.  A level of at most 2^bits vertices keeps
    the F-Hash equation (row = lin)."""
    Rx, Ry, Rz, Rt = (int(v) for v in res4)
    nv = Rx * Ry * Rz * Rt
    lin = np.arange(nv, dtype=np.uint64)
    if nv <= (1 << bits):
        return lin.astype(np.int64), nv
    coord = [lin % Rx, (lin // Rx) % Ry, (lin // (Rx * Ry)) % Rz, lin // (Rx * Ry * Rz)]
    h = np.zeros(nv, np.uint64)
    for c, prime in zip(coord, HASH_PRIMES):
        h ^= (c * np.uint64(prime)) % np.uint64(1 << 32)
    return (h % np.uint64(1 << bits)).astype(np.int64), 1 << bits


class Grid:
    """Oracle-side level structure + (optional) active-vertex slot maps.
    hash_bits > 0 (no mask): the spatial-hash comparison index.
    layout: LAYOUT_ROWS (ranks in the F-Hash equation's order) or LAYOUT_BRICKS
    (ranks in 2 x 2 x 2 x 2 vertex bricks; active index only)."""

    def __init__(self, res, n_features, mask=None, hash_bits: int = 0,
                 layout: int = LAYOUT_ROWS):
        res = np.asarray(res, np.int64).reshape(-1, 4)
        self.res = res
        self.L = res.shape[0]
        self.F = n_features
        self.layout = layout
        self.maps = []
        self.counts = []
        if layout == LAYOUT_BRICKS and (mask is None or hash_bits):
            raise ValueError("the brick order is built for the active-vertex index")
        for l in range(self.L):
            if hash_bits:
                m, c = spatial_hash_slots(res[l], hash_bits)
                self.maps.append(m)
                self.counts.append(c)
                continue
            if mask is None:  # dense box: the slot is the F-Hash equation, no map needed
                self.counts.append(int(np.prod(res[l])))
                continue
            m, c = level_slots(res[l], mask, layout)
            self.maps.append(m)
            self.counts.append(c)
        self.dense = mask is None and not hash_bits
        self.slot_offset = np.zeros(self.L + 1, np.int64)
        self.slot_offset[1:] = np.cumsum(self.counts)
        self.vtx_offset = np.zeros(self.L + 1, np.int64)
        self.vtx_offset[1:] = np.cumsum([int(np.prod(r)) for r in res])
        self._map = None if self.dense else np.concatenate(self.maps)
        g = OrGrid()
        g.n_levels = self.L
        g.n_features = n_features
        for l in range(self.L):
            for d in range(4):
                g.res[l][d] = int(res[l][d])
        for l in range(self.L + 1):
            g.slot_offset[l] = int(self.slot_offset[l])
            g.vtx_offset[l] = int(self.vtx_offset[l])
        g.slot_map = None if self.dense else self._map.ctypes.data_as(P)
        self._g = g

    @property
    def total_slots(self) -> int:
        return int(self.slot_offset[-1])

    def ref(self):
        return C.byref(self._g)


def locate(p: float, R: int):
    c, f = C.c_int64(), C.c_double()
    lib().or_locate(C.c_float(p), R, C.byref(c), C.byref(f))
    return c.value, f.value


def corners(grid: Grid, pos):
    pos = _c(pos, np.float32)
    n = pos.shape[0]
    slots = np.zeros((n, grid.L, 16), np.int64)
    w = np.zeros((n, grid.L, 16), np.float64)
    lib().or_corners(grid.ref(), _p(pos), n, _p(slots), _p(w))
    return slots, w


def encode_fwd(grid: Grid, pos, table):
    pos = _c(pos, np.float32)
    tab = _c(table, np.float64)
    n = pos.shape[0]
    enc = np.zeros((n, grid.L * grid.F), np.float64)
    mag = np.zeros_like(enc)
    lib().or_encode_fwd(grid.ref(), _p(pos), n, _p(tab), _p(enc), _p(mag))
    return enc, mag


def encode_bwd(grid: Grid, pos, d_enc):
    pos = _c(pos, np.float32)
    de = _c(d_enc, np.float64)
    n = pos.shape[0]
    dt = np.zeros((grid.total_slots, grid.F), np.float64)
    mag = np.zeros((grid.total_slots, grid.F), np.float64)  # zero pages, committed where written
    lib().or_encode_bwd(grid.ref(), _p(pos), n, _p(de), _p(dt), _p(mag))
    return dt, mag


# --------------------------------------------------------------------------- MLP
def mlp_num_params(width) -> int:
    w = _c(width, np.int32)
    return int(lib().or_mlp_num_params(len(w) - 1, _p(w)))


def mlp_fwd(width, params, x, x_mag=None):
    w = _c(width, np.int32)
    nl = len(w) - 1
    prm = _c(params, np.float64)
    x = _c(x, np.float64)
    n = x.shape[0]
    y = np.zeros((n, w[-1]), np.float64)
    acts = np.zeros(int(n * w.sum()), np.float64)
    ymag = np.zeros_like(y)
    xm = None if x_mag is None else _c(x_mag, np.float64)
    lib().or_mlp_fwd(nl, _p(w), _p(prm), _p(x), n, _p(y), _p(acts), _p(xm), _p(ymag))
    return y, acts, ymag


def mlp_bwd(width, params, acts, dy, n, dy_mag=None, x_mag=None):
    w = _c(width, np.int32)
    nl = len(w) - 1
    prm = _c(params, np.float64)
    acts = _c(acts, np.float64)
    dy = _c(dy, np.float64)
    dp = np.zeros(prm.shape[0], np.float64)
    dpm = np.zeros_like(dp)
    dx = np.zeros((n, w[0]), np.float64)
    dxm = np.zeros_like(dx)
    dym = None if dy_mag is None else _c(dy_mag, np.float64)
    xm = None if x_mag is None else _c(x_mag, np.float64)
    lib().or_mlp_bwd(nl, _p(w), _p(prm), _p(acts), _p(dy), _p(dym), _p(xm), n, _p(dp), _p(dx),
                     _p(dpm), _p(dxm))
    return dp, dx, dpm, dxm


# --------------------------------------------------------------------------- loss / adam / psnr
def mse(y, v):
    y = _c(y, np.float64).ravel()
    v = _c(v, np.float64).ravel()
    dy = np.zeros_like(y)
    L = lib().or_mse(_p(y), _p(v), y.shape[0], _p(dy))
    return L, dy


def adam(p, g, m, v, lr, beta1, beta2, eps, step):
    """In-place on float64 arrays p, m, v."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    lib().or_adam(_p(p), _p(g), _p(m), _p(v), p.size, lr, beta1, beta2, eps, step)


def psnr(mse_value: float) -> float:
    return float(lib().or_psnr(mse_value))


# --------------------------------------------------------------------------- RNG / sampler
def philox4x32_10(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def sample_ids(seed, step, n, M):
    ids = np.zeros(n, np.uint64)
    lib().or_sample_ids(seed, step, n, M, _p(ids))
    return ids


def voxel_positions(lin, dims):
    """FP32 sample positions of linear voxel ids; dims = (Sx, Sy, Sz, T)."""
    lin = _c(lin, np.uint64)
    S = _c(dims, np.int64)
    pos = np.zeros((lin.shape[0], 4), np.float32)
    lib().or_voxel_positions(_p(lin), lin.shape[0], _p(S), _p(pos))
    return pos


def sample_batch(seed, step, n, field, coreset=None):
    """field: float32 [T][Sz][Sy][Sx].  Returns pos [n][4] f32, target [n] f32."""
    f = _c(field, np.float32)
    S = np.array([f.shape[3], f.shape[2], f.shape[1], f.shape[0]], np.int64)
    pos = np.zeros((n, 4), np.float32)
    tgt = np.zeros(n, np.float32)
    if coreset is None:
        M = int(f.size)
        cs = None
    else:
        cs = _c(coreset, np.uint64)
        M = int(cs.shape[0])
    lib().or_sample_batch(seed, step, n, _p(cs), M, _p(S), _p(f), _p(pos), _p(tgt))
    return pos, tgt



# --------------------------------------------------------------------------- key frames
def key_frame_times(T: int, frames) -> np.ndarray:
    """Time coordinate of every frame of a model trained on key frames (Sec.
    3.2.2: the temporal resolution of the finest level is the number of key
    frames, so key frame k is vertex k of that level, at k / (n_kf - 1)).
    Reading for the frames between key frames: linear in the frame index
    between the two neighbouring key frames; before the first key frame 0,
    after the last 1.  Exact rationals, rounded once to FP32."""
    from fractions import Fraction
    fr = [int(x) for x in frames]
    K = len(fr)
    out = np.zeros(int(T), np.float32)
    for n in range(int(T)):
        if n <= fr[0]:
            tau = Fraction(0)
        elif n >= fr[-1]:
            tau = Fraction(1)
        else:
            k = max(i for i in range(K) if fr[i] <= n)
            tau = (k + Fraction(n - fr[k], fr[k + 1] - fr[k])) / (K - 1)
        out[n] = np.float32(float(tau))  # the double nearest the rational, then to FP32
    return out


def sample_batch_frames(seed, step, n, field, coreset, frame_t=None, box=None):
    """The training batch of or_sample_batch with the time coordinate of frame
    t taken from frame_t[t] (key-frame training), and the spatial coordinates
    those of the box (xmin, ymin, zmin, xmax, ymax, zmax) when given (Sec. 3.1,
    position translation and scaling to the FBB, on [0,1]).  FP32 IEEE
    division, as or_voxel_positions."""
    f = _c(field, np.float32)
    T, Sz, Sy, Sx = f.shape
    cs = _c(coreset, np.uint64) if coreset is not None else None
    M = int(cs.shape[0]) if cs is not None else int(f.size)
    ids = sample_ids(seed, step, n, M)
    lin = cs[ids.astype(np.int64)] if cs is not None else ids
    lin = lin.astype(np.int64)
    t, z, y, x = np.unravel_index(lin, (T, Sz, Sy, Sx))
    lo = np.zeros(3, np.int64) if box is None else np.asarray(box[:3], np.int64)
    ext = (np.array([Sx, Sy, Sz]) - 1) if box is None else (np.asarray(box[3:], np.int64) - lo)
    pos = np.zeros((n, 4), np.float32)
    for d, c in enumerate((x, y, z)):
        pos[:, d] = (c - lo[d]).astype(np.float32) / np.float32(ext[d])
    if frame_t is None:
        pos[:, 3] = t.astype(np.float32) / np.float32(T - 1)
    else:
        pos[:, 3] = np.asarray(frame_t, np.float32)[t]
    return pos, f.ravel()[lin]


# --------------------------------------------------------------------------- render
def render(grid: Grid, table, width, params, mask, view14, t, tf, W, H, ds=0.5,
           alpha_stop=0.99, max_steps=1 << 20, pixel_stats=False, t01=None):
    """Oracle image [H][W][4] (FP64), ambiguity flags [H][W], evaluated samples;
    with pixel_stats also [H][W][3]: composited samples, sum of their output
    magnitudes, smallest |A - alpha_stop| over the composited steps.  t01: the
    model's time coordinate of the samples (default t / (T - 1); a model
    trained on key frames takes its frame time)."""
    tab = _c(table, np.float64)
    w = _c(width, np.int32)
    prm = _c(params, np.float64)
    m = _c(mask, np.uint8)
    S = np.array([m.shape[3], m.shape[2], m.shape[1], m.shape[0]], np.int64)
    cam = _c(view14, np.float32)
    tfa = _c(tf, np.float32)
    rgba = np.zeros((H, W, 4), np.float64)
    amb = np.zeros((H, W), np.uint8)
    pix = np.zeros((H, W, 3), np.float64)
    ev = lib().or_render(grid.ref(), _p(tab), len(w) - 1, _p(w), _p(prm), _p(m), _p(S), _p(cam),
                         C.c_float(t), C.c_float(-1.0 if t01 is None else t01), _p(tfa), W, H,
                         C.c_float(ds), C.c_float(alpha_stop), max_steps, _p(rgba), _p(amb),
                         _p(pix))
    if pixel_stats:
        return rgba, amb.astype(bool), int(ev), pix
    return rgba, amb.astype(bool), int(ev)


def occupied(mask, p3, t):
    m = _c(mask, np.uint8)
    S = np.array([m.shape[3], m.shape[2], m.shape[1], m.shape[0]], np.int64)
    p = _c(p3, np.float32)
    return bool(lib().or_occupied(_p(m), _p(S), _p(p), C.c_float(t)))
