"""ctypes binding of libfhash.so (the C ABI declared in include/fhash.h).

Argument marshalling only: every function here has the name of the C entry
point it calls, takes torch tensors for device buffers, passes their raw
pointers and the current HIP stream, and raises FHashError on a non-zero
status.  No computation happens in Python.  There is no CPU fallback: loading
fails loudly when the HIP library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfhash.so")

MAX_LEVELS = 24
MAX_LAYERS = 8
F32, F16, BF16, F32_PAIRED = 0, 1, 2, 3
OK, EINVAL, ENOMEM, EHIP, ERANGE, ENOTSUP = 0, -1, -2, -3, -4, -5
_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", ERANGE: "ERANGE", ENOTSUP: "ENOTSUP"}


class FHashError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func}: {_STATUS.get(code, code)}: {msg}")
        self.code = code


LAYOUT_ROWS, LAYOUT_BRICKS = 0, 1


class GridDesc(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_features", C.c_int32),
                ("res", (C.c_int32 * 4) * MAX_LEVELS), ("layout", C.c_int32)]


class MaskDesc(C.Structure):
    _fields_ = [("bits", C.c_void_p), ("dims", C.c_int64 * 4)]


class Index(C.Structure):
    _fields_ = [("grid", GridDesc), ("active", C.c_int32), ("hash_bits", C.c_int32),
                ("dir", C.c_void_p), ("dir_offset", C.c_int64 * (MAX_LEVELS + 1)),
                ("slot_offset", C.c_int64 * (MAX_LEVELS + 1))]


class MlpDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("width", C.c_int32 * (MAX_LAYERS + 1)),
                ("compute_dt", C.c_int32)]


MOMENTS_SEPARATE, MOMENTS_PAIRED, MOMENTS_WITH_PARAMS = 0, 1, 2


class AdamDesc(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("step", C.c_int64), ("grad_scale", C.c_double),
                ("moments", C.c_int64)]


class View(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("fwd", C.c_float * 3), ("right", C.c_float * 3),
                ("up", C.c_float * 3), ("tan_half_fovy", C.c_float), ("aspect", C.c_float)]


class RenderOpts(C.Structure):
    _fields_ = [("ds", C.c_float), ("alpha_stop", C.c_float), ("arm_max", C.c_int32),
                ("max_steps", C.c_int32)]


class RenderState(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("t", C.c_float), ("cur", C.c_int32),
                ("n_alive", C.c_int32), ("pending", C.c_int32), ("iterations", C.c_int64),
                ("samples", C.c_int64), ("ws", C.c_void_p), ("dims", C.c_int64 * 4),
                ("t01", C.c_float)]


class RenderStats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("samples", C.c_int64)]


class Touch(C.Structure):
    _fields_ = [("flags", C.c_void_p), ("begin", C.c_int64), ("end", C.c_int64)]


TOUCH_FLOATS = 16


def touch_desc(flags: torch.Tensor, begin: int, end: int) -> Touch:
    """Touched-segment descriptor over a uint8 flag tensor (kept alive by the caller)."""
    t = Touch()
    t.flags = flags.data_ptr()
    t.begin, t.end = int(begin), int(end)
    return t


def _touch(t):
    return None if t is None else C.byref(t)


class Lazy(C.Structure):
    _fields_ = [("ws", C.c_void_p), ("begin", C.c_int64), ("end", C.c_int64),
                ("max_steps", C.c_int64), ("steps", C.c_int64), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("flags", C.c_int64),
                ("moments", C.c_int64)]


LAZY_FLOATS = 16


class LazyState:
    """A deferred-Adam descriptor with its device workspace (see fhash_lazy_init)."""

    def __init__(self, begin: int, end: int, max_steps: int, device="cuda",
                 moments: int = MOMENTS_SEPARATE):
        nb = lib().fhash_lazy_workspace_bytes(int(end) - int(begin), int(max_steps))
        if nb == 0:
            raise ValueError("bad lazy range or max_steps")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.desc = Lazy()
        self.desc.ws = self.ws.data_ptr()
        self.desc.begin, self.desc.end = int(begin), int(end)
        self.desc.max_steps = int(max_steps)
        self.desc.moments = int(moments)
        _check(lib().fhash_lazy_init(C.byref(self.desc), _stream()), "fhash_lazy_init")

    @property
    def steps(self) -> int:
        return int(self.desc.steps)


_lib = None


def lib() -> C.CDLL:
    """Load libfhash.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "python -m paper_2507_03836_amd.build (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    P, I64, U64, I32, F = C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, C.c_float
    sig = {
        "fhash_version": (C.c_int, []),
        "fhash_last_error": (C.c_char_p, []),
        "fhash_index_dir_entries": (C.c_int, [P, P]),
        "fhash_build_index": (C.c_int, [P, P, P, P, P, P, P, P]),
        "fhash_dense_index": (C.c_int, [P, P, P]),
        "fhash_hash_index": (C.c_int, [P, I32, P, P]),
        "fhash_encode_fwd": (C.c_int, [P, P, I64, P, C.c_int, P, P]),
        "fhash_encode_bwd": (C.c_int, [P, P, I64, P, P, P, P]),
        "fhash_corner_rows": (C.c_int, [P, P, I64, P, P, P]),
        "fhash_mlp_num_params": (I64, [P]),
        "fhash_mlp_fwd": (C.c_int, [P, P, P, P, I64, P, P]),
        "fhash_mlp_bwd": (C.c_int, [P, P, P, P, P, I64, P, P, P, P, P]),
        "fhash_fused_fwd": (C.c_int, [P, P, P, I64, P, C.c_int, P, P, P, P]),
        "fhash_fused_bwd": (C.c_int, [P, P, P, I64, P, C.c_int, P, P, P, P, P, C.c_uint32, P, P,
                                      P, P]),
        "fhash_fused_train": (C.c_int, [P, P, P, P, I64, P, C.c_int, P, P, F, P, P, P, C.c_uint32,
                                        P, P, P, P]),
        "fhash_step": (C.c_int, [P, P, P, P, P, P, C.c_int, I64, P, P, P]),
        "fhash_lazy_workspace_bytes": (C.c_size_t, [I64, I64]),
        "fhash_lazy_init": (C.c_int, [P, P]),
        "fhash_lazy_prepare": (C.c_int, [P, P, I64, P, P, P, P, P, P, C.c_int, C.c_uint32, P]),
        "fhash_lazy_stats": (C.c_int, [P, P, P]),
        "fhash_step_lazy": (C.c_int, [P, P, P, P, P, P, C.c_int, I64, P, P, P]),
        "fhash_lazy_flush": (C.c_int, [P, P, P, P, P, P, C.c_int, P]),
        "fhash_check_finite": (C.c_int, [P, I64, P, P]),
        "fhash_cast": (C.c_int, [P, P, C.c_int, I64, P]),
        "fhash_sample": (C.c_int, [U64, U64, I64, P, U64, P, P, P, P, P, P, P]),
        "fhash_coreset_frames": (C.c_int, [P, P, P, I32, P, I64, P, P, P, P]),
        "fhash_fold_resolutions": (C.c_int, [P, I32, P, P]),
        "fhash_key_frame_times": (C.c_int, [I64, P, I32, P]),
        "fhash_sq_err_sum": (C.c_int, [P, P, I64, P, P]),
        "fhash_mse_grad": (C.c_int, [P, P, I64, F, P, P, P]),
        "fhash_sort_samples": (C.c_int, [P, P, I64, P, P, P]),
        "fhash_feature_mask": (C.c_int, [P, P, I32, F, F, P, P, P, P]),
        "fhash_dilate_mask": (C.c_int, [P, P, I32, P, P]),
        "fhash_feature_boxes": (C.c_int, [P, P, P, P]),
        "fhash_occupancy_words": (I64, [P]),
        "fhash_occupancy_grid": (C.c_int, [P, P, P, P]),
        "fhash_coreset": (C.c_int, [P, P, P, I64, P, P, P, P]),
        "fhash_render_state_bytes": (C.c_int, [I32, I32, P, P]),
        "fhash_render_begin": (C.c_int, [P, F, I32, I32, P, P, P, C.c_size_t, P, P, P]),
        "fhash_render_begin_grid": (C.c_int, [P, F, I32, I32, P, P, P, C.c_size_t, P, P, P]),
        "fhash_render_pace": (I32, [I64, I64, I32]),
        "fhash_render_march": (C.c_int, [P, P, I32, P, I64, P, P]),
        "fhash_render_composite": (C.c_int, [P, P, P, P, P, P]),
        "fhash_render_march_batch": (C.c_int, [P, P, I32, P, P, I64, I64, P, P, P]),
        "fhash_render_composite_batch": (C.c_int, [P, I32, P, P, P, P, P, P]),
        "fhash_render": (C.c_int, [P, P, P, C.c_int, P, P, P, P, F, P, I32, I32, P, P, P, P, P,
                                   P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


def exported_symbols() -> list[str]:
    return ["fhash_version", "fhash_last_error", "fhash_index_dir_entries", "fhash_build_index",
            "fhash_dense_index", "fhash_hash_index", "fhash_encode_fwd", "fhash_encode_bwd", "fhash_mlp_num_params",
            "fhash_mlp_fwd", "fhash_mlp_bwd", "fhash_fused_fwd", "fhash_fused_bwd",
            "fhash_fused_train", "fhash_step", "fhash_check_finite", "fhash_cast",
            "fhash_sample", "fhash_sq_err_sum", "fhash_mse_grad", "fhash_render_state_bytes",
            "fhash_render_begin", "fhash_render_begin_grid", "fhash_render_pace",
            "fhash_render_march",
            "fhash_render_composite", "fhash_render_march_batch",
            "fhash_render_composite_batch", "fhash_render", "fhash_sort_samples",
            "fhash_lazy_workspace_bytes", "fhash_lazy_init", "fhash_lazy_prepare",
            "fhash_step_lazy", "fhash_lazy_flush", "fhash_lazy_stats", "fhash_feature_mask",
            "fhash_dilate_mask", "fhash_feature_boxes", "fhash_occupancy_words",
            "fhash_occupancy_grid", "fhash_coreset"]


def _check(rc: int, func: str):
    if rc != OK:
        raise FHashError(rc, func, lib().fhash_last_error().decode())


class Paired:
    """A table argument stored in runs of 16 floats separated by 16-float gaps
    (FHASH_F32_PAIRED): the parameter array of the optimiser layout
    MOMENTS_WITH_PARAMS, whose gaps hold the first moments."""

    def __init__(self, t: torch.Tensor):
        if t.dtype != torch.float32:
            raise TypeError("a paired table is FP32")
        self.t = t


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return C.c_void_p(t.data_ptr())
    if isinstance(t, Paired):
        return C.c_void_p(t.t.data_ptr())
    return t


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dt(t) -> int:
    if isinstance(t, Paired):
        return F32_PAIRED
    return {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}[t.dtype]


# --------------------------------------------------------------------------- descriptors
def grid_desc(res, n_features: int, layout: int = LAYOUT_ROWS) -> GridDesc:
    g = GridDesc()
    g.n_levels = len(res)
    g.n_features = n_features
    g.layout = layout
    for l, r in enumerate(res):
        for d in range(4):
            g.res[l][d] = int(r[d])
    return g


def mlp_desc(width, compute_dt: int = F32) -> MlpDesc:
    m = MlpDesc()
    m.n_layers = len(width) - 1
    for k, w in enumerate(width):
        m.width[k] = int(w)
    m.compute_dt = compute_dt
    return m


# --------------------------------------------------------------------------- entry points
def fhash_version() -> int:
    return lib().fhash_version()


def fhash_index_dir_entries(grid: GridDesc) -> int:
    e = C.c_int64()
    _check(lib().fhash_index_dir_entries(C.byref(grid), C.byref(e)), "fhash_index_dir_entries")
    return e.value


def fhash_hash_index(grid: GridDesc, hash_bits: int):
    """Spatial-hash comparison index (host only): (index, rows per level)."""
    idx = Index()
    slots = (C.c_int64 * MAX_LEVELS)()
    _check(lib().fhash_hash_index(C.byref(grid), int(hash_bits), C.byref(idx), slots),
           "fhash_hash_index")
    return idx, [int(slots[l]) for l in range(grid.n_levels)]


def fhash_dense_index(grid: GridDesc):
    idx = Index()
    slots = (C.c_int64 * MAX_LEVELS)()
    _check(lib().fhash_dense_index(C.byref(grid), C.byref(idx), slots), "fhash_dense_index")
    return idx, [slots[l] for l in range(grid.n_levels)]


def fhash_build_index(grid: GridDesc, mask_bits: torch.Tensor | None, dims, dir_buf=None,
                      ws=None):
    """Build the index.  Returns (Index, slots_per_level, dir tensor, ws tensor).
    dir/ws are allocated here with torch when not given (they must outlive the
    index: the Index only points into dir)."""
    L = lib()
    m = MaskDesc()
    m.bits = None if mask_bits is None else mask_bits.data_ptr()
    for d in range(4):
        m.dims[d] = int(dims[d])
    if mask_bits is None:
        return (*fhash_dense_index(grid), None, None)
    dev = mask_bits.device
    nb = C.c_size_t(0)
    _check(L.fhash_build_index(C.byref(grid), C.byref(m), None, None, C.byref(nb), None, None,
                               _stream()), "fhash_build_index")
    if ws is None:
        ws = torch.empty(max(int(nb.value), 16), dtype=torch.uint8, device=dev)
    if dir_buf is None:
        ents = fhash_index_dir_entries(grid)
        dir_buf = torch.empty((ents, 2), dtype=torch.int64, device=dev)
    idx = Index()
    slots = (C.c_int64 * MAX_LEVELS)()
    nb = C.c_size_t(ws.numel() * ws.element_size())
    _check(L.fhash_build_index(C.byref(grid), C.byref(m), _ptr(dir_buf), _ptr(ws), C.byref(nb),
                               C.byref(idx), slots, _stream()), "fhash_build_index")
    return idx, [slots[l] for l in range(grid.n_levels)], dir_buf, ws


def fhash_encode_fwd(idx: Index, pos, n, table, enc):
    _check(lib().fhash_encode_fwd(C.byref(idx), _ptr(pos), n, _ptr(table), _dt(table), _ptr(enc),
                                  _stream()), "fhash_encode_fwd")


def fhash_encode_bwd(idx: Index, pos, n, d_enc, d_table, touch=None):
    _check(lib().fhash_encode_bwd(C.byref(idx), _ptr(pos), n, _ptr(d_enc), _ptr(d_table),
                                  _touch(touch), _stream()), "fhash_encode_bwd")


def fhash_corner_rows(idx: Index, pos, n, out_dir=None, out_slot=None):
    """Directory entries and table rows the encoding of each sample touches
    (instrumentation): two int64 tensors [n][L][8][2]."""
    L = idx.grid.n_levels
    if out_dir is None:
        out_dir = torch.empty((n, L, 8, 2), dtype=torch.int64, device=pos.device)
    if out_slot is None:
        out_slot = torch.empty((n, L, 8, 2), dtype=torch.int64, device=pos.device)
    _check(lib().fhash_corner_rows(C.byref(idx), _ptr(pos), n, _ptr(out_dir), _ptr(out_slot),
                                   _stream()), "fhash_corner_rows")
    return out_dir, out_slot


def fhash_mlp_num_params(mlp: MlpDesc) -> int:
    return int(lib().fhash_mlp_num_params(C.byref(mlp)))


def fhash_mlp_fwd(mlp: MlpDesc, params, x, n, y, shadow=None):
    _check(lib().fhash_mlp_fwd(C.byref(mlp), _ptr(params), _ptr(shadow), _ptr(x), n, _ptr(y),
                               _stream()), "fhash_mlp_fwd")


def _ws_query(fn, args_before_ws, name):
    nb = C.c_size_t(0)
    _check(fn(*args_before_ws, None, C.byref(nb), _stream()), name)
    return int(nb.value)


def fhash_mlp_bwd(mlp: MlpDesc, params, x, dy, n, d_params, dx=None, shadow=None, ws=None):
    L = lib()
    head = (C.byref(mlp), _ptr(params), _ptr(shadow), _ptr(x), _ptr(dy), n, _ptr(d_params),
            _ptr(dx))
    need = _ws_query(L.fhash_mlp_bwd, head, "fhash_mlp_bwd")
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device=params.device)
    nb = C.c_size_t(ws.numel() * ws.element_size())
    _check(L.fhash_mlp_bwd(*head, _ptr(ws), C.byref(nb), _stream()), "fhash_mlp_bwd")
    return ws


def fhash_fused_fwd(idx: Index, mlp: MlpDesc, pos, n, table, params, y, shadow=None):
    _check(lib().fhash_fused_fwd(C.byref(idx), C.byref(mlp), _ptr(pos), n, _ptr(table),
                                 _dt(table), _ptr(params), _ptr(shadow), _ptr(y), _stream()),
           "fhash_fused_fwd")


SAMPLES_SORTED, GRAD_PAIRED, COARSE_LDS = 1, 2, 4


def fhash_fused_bwd(idx: Index, mlp: MlpDesc, pos, n, table, params, dy, d_table, d_params,
                    shadow=None, ws=None, flags=0, touch=None):
    L = lib()
    head = (C.byref(idx), C.byref(mlp), _ptr(pos), n, _ptr(table), _dt(table), _ptr(params),
            _ptr(shadow), _ptr(dy), _ptr(d_table), _ptr(d_params), C.c_uint32(flags),
            _touch(touch))
    need = _ws_query(L.fhash_fused_bwd, head, "fhash_fused_bwd")
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device=params.device)
    nb = C.c_size_t(ws.numel() * ws.element_size())
    _check(L.fhash_fused_bwd(*head, _ptr(ws), C.byref(nb), _stream()), "fhash_fused_bwd")
    return ws


def fhash_fused_train(idx: Index, mlp: MlpDesc, pos, target, n, table, params, d_table,
                      d_params, loss_sum=None, loss_scale=1.0, shadow=None, ws=None, flags=0,
                      touch=None):
    L = lib()
    head = (C.byref(idx), C.byref(mlp), _ptr(pos), _ptr(target), n, _ptr(table), _dt(table),
            _ptr(params), _ptr(shadow), C.c_float(loss_scale), _ptr(d_table), _ptr(d_params),
            _ptr(loss_sum), C.c_uint32(flags), _touch(touch))
    need = _ws_query(L.fhash_fused_train, head, "fhash_fused_train")
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device=params.device)
    nb = C.c_size_t(ws.numel() * ws.element_size())
    _check(L.fhash_fused_train(*head, _ptr(ws), C.byref(nb), _stream()), "fhash_fused_train")
    return ws


def fhash_step(opt: AdamDesc, param, grad, m, v, shadow=None, found_inf=None, touch=None,
               n=None):
    """n: the parameter count (param.numel() by default; pass it for the
    layout MOMENTS_WITH_PARAMS, whose arrays are longer)."""
    sdt = F16 if shadow is None else _dt(shadow)
    n = param.numel() if n is None else int(n)
    _check(lib().fhash_step(C.byref(opt), _ptr(param), _ptr(grad), _ptr(m), _ptr(v),
                            _ptr(shadow), sdt, n, _ptr(found_inf), _touch(touch),
                            _stream()), "fhash_step")


LAZY_MARK, LAZY_CATCH_UP, LAZY_PREPARE = 1, 2, 3


def fhash_lazy_prepare(idx: Index, pos, n, lazy: LazyState, param, grad, m, v, shadow=None,
                       phases=LAZY_PREPARE):
    sdt = F16 if shadow is None else _dt(shadow)
    _check(lib().fhash_lazy_prepare(C.byref(idx), _ptr(pos), n, C.byref(lazy.desc), _ptr(param),
                                    _ptr(grad), _ptr(m), _ptr(v), _ptr(shadow), sdt,
                                    C.c_uint32(phases), _stream()), "fhash_lazy_prepare")


def fhash_lazy_stats(lazy: LazyState) -> dict:
    out = (C.c_int64 * 4)()
    _check(lib().fhash_lazy_stats(C.byref(lazy.desc), out, _stream()), "fhash_lazy_stats")
    return {"segments": out[0], "loaded": out[1], "pending": out[2], "segment_steps": out[3]}


def fhash_step_lazy(opt: AdamDesc, param, grad, m, v, lazy: LazyState, shadow=None,
                    found_inf=None, n=None):
    sdt = F16 if shadow is None else _dt(shadow)
    n = param.numel() if n is None else int(n)
    _check(lib().fhash_step_lazy(C.byref(opt), _ptr(param), _ptr(grad), _ptr(m), _ptr(v),
                                 _ptr(shadow), sdt, n, _ptr(found_inf),
                                 C.byref(lazy.desc), _stream()), "fhash_step_lazy")


def fhash_lazy_flush(lazy: LazyState, param, grad, m, v, shadow=None):
    sdt = F16 if shadow is None else _dt(shadow)
    _check(lib().fhash_lazy_flush(C.byref(lazy.desc), _ptr(param), _ptr(grad), _ptr(m), _ptr(v),
                                  _ptr(shadow), sdt, _stream()), "fhash_lazy_flush")


def fhash_check_finite(grad, found_inf):
    _check(lib().fhash_check_finite(_ptr(grad), grad.numel(), _ptr(found_inf), _stream()),
           "fhash_check_finite")


def fhash_cast(src, dst):
    _check(lib().fhash_cast(_ptr(src), _ptr(dst), _dt(dst), src.numel(), _stream()), "fhash_cast")


def fhash_sample(seed, step, n, coreset, M, dims, field, pos, target, frame_t=None, box=None):
    """frame_t: device float [T] frame times (key-frame training) or None;
    box: 6 ints (inclusive voxel bounds of the spatial frame) or None."""
    d = (C.c_int64 * 4)(*[int(x) for x in dims])
    b = None if box is None else (C.c_int32 * 6)(*[int(x) for x in box])
    _check(lib().fhash_sample(seed, step, n, _ptr(coreset), M, d, _ptr(field), _ptr(frame_t),
                              b, _ptr(pos), _ptr(target), _stream()), "fhash_sample")


def fhash_coreset_frames(bits, dims, frames, ws=None):
    """Coreset ids (int64 view of uint64, increasing) of the listed frames
    only.  Synchronises."""
    L = lib()
    d = _dims(dims)
    fr = (C.c_int32 * max(1, len(frames)))(*[int(x) for x in frames])
    nb = C.c_size_t(0)
    cnt = C.c_int64(0)
    _check(L.fhash_coreset_frames(_ptr(bits), d, fr, len(frames), None, 0, None, C.byref(nb),
                                  C.byref(cnt), None), "fhash_coreset_frames")
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(max(int(nb.value), 16), dtype=torch.uint8, device=bits.device)
    nb = C.c_size_t(ws.numel())
    _check(L.fhash_coreset_frames(_ptr(bits), d, fr, len(frames), None, 0, _ptr(ws), C.byref(nb),
                                  C.byref(cnt), _stream()), "fhash_coreset_frames")
    ids = torch.empty(max(cnt.value, 1), dtype=torch.int64, device=bits.device)
    _check(L.fhash_coreset_frames(_ptr(bits), d, fr, len(frames), _ptr(ids), cnt.value, _ptr(ws),
                                  C.byref(nb), C.byref(cnt), _stream()), "fhash_coreset_frames")
    return ids[:cnt.value]


def fhash_fold_resolutions(size, fold):
    """Level resolutions (list of [x, y, z, t], coarsest first) by the fold policy."""
    s = (C.c_int64 * 4)(*[int(x) for x in size])
    res = (C.c_int32 * (4 * MAX_LEVELS))()
    L = C.c_int32(0)
    _check(lib().fhash_fold_resolutions(s, fold, res, C.byref(L)), "fhash_fold_resolutions")
    return [[res[4 * l + d] for d in range(4)] for l in range(L.value)]


def fhash_key_frame_times(T, frames):
    """FP32 time coordinate of every frame (numpy float32 [T]) under key-frame training."""
    import numpy as np
    fr = (C.c_int32 * len(frames))(*[int(x) for x in frames])
    out = np.zeros(int(T), np.float32)
    _check(lib().fhash_key_frame_times(int(T), fr, len(frames), out.ctypes.data_as(C.c_void_p)),
           "fhash_key_frame_times")
    return out


FEATURE_INTERVAL, FEATURE_ISOSURFACE = 0, 1


def _dims(dims):
    return (C.c_int64 * 4)(*[int(x) for x in dims])


def mask_words(dims) -> int:
    return int(dims[3]) * int(dims[2]) * int(dims[1]) * ((int(dims[0]) + 63) // 64)


def fhash_feature_mask(field, dims, kind, lo, hi=0.0, bits=None):
    """Feature extraction into mask words (int64 tensor [T][Sz][Sy][ceil(Sx/64)],
    allocated here when not given; the isosurface workspace too)."""
    L = lib()
    d = _dims(dims)
    if bits is None:
        bits = torch.empty(mask_words(dims), dtype=torch.int64, device=field.device)
    nb = C.c_size_t(0)
    _check(L.fhash_feature_mask(_ptr(field), d, kind, lo, hi, None, None, C.byref(nb), None),
           "fhash_feature_mask")
    ws = None
    if nb.value:
        ws = torch.empty(nb.value, dtype=torch.uint8, device=field.device)
    _check(L.fhash_feature_mask(_ptr(field), d, kind, lo, hi, _ptr(bits), _ptr(ws),
                                None if ws is None else C.byref(nb), _stream()),
           "fhash_feature_mask")
    return bits


def fhash_dilate_mask(bits_in, dims, r, out=None):
    if out is None:
        out = torch.empty_like(bits_in)
    _check(lib().fhash_dilate_mask(_ptr(bits_in), _dims(dims), r, _ptr(out), _stream()),
           "fhash_dilate_mask")
    return out


def fhash_feature_boxes(bits, dims, box=None):
    if box is None:
        box = torch.empty((int(dims[3]) + 1, 6), dtype=torch.int32, device=bits.device)
    _check(lib().fhash_feature_boxes(_ptr(bits), _dims(dims), _ptr(box), _stream()),
           "fhash_feature_boxes")
    return box


def fhash_occupancy_words(dims) -> int:
    n = lib().fhash_occupancy_words(_dims(dims))
    if n < 0:
        raise FHashError(EINVAL, "fhash_occupancy_words", lib().fhash_last_error().decode())
    return int(n)


def fhash_occupancy_grid(bits, dims, occ=None):
    if occ is None:
        occ = torch.empty(fhash_occupancy_words(dims), dtype=torch.int64, device=bits.device)
    _check(lib().fhash_occupancy_grid(_ptr(bits), _dims(dims), _ptr(occ), _stream()),
           "fhash_occupancy_grid")
    return occ


def fhash_coreset(bits, dims, ws=None):
    """Coreset voxel ids (int64 view of uint64, increasing).  Synchronises."""
    L = lib()
    d = _dims(dims)
    nb = C.c_size_t(0)
    cnt = C.c_int64(0)
    _check(L.fhash_coreset(_ptr(bits), d, None, 0, None, C.byref(nb), C.byref(cnt), None),
           "fhash_coreset")
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(max(int(nb.value), 16), dtype=torch.uint8, device=bits.device)
    nb = C.c_size_t(ws.numel())
    _check(L.fhash_coreset(_ptr(bits), d, None, 0, _ptr(ws), C.byref(nb), C.byref(cnt),
                           _stream()), "fhash_coreset")
    ids = torch.empty(max(cnt.value, 1), dtype=torch.int64, device=bits.device)
    _check(L.fhash_coreset(_ptr(bits), d, _ptr(ids), cnt.value, _ptr(ws), C.byref(nb),
                           C.byref(cnt), _stream()), "fhash_coreset")
    return ids[:cnt.value]


def fhash_sort_samples(pos, target, n, ws=None):
    L = lib()
    nb = C.c_size_t(0)
    _check(L.fhash_sort_samples(_ptr(pos), _ptr(target), n, None, C.byref(nb), _stream()),
           "fhash_sort_samples")
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(max(int(nb.value), 16), dtype=torch.uint8, device=pos.device)
    nb = C.c_size_t(ws.numel())
    _check(L.fhash_sort_samples(_ptr(pos), _ptr(target), n, _ptr(ws), C.byref(nb), _stream()),
           "fhash_sort_samples")
    return ws


def fhash_sq_err_sum(y, v, n, out):
    _check(lib().fhash_sq_err_sum(_ptr(y), _ptr(v), n, _ptr(out), _stream()), "fhash_sq_err_sum")


def fhash_mse_grad(y, v, n, dy, loss_sum=None, loss_scale=1.0):
    _check(lib().fhash_mse_grad(_ptr(y), _ptr(v), n, C.c_float(loss_scale), _ptr(dy),
                                _ptr(loss_sum), _stream()), "fhash_mse_grad")


# --------------------------------------------------------------------------- rendering
def view_struct(v14) -> View:
    """View from 14 floats: eye, fwd, right, up, tan_half_fovy, aspect."""
    v = View()
    for k in range(3):
        v.eye[k], v.fwd[k], v.right[k], v.up[k] = (float(v14[k]), float(v14[3 + k]),
                                                    float(v14[6 + k]), float(v14[9 + k]))
    v.tan_half_fovy, v.aspect = float(v14[12]), float(v14[13])
    return v


def render_opts(ds=0.5, alpha_stop=0.99, arm_max=64, max_steps=1 << 20) -> RenderOpts:
    o = RenderOpts()
    o.ds, o.alpha_stop, o.arm_max, o.max_steps = ds, alpha_stop, arm_max, max_steps
    return o


def _dims(d):
    return (C.c_int64 * 4)(*[int(x) for x in d])


def fhash_render(idx, mlp, table, params, mask_bits, dims, view: View, t, tf, W, H,
                 opts: RenderOpts, rgba, ws=None):
    L = lib()
    head = (C.byref(idx), C.byref(mlp), _ptr(table), _dt(table), _ptr(params), _ptr(mask_bits),
            _dims(dims), C.byref(view), C.c_float(t), _ptr(tf), W, H, C.byref(opts), _ptr(rgba))
    nb = C.c_size_t(0)
    _check(L.fhash_render(*head, None, C.byref(nb), None, _stream()), "fhash_render")
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(max(int(nb.value), 16), dtype=torch.uint8, device=rgba.device)
    nb = C.c_size_t(ws.numel())
    st = RenderStats()
    _check(L.fhash_render(*head, _ptr(ws), C.byref(nb), C.byref(st), _stream()), "fhash_render")
    return st, ws


def fhash_render_state_bytes(W, H, dims) -> int:
    nb = C.c_size_t(0)
    _check(lib().fhash_render_state_bytes(W, H, _dims(dims), C.byref(nb)),
           "fhash_render_state_bytes")
    return int(nb.value)


def fhash_render_begin(view: View, t, W, H, mask_bits, dims, ws, rgba) -> RenderState:
    st = RenderState()
    _check(lib().fhash_render_begin(C.byref(view), C.c_float(t), W, H, _ptr(mask_bits),
                                    _dims(dims), _ptr(ws), ws.numel() * ws.element_size(),
                                    _ptr(rgba), C.byref(st), _stream()), "fhash_render_begin")
    return st


def fhash_render_begin_grid(view: View, t, W, H, occ, dims, ws, rgba) -> RenderState:
    """fhash_render_begin from the coreset's occupancy grid (fhash_occupancy_grid)."""
    st = RenderState()
    _check(lib().fhash_render_begin_grid(C.byref(view), C.c_float(t), W, H, _ptr(occ),
                                         _dims(dims), _ptr(ws), ws.numel() * ws.element_size(),
                                         _ptr(rgba), C.byref(st), _stream()),
           "fhash_render_begin_grid")
    return st


def fhash_render_pace(budget, alive, arm_max) -> int:
    return int(lib().fhash_render_pace(int(budget), int(alive), int(arm_max)))


def fhash_render_march(st: RenderState, opts: RenderOpts, pace, pos_out, cap) -> int:
    ns = C.c_int64(0)
    _check(lib().fhash_render_march(C.byref(st), C.byref(opts), pace, _ptr(pos_out), cap,
                                    C.byref(ns), _stream()), "fhash_render_march")
    return ns.value


RENDER_BATCH_MAX = 32


def _state_array(states):
    return (C.POINTER(RenderState) * len(states))(*[C.pointer(st) for st in states])


def fhash_render_march_batch(states, paces, opts: RenderOpts, pos, out_base, cap, counts) -> list:
    """One march launch over several requests; samples go to pos[out_base:],
    interleaved.  counts: device int32 tensor of at least 1 + len(states)."""
    n = len(states)
    ns = (C.c_int64 * n)()
    _check(lib().fhash_render_march_batch(_state_array(states), (C.c_int32 * n)(*paces), n,
                                          C.byref(opts), _ptr(pos), int(out_base), int(cap),
                                          _ptr(counts), ns, _stream()),
           "fhash_render_march_batch")
    return list(ns)


def fhash_render_composite_batch(states, y, tfs, opts: RenderOpts, rgbas, counts) -> list:
    """One composite launch over several requests (y in the march's frame);
    returns each request's alive-ray count."""
    n = len(states)
    tf = (C.c_void_p * n)(*[t.data_ptr() for t in tfs])
    rg = (C.c_void_p * n)(*[t.data_ptr() for t in rgbas])
    _check(lib().fhash_render_composite_batch(_state_array(states), n, _ptr(y), tf, rg,
                                              C.byref(opts), _ptr(counts), _stream()),
           "fhash_render_composite_batch")
    return [int(st.n_alive) for st in states]


def fhash_render_composite(st: RenderState, y, tf, opts: RenderOpts, rgba):
    _check(lib().fhash_render_composite(C.byref(st), _ptr(y), _ptr(tf), C.byref(opts), _ptr(rgba),
                                        _stream()), "fhash_render_composite")
