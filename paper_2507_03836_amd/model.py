"""F-Hash model state on the device and the training / inference steps.

Everything numerical runs in libfhash (HIP); this module only owns the torch
allocations (tables, MLP parameters, Adam moments, workspaces) and sequences
the C-ABI calls of one training step:

    fhash_sample -> fhash_fused_train -> fhash_step

Parameter memory is one flat FP32 vector per quantity (parameters, gradients,
Adam m and v): the embedding tables (rows x F, level after level) followed by
the packed MLP parameters, so one dense Adam launch covers every parameter.

Mixed precision (precision="mixed"): the fused kernels read an FP16 copy of
the tables that the Adam sweep rewrites from the FP32 master values (the
shadow; table_reads="f32" reads the FP32 master instead and keeps no copy)
and run the decoder on 16-bit MFMA (BF16 by default, `decoder`),
accumulating in FP32; gradients, Adam moments and master weights stay FP32.
The loss is scaled by a dynamic factor (start 2^16, doubled after
`scale_window` clean steps, halved with the step skipped when a gradient is
not finite: the output-bias gradient is the sum of every sample's output
gradient, so a non-finite sample gradient shows up there).

Touched-segment tracking (on by default): a step's scatter-add writes only a
small part of the fine levels' gradient, so the scatter flags every 64-byte
gradient segment it writes from the first level of at least 2^21 segments
(128 MiB of FP32 table) on, and the Adam sweep reads the gradient only in
flagged segments there (zero elsewhere).  The update is the dense Adam update
of every parameter either way.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib as fl


@dataclasses.dataclass
class FHashConfig:
    res: list                 # per level (x, y, z, t) vertex counts, level 0 coarsest
    n_features: int = 2
    hidden: int = 64
    n_hidden: int = 2
    lr: float = 0.01
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    layout: int = 0           # slot order of the active index: 0 rows (F-Hash order), 1 bricks

    @property
    def n_levels(self) -> int:
        return len(self.res)

    @property
    def width(self) -> list:
        return [self.n_levels * self.n_features] + [self.hidden] * self.n_hidden + [1]


def geometric_resolutions(L, rmin_s, rmax_s, rmin_t, rmax_t, dims):
    """R_l = floor(Rmin * b^l + 0.5), b = (Rmax/Rmin)^(1/(L-1)), clamped to [2, S_d]."""
    out = []
    for l in range(L):
        r = []
        for d in range(4):
            lo, hi = (rmin_s, rmax_s) if d < 3 else (rmin_t, rmax_t)
            v = lo if L == 1 else lo * ((hi / lo) ** (1.0 / (L - 1))) ** l
            R = int(np.floor(v + 0.5))
            r.append(max(2, min(R, int(dims[d]))))
        out.append(r)
    return out


class FHashModel:
    """Device-resident F-Hash model (index + tables + decoder + Adam state)."""

    def __init__(self, cfg: FHashConfig, mask_bits: torch.Tensor | None, dims, device="cuda",
                 table_init: torch.Tensor | None = None, mlp_init: torch.Tensor | None = None,
                 init_seed: int = 3000, precision: str = "fp32", loss_scale: float = 2.0 ** 16,
                 scale_window: int = 2000, track_touched: bool = True, lazy: bool = False,
                 max_steps: int = 1 << 16, hash_bits: int = 0, decoder: str | None = None,
                 paired_moments: bool = False, moments_with_params: bool = False,
                 table_reads: str | None = None):
        if precision not in ("fp32", "mixed"):
            raise ValueError(f"precision must be 'fp32' or 'mixed', not {precision!r}")
        if decoder is None:
            decoder = "bf16" if precision == "mixed" else "f32"
        if decoder not in ("f32", "f16", "bf16"):
            raise ValueError(f"decoder must be 'f32', 'f16' or 'bf16', not {decoder!r}")
        if table_reads is None:
            table_reads = "f16" if precision == "mixed" else "f32"
        if table_reads not in ("f32", "f16") or (table_reads == "f16" and precision != "mixed"):
            raise ValueError(f"table_reads must be 'f32', or 'f16' under mixed precision, "
                             f"not {table_reads!r}")
        self.table_reads = table_reads
        self.cfg = cfg
        self.precision = precision
        self.decoder = decoder
        self.device = torch.device(device)
        self.grid = fl.grid_desc(cfg.res, cfg.n_features,
                                 fl.LAYOUT_ROWS if mask_bits is None else cfg.layout)
        self.mlp = fl.mlp_desc(cfg.width, {"f32": fl.F32, "f16": fl.F16, "bf16": fl.BF16}[decoder])
        if hash_bits:  # spatial-hash comparison index (mask not used)
            self.index, self.slots_per_level = fl.fhash_hash_index(self.grid, hash_bits)
            self._dir = None
        else:
            self.index, self.slots_per_level, self._dir, _ws = fl.fhash_build_index(
                self.grid, mask_bits, dims)
            del _ws
        self.rows = int(self.index.slot_offset[cfg.n_levels])
        self.n_table = self.rows * cfg.n_features
        self.n_mlp = fl.fhash_mlp_num_params(self.mlp)
        # pad the table part to a multiple of 4 floats so the MLP part is 16-byte aligned
        self.mlp_off = (self.n_table + 3) // 4 * 4
        self.n_params = self.mlp_off + self.n_mlp
        n_alloc = (self.n_params + 3) // 4 * 4
        f32 = dict(dtype=torch.float32, device=self.device)
        self.paired = bool(paired_moments)
        self.moments_with_params = bool(moments_with_params)
        # the vector Adam sees as one: every parameter, or with the moments
        # stored beside the parameters the table part only (the decoder then
        # has arrays of its own and a second, dense update)
        n_vec = (self.mlp_off + 15) // 16 * 16 if self.moments_with_params else n_alloc
        self.n_vec = n_vec
        self.pm = self.gv = self.mv = None
        if self.moments_with_params:
            # runs of 16 table parameters, each followed by their 16 m values,
            # and runs of their 16 gradients, each followed by their 16 v
            # values: a segment's optimiser state is two 128-byte lines, and
            # the lines the forward gathers from take none of the atomics
            self.pm = torch.zeros(2 * n_vec, **f32)
            self.gv = torch.zeros(2 * n_vec, **f32)
            self.m, self.v = self.pm[16:], self.gv[16:]
            self.params = self.grads = None
            n_mlp4 = (self.n_mlp + 3) // 4 * 4
            self.mlp_p = torch.zeros(n_mlp4, **f32)
            self.mlp_g = torch.zeros(n_mlp4, **f32)
            self.mlp_m = torch.zeros(n_mlp4, **f32)
            self.mlp_v = torch.zeros(n_mlp4, **f32)
        else:
            self.params = torch.zeros(n_alloc, **f32)
            self.grads = torch.zeros(n_alloc, **f32)
            # Adam moments: separate arrays, or paired (blocks of 16 m then the
            # same parameters' 16 v: one 128-byte line per segment for the
            # deferred update); m and v then point into the pair array
            if self.paired:
                self.mv = torch.zeros((n_vec + 15) // 16 * 32, **f32)
                self.m, self.v = self.mv, self.mv[16:]
            else:
                self.m = torch.zeros(n_vec, **f32)
                self.v = torch.zeros(n_vec, **f32)
        if table_init is not None:
            table0 = table_init.reshape(-1).to(**f32)
        else:
            g = torch.Generator(device=self.device)
            g.manual_seed(init_seed)
            table0 = torch.empty(self.n_table, **f32).uniform_(-1e-4, 1e-4, generator=g)
        self._set_table(table0)
        del table0
        if mlp_init is not None:
            self.mlp_params.copy_(mlp_init.reshape(-1))
        else:
            g = torch.Generator(device="cpu")
            g.manual_seed(init_seed + 1)
            parts = []
            w = cfg.width
            for k in range(len(w) - 1):
                bound = 1.0 / np.sqrt(w[k])
                parts.append(torch.empty(w[k + 1] * w[k]).uniform_(-bound, bound, generator=g))
                parts.append(torch.empty(w[k + 1]).uniform_(-bound, bound, generator=g))
            self.mlp_params.copy_(torch.cat(parts))
        self.step_count = 0
        self.loss_sum = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._ws = None
        # FHASH_COARSE_LDS: the coarse levels' gradient summed in LDS per chunk
        # of the batch before its atomics
        self.coarse_lds = False
        self.shadow = None
        self.loss_scale = 1.0
        self.touch = None
        self._touch_flags = None
        self.lazy = None
        # large levels (2^21 segments of 16 floats or more): tracked or deferred
        F, seg = cfg.n_features, fl.TOUCH_FLOATS
        first = next((l for l in range(cfg.n_levels)
                      if self.slots_per_level[l] * F // seg >= (1 << 21)), None)
        begin = None if first is None else int(self.index.slot_offset[first]) * F // seg * seg
        if lazy:
            # deferred Adam on [begin, end of the padded table); dense elsewhere
            self.lazy = fl.LazyState(0 if begin is None else begin, self.mlp_off, max_steps,
                                     device=self.device, moments=self._moments_layout())
        elif track_touched and begin is not None:
            self._touch_flags = torch.zeros((self.n_table + seg - 1) // seg,
                                            dtype=torch.uint8, device=self.device)
            self.touch = fl.touch_desc(self._touch_flags, begin, self.n_table)
        if table_reads == "f16":
            self.shadow = torch.zeros(n_vec, dtype=torch.float16, device=self.device)
            if self.moments_with_params:
                fl.fhash_cast(self.table, self.shadow[: self.n_table])
            else:
                fl.fhash_cast(self.params, self.shadow)
        if precision == "mixed":
            self.found_inf = torch.zeros(1, dtype=torch.int32, device=self.device)
            self.loss_scale = float(loss_scale)
            self.scale_window = int(scale_window)
            self._clean = 0
            self.skipped = 0

    # views into the flat vectors (copies of the table part when the moments
    # are stored beside the parameters)
    @staticmethod
    def _runs(a: torch.Tensor, k: int) -> torch.Tensor:
        """The values of an array of 32-float blocks: first (k = 0) or second
        (k = 1) 16 of every block, as one flat copy."""
        return a.view(-1, 2, 16)[:, k].reshape(-1)

    @property
    def table(self) -> torch.Tensor:
        if self.moments_with_params:
            return self._runs(self.pm, 0)[: self.n_table]
        return self.params[: self.n_table]

    def _set_table(self, t: torch.Tensor):
        if self.moments_with_params:
            full = torch.zeros(self.n_vec, dtype=torch.float32, device=self.device)
            full[: self.n_table] = t
            self.pm.view(-1, 2, 16)[:, 0] = full.view(-1, 16)
        else:
            self.params[: self.n_table] = t

    @property
    def read_table(self):
        """The table the fused kernels read: the FP16 shadow or the FP32 master
        (fl.Paired when the moments are stored beside the parameters)."""
        if self.shadow is not None:
            return self.shadow[: self.n_table]
        return fl.Paired(self.pm) if self.moments_with_params else self.table

    @property
    def mlp_params(self) -> torch.Tensor:
        if self.moments_with_params:
            return self.mlp_p[: self.n_mlp]
        return self.params[self.mlp_off: self.mlp_off + self.n_mlp]

    @property
    def d_table(self) -> torch.Tensor:
        if self.moments_with_params:
            return self._runs(self.gv, 0)[: self.n_table]
        return self.grads[: self.n_table]

    @property
    def d_mlp(self) -> torch.Tensor:
        if self.moments_with_params:
            return self.mlp_g[: self.n_mlp]
        return self.grads[self.mlp_off: self.mlp_off + self.n_mlp]

    def _grad_args(self):
        """(d_table pointer tensor, extra fused flags) of the table gradient."""
        if self.moments_with_params:
            return self.gv, fl.GRAD_PAIRED
        return self.d_table, 0

    def flat_params(self) -> torch.Tensor:
        """Every parameter as one flat vector [table | pad | decoder] (a copy in
        the paired parameter layout)."""
        if not self.moments_with_params:
            return self.params[: self.n_params]
        out = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        out[: self.n_table] = self.table
        out[self.mlp_off:] = self.mlp_params
        return out

    def flat_grads(self) -> torch.Tensor:
        if not self.moments_with_params:
            return self.grads[: self.n_params]
        out = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        out[: self.n_table] = self.d_table
        out[self.mlp_off:] = self.d_mlp
        return out

    def _moments_layout(self) -> int:
        if self.moments_with_params:
            return fl.MOMENTS_WITH_PARAMS
        return fl.MOMENTS_PAIRED if self.paired else fl.MOMENTS_SEPARATE

    def moments(self):
        """(m, v) of the parameters as flat arrays (copies in the layouts with
        runs)."""
        n = self.n_params
        if self.moments_with_params:
            m, v = self._runs(self.pm, 1), self._runs(self.gv, 1)
        elif self.paired:
            m, v = self._runs(self.mv, 0), self._runs(self.mv, 1)
        else:
            m, v = self.m, self.v
        if not self.moments_with_params:
            return m[:n], v[:n]
        mm = torch.zeros(n, dtype=torch.float32, device=self.device)
        vv = torch.zeros_like(mm)
        mm[: self.mlp_off], vv[: self.mlp_off] = m[: self.mlp_off], v[: self.mlp_off]
        mm[self.mlp_off:], vv[self.mlp_off:] = self.mlp_m[: self.n_mlp], self.mlp_v[: self.n_mlp]
        return mm, vv

    def adam_desc(self, step: int, grad_scale: float = 1.0) -> fl.AdamDesc:
        c = self.cfg
        o = fl.AdamDesc()
        o.lr, o.beta1, o.beta2, o.eps = c.lr, c.beta1, c.beta2, c.eps
        o.step = step
        o.grad_scale = grad_scale
        o.moments = self._moments_layout()
        return o

    def _pg(self):
        """(param, grad) arguments of the table vector for the optimiser calls."""
        if self.moments_with_params:
            return self.pm, self.gv
        return self.params, self.grads

    def prepare(self, pos: torch.Tensor, phases: int = fl.LAZY_PREPARE):
        """Under deferred Adam: bring the table rows that pos reads up to date
        (and enrol them in the next step)."""
        if self.lazy is not None:
            p, g = self._pg()
            fl.fhash_lazy_prepare(self.index, pos, pos.shape[0], self.lazy, p, g, self.m, self.v,
                                  shadow=self.shadow, phases=phases)

    def flush(self):
        """Under deferred Adam: bring every parameter up to date and apply the
        pending gradients (before the whole table is read: rendering, export)."""
        if self.lazy is not None:
            p, g = self._pg()
            fl.fhash_lazy_flush(self.lazy, p, g, self.m, self.v, shadow=self.shadow)

    def forward(self, pos: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        n = pos.shape[0]
        self.prepare(pos)
        if y is None:
            y = torch.empty(n, dtype=torch.float32, device=self.device)
        fl.fhash_fused_fwd(self.index, self.mlp, pos, n, self.read_table, self.mlp_params, y)
        return y

    def fwd_bwd(self, pos: torch.Tensor, target: torch.Tensor, loss_scale: float | None = None,
                sorted_batch: bool = False, prepared: bool = False):
        """Fused forward + MSE + backward; gradients accumulate into self.grads
        (multiplied by the loss scale; the model's own scale when None).
        prepared: the caller has already called prepare(pos)."""
        n = pos.shape[0]
        s = self.loss_scale if loss_scale is None else loss_scale
        if not prepared:
            self.prepare(pos)
        d_table, gflag = self._grad_args()
        self._ws = fl.fhash_fused_train(self.index, self.mlp, pos, target, n, self.read_table,
                                        self.mlp_params, d_table, self.d_mlp,
                                        self.loss_sum, s, ws=self._ws,
                                        flags=(fl.SAMPLES_SORTED if sorted_batch else 0) | gflag
                                        | (fl.COARSE_LDS if self.coarse_lds else 0),
                                        touch=self.touch)

    def optimizer_step(self, grad_scale: float | None = None, found_inf=None) -> bool:
        """Adam over every parameter (dense, or deferred on the large levels
        with the same results); gradients are reset.  The mixed path
        unscales, skips the update on a non-finite gradient and adapts the
        loss scale.  Returns whether the parameters were updated."""
        if self.precision != "mixed":
            self.step_count += 1
            self._step(self.adam_desc(self.step_count, 1.0 if grad_scale is None else grad_scale),
                       None, found_inf)
            return True
        self.found_inf.zero_()
        fl.fhash_check_finite(self.d_mlp, self.found_inf)
        opt = self.adam_desc(self.step_count + 1, 1.0 / self.loss_scale)
        self._step(opt, self.shadow, self.found_inf)
        if int(self.found_inf.item()):
            self.loss_scale *= 0.5
            self._clean = 0
            self.skipped += 1
            return False
        self.step_count += 1
        self._clean += 1
        if self._clean >= self.scale_window:
            self.loss_scale *= 2.0
            self._clean = 0
        return True

    def _step(self, opt, shadow, found_inf):
        p, g = self._pg()
        n = self.n_vec if self.moments_with_params else self.n_params
        args = (opt, p, g, self.m, self.v)
        if self.lazy is not None:
            fl.fhash_step_lazy(*args, self.lazy, shadow=shadow, found_inf=found_inf, n=n)
        else:
            fl.fhash_step(*args, shadow=shadow, found_inf=found_inf, touch=self.touch, n=n)
        if self.moments_with_params:
            # the decoder: its own dense arrays, same step constants
            om = self.adam_desc(opt.step, opt.grad_scale)
            om.moments = fl.MOMENTS_SEPARATE
            fl.fhash_step(om, self.mlp_p, self.mlp_g, self.mlp_m, self.mlp_v,
                          found_inf=found_inf, n=self.n_mlp)

    def train_step(self, pos: torch.Tensor, target: torch.Tensor):
        self.fwd_bwd(pos, target)
        self.optimizer_step()


def psnr_on(model: FHashModel, pos: torch.Tensor, target: torch.Tensor, chunk: int = 1 << 20):
    """Volume-space PSNR (data range 1): the decoder output on pos against
    target, squared errors summed on the device in FP64 (fhash_sq_err_sum)."""
    acc = torch.zeros(1, dtype=torch.float64, device=model.device)
    y = torch.empty(min(chunk, pos.shape[0]), dtype=torch.float32, device=model.device)
    for s in range(0, pos.shape[0], chunk):
        e = min(s + chunk, pos.shape[0])
        yy = y[: e - s]
        model.forward(pos[s:e], yy)
        fl.fhash_sq_err_sum(yy, target[s:e], e - s, acc)
    mse = acc.item() / pos.shape[0]
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else float("inf")
