"""The optimiser layout with the moments stored beside the parameters (a
segment's 16 parameters followed by their 16 m values in one array, its 16
gradients followed by their 16 v values in another: FHASH_MOMENTS_WITH_PARAMS,
with the table read as FHASH_F32_PAIRED and the gradient written with
FHASH_GRAD_PAIRED) changes where the state lives, not the arithmetic:

- reading the table stored in runs gives the bits of reading the dense table
  (encoding and fused forward);
- the fused backward writes the same gradient into the gradient array's runs
  (up to the FP32 summation order of the atomics, and of the decoder
  gradient's adds into the workgroups' LDS images);
- Adam, dense and deferred, FP32 and mixed precision, follows the separate
  layout's trajectory bit for bit when both models receive the same gradient
  at every step: forward values between steps, and after a flush every
  parameter, moment, gradient and FP16 shadow value.
"""
import numpy as np
import pytest
import torch

from paper_2507_03836_amd import synth

from workloads import tiny_volume

pytestmark = pytest.mark.gpu

TINY_RES = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


def _models(precision, lazy, begin_level=0, **kw):
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd.model import FHashConfig, FHashModel
    f, mask = tiny_volume()
    T, Sz, Sy, Sx = mask.shape
    dims = [Sx, Sy, Sz, T]
    cfg = FHashConfig(res=TINY_RES, n_features=2, hidden=32, n_hidden=2)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    probe = FHashModel(cfg, bits, dims, precision=precision, track_touched=False)
    rows = probe.rows
    del probe
    rng = np.random.default_rng(81)
    table0 = torch.from_numpy(rng.uniform(-0.3, 0.3, (rows, 2)).astype(np.float32))
    mlp0 = torch.from_numpy(synth.mlp_init(cfg.width, seed=82))
    mk = lambda paired: FHashModel(cfg, bits, dims, table_init=table0, mlp_init=mlp0,
                                   precision=precision, track_touched=False, lazy=lazy,
                                   paired_moments=not paired, moments_with_params=paired,
                                   **kw)
    sep, par = mk(False), mk(True)
    if lazy and begin_level:
        for mo in (sep, par):
            begin = int(mo.index.slot_offset[begin_level]) * 2 // 16 * 16
            mo.lazy = fl.LazyState(begin, mo.mlp_off, 64, moments=mo._moments_layout())
    return cfg, sep, par


def _same(a, b, what):
    a = a.view(torch.int32) if a.dtype == torch.float32 else a
    b = b.view(torch.int32) if b.dtype == torch.float32 else b
    assert torch.equal(a, b), what


def _set_grads(model, flat):
    """Write a flat [table | pad | decoder] gradient into a model's arrays."""
    if model.moments_with_params:
        full = torch.zeros(model.n_vec, dtype=torch.float32, device=flat.device)
        full[: model.n_table] = flat[: model.n_table]
        model.gv.view(-1, 2, 16)[:, 0] = full.view(-1, 16)
        model.mlp_g[: model.n_mlp] = flat[model.mlp_off:]
    else:
        model.grads[: model.n_params] = flat


def test_paired_table_reads_are_the_dense_reads(fl):
    _, sep, par = _models("fp32", lazy=False)
    assert par.pm.numel() == par.gv.numel() == 2 * par.n_vec and par.params is None
    _same(par.table, sep.table, "table after init")
    g = torch.Generator().manual_seed(3)
    pos = torch.rand(3000, 4, generator=g).cuda()
    L, F = len(TINY_RES), 2
    e0 = torch.empty(3000, L * F, device="cuda")
    e1 = torch.empty_like(e0)
    fl.fhash_encode_fwd(sep.index, pos, 3000, sep.table, e0)
    fl.fhash_encode_fwd(par.index, pos, 3000, fl.Paired(par.pm), e1)
    _same(e1, e0, "encoding")
    _same(par.forward(pos), sep.forward(pos), "fused forward")


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_paired_gradient_scatter(fl, precision):
    _, sep, par = _models(precision, lazy=False)
    g = torch.Generator().manual_seed(4)
    pos = torch.rand(4000, 4, generator=g).cuda()
    tgt = torch.rand(4000, generator=g).cuda()
    sep.fwd_bwd(pos, tgt)
    par.fwd_bwd(pos, tgt)
    torch.cuda.synchronize()
    # decoder gradient: the same per-sample terms, summed in arrival order
    da, db = par.d_mlp, sep.d_mlp
    assert torch.allclose(da, db, rtol=1e-5, atol=1e-6 * db.abs().max().item())
    a, b = par.d_table, sep.d_table
    assert bool((b != 0).any())
    mag = b.abs().max().item()
    assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * mag), (a - b).abs().max().item()
    # nothing written into the parameter or moment runs
    _same(par.table, sep.table, "parameters untouched by the backward")
    assert not bool(par.pm.view(-1, 2, 16)[:, 1].any())
    assert not bool(par.gv.view(-1, 2, 16)[:, 1].any())


def _run(fl, sep, par, steps, batch, flush_at=(), inf_at=()):
    g = torch.Generator().manual_seed(11 + batch)
    for s in range(steps):
        pos = torch.rand(batch, 4, generator=g).cuda()
        tgt = torch.rand(batch, generator=g).cuda()
        _same(par.forward(pos), sep.forward(pos), f"batch forward, step {s}")
        # one gradient for both: computed by the separate model, handed to the
        # paired one (whose own prepare keeps its deferred state in step)
        sep.fwd_bwd(pos, tgt)
        par.prepare(pos)
        if s in inf_at:
            sep.grads[sep.mlp_off] = float("inf")
        _set_grads(par, sep.flat_grads().clone())
        assert sep.optimizer_step() == par.optimizer_step()
        if s % 3 == 1:
            probe = torch.rand(97, 4, generator=g).cuda()
            _same(par.forward(probe), sep.forward(probe), f"probe forward, step {s}")
        if s in flush_at:
            sep.flush()
            par.flush()
    sep.flush()
    par.flush()
    torch.cuda.synchronize()
    _same(par.flat_params(), sep.flat_params(), "parameters")
    _same(par.flat_grads(), sep.flat_grads(), "gradients")
    for name, a, b in zip(("m", "v"), par.moments(), sep.moments()):
        _same(a, b, name)
    if sep.shadow is not None:
        n = sep.n_table
        _same(par.shadow[:n], sep.shadow[:n], "shadow")


@pytest.mark.parametrize("lazy,begin_level", [(False, 0), (True, 0), (True, 2)])
def test_moments_with_params_follow_separate_fp32(fl, lazy, begin_level):
    _, sep, par = _models("fp32", lazy=lazy, begin_level=begin_level)
    _run(fl, sep, par, steps=10, batch=300, flush_at=(4,))
    assert sep.step_count == par.step_count == 10


def test_moments_with_params_follow_separate_mixed_with_skipped_step(fl):
    _, sep, par = _models("mixed", lazy=True, begin_level=1, loss_scale=2.0 ** 12)
    _run(fl, sep, par, steps=10, batch=64, inf_at=(3,))
    assert sep.skipped == par.skipped == 1
    assert sep.loss_scale == par.loss_scale


def test_layout_arguments_checked(fl):
    _, sep, par = _models("fp32", lazy=True)
    o = par.adam_desc(1)
    n = par.n_vec
    with pytest.raises(fl.FHashError) as e:  # m must be param + 16
        fl.fhash_step(o, par.pm, par.gv, par.pm[32:], par.v, n=n)
    assert e.value.code == fl.EINVAL
    with pytest.raises(fl.FHashError) as e:  # v must be grad + 16
        fl.fhash_step(o, par.pm, par.gv, par.m, par.gv[32:], n=n)
    assert e.value.code == fl.EINVAL
    o.moments = fl.MOMENTS_PAIRED  # differs from the deferred state's layout
    with pytest.raises(fl.FHashError) as e:
        fl.fhash_step_lazy(o, par.pm, par.gv, par.m, par.v, par.lazy, n=n)
    assert e.value.code == fl.EINVAL
    pos = torch.rand(16, 4).cuda()
    tgt = torch.rand(16).cuda()
    with pytest.raises(fl.FHashError) as e:  # unknown flag bit
        fl.fhash_fused_train(par.index, par.mlp, pos, tgt, 16, fl.Paired(par.pm), par.mlp_params,
                             par.gv, par.d_mlp, flags=8)
    assert e.value.code == fl.EINVAL
