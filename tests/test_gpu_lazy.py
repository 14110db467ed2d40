"""Deferred Adam (fhash_lazy_prepare / fhash_step_lazy / fhash_lazy_flush)
against the dense update (fhash_step over every parameter at every step).

The two models start from the same values and receive the same gradient at
every step (the deferred model computes it with the fused kernel after its
prepare call; the dense model gets a copy of what that backward wrote), so the
two trajectories must be identical bit for bit:

- every forward value read between steps (training batch and probe points)
  is equal, i.e. every prepared segment holds the dense values;
- after a flush, parameters, moments, FP16 shadow and gradients are equal
  everywhere, also with a flush in the middle of the run, a deferred range that
  starts inside the table (dense prefix), and a step that a non-finite
  gradient skips (mixed precision).
"""
import numpy as np
import pytest
import torch

from paper_2507_03836_amd import synth

from workloads import coreset_ids, tiny_volume

pytestmark = pytest.mark.gpu

TINY_RES = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


def _pair(precision, begin_level, dense_kw=None, lazy_kw=None, **kw):
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
    rng = np.random.default_rng(71)
    table0 = torch.from_numpy(rng.uniform(-0.3, 0.3, (rows, 2)).astype(np.float32))
    mlp0 = torch.from_numpy(synth.mlp_init(cfg.width, seed=72))
    mk = lambda **a: FHashModel(cfg, bits, dims, table_init=table0, mlp_init=mlp0,
                                precision=precision, **a, **kw)
    dense = mk(track_touched=False, **(dense_kw or {}))
    lazy = mk(lazy=True, **(lazy_kw or {}))
    if begin_level:
        begin = int(lazy.index.slot_offset[begin_level]) * 2 // 16 * 16
        lazy.lazy = fl.LazyState(begin, lazy.mlp_off, 64, moments=lazy._moments_layout())
    return cfg, dense, lazy


def _same(a, b, what):
    assert torch.equal(a.view(torch.int32) if a.dtype == torch.float32 else a,
                       b.view(torch.int32) if b.dtype == torch.float32 else b), what


def _fresh_mask(lazy):
    """Where the open step's backward writes: in the deferred range only the
    segments enrolled in that step (others may still hold an earlier step's
    gradient, applied at their next catch-up), everywhere else."""
    lz = lazy.lazy
    b, e = lz.desc.begin, lz.desc.end
    nseg = (e - b + 15) // 16
    stamp = lz.ws[: nseg * 8].view(torch.int32).view(nseg, 2)[:, 1]
    mask = torch.ones(lazy.grads.numel(), dtype=torch.bool, device=lazy.grads.device)
    mask[b:e] = (stamp == lz.steps + 1).repeat_interleave(16)[: e - b]
    return mask


def _fresh_grad(lazy):
    """The gradient the open step's backward wrote."""
    return torch.where(_fresh_mask(lazy), lazy.grads, torch.zeros_like(lazy.grads))


def _run(fl, dense, lazy, steps, batch, flush_at=(), inf_at=()):
    g = torch.Generator().manual_seed(5 + batch)
    for s in range(steps):
        pos = torch.rand(batch, 4, generator=g).cuda()
        tgt = torch.rand(batch, generator=g).cuda()
        # forward values after the prepare equal the dense model's
        _same(lazy.forward(pos), dense.forward(pos), f"batch forward, step {s}")
        lazy.fwd_bwd(pos, tgt)
        if s in inf_at:
            lazy.grads[lazy.mlp_off] = float("inf")
        dense.grads.copy_(_fresh_grad(lazy))
        assert dense.optimizer_step() == lazy.optimizer_step()
        if s % 3 == 1:
            probe = torch.rand(97, 4, generator=g).cuda()
            _same(lazy.forward(probe), dense.forward(probe), f"probe forward, step {s}")
        if s in flush_at:
            lazy.flush()
    lazy.flush()
    torch.cuda.synchronize()
    n = dense.n_params
    for name in ("params", "grads"):
        _same(getattr(lazy, name)[:n], getattr(dense, name)[:n], name)
    for name, a, b in zip(("m", "v"), lazy.moments(), dense.moments()):
        _same(a, b, name)
    if dense.shadow is not None:
        _same(lazy.shadow[:n], dense.shadow[:n], "shadow")
    assert lazy.lazy.steps == steps
    assert bool((dense.grads == 0).all())


@pytest.mark.parametrize("begin_level,batch", [(0, 40), (2, 40), (0, 1000)])
def test_lazy_equals_dense_fp32(fl, begin_level, batch):
    _, dense, lazy = _pair("fp32", begin_level)
    _run(fl, dense, lazy, steps=14, batch=batch, flush_at=(6,))
    # the parameters did move (a no-op optimiser would also be "equal")
    assert dense.step_count == 14


@pytest.mark.parametrize("dense_paired,lazy_paired", [(False, True), (True, True), (True, False)])
def test_paired_moments_equal_separate(fl, dense_paired, lazy_paired):
    """The paired moments layout (a segment's m and v in one 128-byte line)
    changes where m and v live, not a bit of the update: dense and deferred,
    either layout, against each other."""
    _, dense, lazy = _pair("fp32", 2, dense_kw={"paired_moments": dense_paired},
                           lazy_kw={"paired_moments": lazy_paired})
    assert dense.paired == dense_paired and lazy.paired == lazy_paired
    _run(fl, dense, lazy, steps=10, batch=200, flush_at=(4,))
    assert dense.step_count == 10


def test_lazy_equals_dense_mixed_with_skipped_step(fl):
    _, dense, lazy = _pair("mixed", 1, loss_scale=2.0 ** 12)
    _run(fl, dense, lazy, steps=12, batch=64, inf_at=(4,))
    assert lazy.skipped == dense.skipped == 1
    assert lazy.step_count == dense.step_count == 11
    assert lazy.loss_scale == dense.loss_scale


def test_lazy_replay_is_exercised(fl):
    """Segments really are deferred: before a flush, some parameter the run
    never read differs from the dense value (its missed steps are pending)."""
    _, dense, lazy = _pair("fp32", 0)
    g = torch.Generator().manual_seed(3)
    # step 1 touches many rows, steps 2-5 only a few: the rows of step 1 lag
    for s, b in enumerate([3000, 8, 8, 8, 8]):
        pos = torch.rand(b, 4, generator=g).cuda()
        tgt = torch.rand(b, generator=g).cuda()
        lazy.fwd_bwd(pos, tgt)
        dense.grads.copy_(_fresh_grad(lazy))
        dense.optimizer_step()
        lazy.optimizer_step()
    n = dense.n_table
    assert not torch.equal(lazy.params[:n], dense.params[:n])
    st = fl.fhash_lazy_stats(lazy.lazy)
    # the 8-sample steps re-read some step-1 rows: loaded, pending, replayed
    assert 0 < st["pending"] <= st["loaded"] <= st["segments"]
    assert st["segment_steps"] >= st["pending"]
    lazy.flush()
    _same(lazy.params[:n], dense.params[:n], "params after flush")
    _same(lazy.m[:n], dense.m[:n], "m after flush")


def test_lazy_limits(fl):
    _, dense, lazy = _pair("fp32", 0)
    lz = fl.LazyState(0, lazy.mlp_off, 2)
    lazy.lazy = lz
    pos = torch.rand(16, 4).cuda()
    tgt = torch.rand(16).cuda()
    for _ in range(2):
        lazy.fwd_bwd(pos, tgt)
        lazy.optimizer_step()
    lazy.fwd_bwd(pos, tgt)
    with pytest.raises(fl.FHashError) as e:
        lazy.optimizer_step()
    assert e.value.code == fl.ERANGE
    lz2 = fl.LazyState(0, lazy.mlp_off, 8)
    lazy.lazy = lz2
    lazy.optimizer_step()
    opt = lazy.adam_desc(5)
    opt.beta1 = 0.8
    with pytest.raises(fl.FHashError) as e:
        fl.fhash_step_lazy(opt, lazy.params[: lazy.n_params], lazy.grads[: lazy.n_params],
                           lazy.m[: lazy.n_params], lazy.v[: lazy.n_params], lz2)
    assert e.value.code == fl.EINVAL
    with pytest.raises(fl.FHashError) as e:
        fl.fhash_lazy_prepare(lazy.index, pos, 16, lz2, lazy.params, lazy.grads, lazy.m, lazy.v,
                              phases=4)
    assert e.value.code == fl.EINVAL


def test_split_phases_equal_one_call(fl):
    """Mark and catch-up called separately (as the benchmark times them), once
    with a flush in between, give the same trajectory as the combined prepare."""
    _, _, b = _pair("fp32", 0)
    _, _, c = _pair("fp32", 0)
    g = torch.Generator().manual_seed(9)
    for s in range(6):
        pos = torch.rand(200, 4, generator=g).cuda()
        tgt = torch.rand(200, generator=g).cuda()
        b.fwd_bwd(pos, tgt)  # combined prepare, then the fused backward
        c.prepare(pos, fl.LAZY_MARK)
        if s == 3:
            c.flush()  # between a mark and its catch-up: the flush catches up first
        c.prepare(pos, fl.LAZY_CATCH_UP)
        # the same fresh gradient (no second summation order); c keeps its own
        # pending gradients, which its flush may already have applied
        c.grads.copy_(torch.where(_fresh_mask(b), b.grads, c.grads))
        b.optimizer_step()
        c.optimizer_step()
    b.flush()
    c.flush()
    for name in ("params", "m", "v", "grads"):
        _same(getattr(b, name), getattr(c, name), name)
