"""The 16-bit MFMA training decoder (FP16 or BF16 operands, FP32 accumulation)
against the FP64 oracle.

Every weight, hidden-layer input and backward delta is rounded to the 16-bit
type (unit roundoff u = 2^-11 for FP16, 2^-8 for BF16) before an MFMA; biases,
the output layer and all sums stay FP32.  The bounds below are built layer by
layer from those roundings (first order plus the u^2 terms, magnitudes from the
weights and the oracle's activations), plus the 1e-5 * magnitude allowance of
the FP32 path for the FP32 arithmetic.  A ReLU whose pre-activation lies within
its forward error bound of zero may switch either way: in the forward that is
covered by the ReLU being 1-Lipschitz, in the backward the delta of such a unit
is bounded by its whole magnitude (plus its propagated error).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import tiny_volume

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-12
U = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
TINY_SUB = 2.0 ** -24  # absolute rounding below the FP16 normal range (BF16 has none there)


def _wide_res(L, rmax=(70, 24, 20, 8)):
    return [[max(2, int(np.floor(2.0 * (r / 2.0) ** (l / (L - 1)) + 0.5))) for r in rmax]
            for l in range(L)]


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


def _unpack(width, params):
    Ws, bs, off = [], [], 0
    for k in range(len(width) - 1):
        W = params[off: off + width[k + 1] * width[k]].astype(np.float64).reshape(width[k + 1],
                                                                                 width[k])
        off += width[k + 1] * width[k]
        Ws.append(W)
        bs.append(params[off: off + width[k + 1]].astype(np.float64))
        off += width[k + 1]
    return Ws, bs


def _analysis(width, params, x, x_err, dy, u):
    """Test-side FP64 forward/backward with error bounds of the 16-bit decoder.

    Returns (bound of y, bound of each parameter's gradient in the packed
    layout, bound of dx, fraction of hidden units whose ReLU may switch)."""
    Ws, bs = _unpack(width, params)
    NH = len(width) - 2
    tiny = TINY_SUB if u == U["f16"] else 0.0
    h, e, zs, amb = [x], [x_err], [], []
    for k in range(NH):
        aW = np.abs(Ws[k])
        z = h[k] @ Ws[k].T + bs[k]
        m_in = np.abs(h[k]) + e[k]
        err = (e[k] * (1 + 2 * u) + (2 * u + u * u) * m_in + tiny) @ aW.T + \
            tiny * m_in.sum(axis=1, keepdims=True) + RTOL * (m_in @ aW.T + np.abs(bs[k])) + ATOL
        zs.append(z)
        amb.append(np.abs(z) <= err)
        h.append(np.maximum(z, 0.0))
        e.append(err)  # relu is 1-Lipschitz
    wout, bout = Ws[NH][0], bs[NH]
    y_err = e[NH] @ np.abs(wout) + RTOL * (np.abs(h[NH]) @ np.abs(wout) + abs(bout[0])) + ATOL
    dyc = dy.reshape(-1, 1)
    grads = [None] * (2 * (NH + 1))
    v = wout[None, :] * dyc                     # gradient at h_NH (pre-mask)
    delta = (zs[NH - 1] > 0) * v
    E = np.where(amb[NH - 1], np.abs(v), 0.0) + RTOL * np.abs(v)
    grads[2 * NH] = (np.abs(dyc) * e[NH]).sum(0) + RTOL * (np.abs(dyc) * np.abs(h[NH])).sum(0)
    grads[2 * NH + 1] = np.array([RTOL * np.abs(dy).sum() + ATOL])
    for k in range(NH - 1, -1, -1):
        ad, ah = np.abs(delta), np.abs(h[k])
        grads[2 * k + 1] = E.sum(0) + RTOL * ad.sum(0)
        gW = ((ad + E) * (1 + u)).T @ ((ah + e[k]) * (2 * u + u * u)) + E.T @ ah + ad.T @ e[k] \
            + E.T @ e[k] + RTOL * (ad.T @ ah)
        grads[2 * k] = gW.ravel()
        aW = np.abs(Ws[k])
        prop = (E + (2 * u + u * u) * (ad + E) + tiny) @ aW + RTOL * (ad @ aW)
        v = delta @ Ws[k]                       # gradient at h_k (pre-mask)
        if k > 0:
            act = zs[k - 1] > 0
            delta = act * v
            E = np.where(amb[k - 1], np.abs(v) + prop, act * prop)
        else:
            dx_err = prop
    frac = float(np.mean([a.mean() for a in amb]))
    return y_err, np.concatenate(grads), dx_err, frac


CASES = [("bf16", [32, 64, 64, 1]), ("bf16", [32, 64, 64, 64, 1]),
         ("f16", [32, 64, 64, 1]), ("f16", [32, 64, 64, 64, 1]), ("bf16", [32, 32, 32, 32, 1])]


@pytest.mark.parametrize("dt,width", CASES, ids=[f"{c[0]}-{len(c[1]) - 2}x{c[1][1]}" for c in CASES])
def test_decoder16_train_within_rounding_bounds(fl, dt, width):
    f, mask = tiny_volume()
    T, Sz, Sy, Sx = mask.shape
    res = _wide_res(16)
    g = O.Grid(np.array(res), 2, mask)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    idx, counts, _dir, _ = fl.fhash_build_index(fl.grid_desc(res, 2), bits, [Sx, Sy, Sz, T])
    rng = np.random.default_rng(7 + len(width))
    table = rng.uniform(-1, 1, (g.total_slots, 2)).astype(np.float32)
    params = synth.mlp_init(width, seed=11)
    u = U[dt]
    n = 3000
    pos = synth.probe_points(n, 91).astype(np.float32)
    enc, emag = O.encode_fwd(g, pos, table.astype(np.float64))
    dy = rng.normal(size=n).astype(np.float32)
    y_err, g_err, dx_err, frac = _analysis(width, params, enc, RTOL * emag + ATOL,
                                           dy.astype(np.float64), u)
    y_ref, acts, _ = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
    dp_ref, dx_ref, _, _ = O.mlp_bwd(width, params.astype(np.float64), acts,
                                     dy.astype(np.float64).reshape(-1, 1), n, x_mag=emag)
    dt_ref, _ = O.encode_bwd(g, pos, dx_ref)
    dt_err, _ = O.encode_bwd(g, pos, dx_err)
    _, dt_mag = O.encode_bwd(g, pos, np.abs(dx_ref) + dx_err)
    mlp = fl.mlp_desc(width, fl.BF16 if dt == "bf16" else fl.F16)
    pos_d, tab_d = torch.from_numpy(pos).cuda(), torch.from_numpy(table).cuda()
    prm = torch.from_numpy(params).cuda()
    y = torch.empty(n, device="cuda")
    fl.fhash_fused_fwd(idx, mlp, pos_d, n, tab_d, prm, y)
    err = np.abs(y.cpu().numpy() - y_ref[:, 0])
    assert (err <= y_err).all(), float((err - y_err).max())
    d_tab = torch.zeros(g.total_slots, 2, device="cuda")
    d_par = torch.zeros(len(params), device="cuda")
    fl.fhash_fused_bwd(idx, mlp, pos_d, n, tab_d, prm, torch.from_numpy(dy).cuda(), d_tab, d_par)
    gp = d_par.cpu().numpy().astype(np.float64)
    bad = np.abs(gp - dp_ref) > g_err + ATOL
    assert not bad.any(), (int(bad.sum()), float((np.abs(gp - dp_ref) - g_err).max()))
    gt = d_tab.cpu().numpy().astype(np.float64)
    tol = dt_err + RTOL * dt_mag + ATOL
    assert (np.abs(gt - dt_ref) <= tol).all(), float((np.abs(gt - dt_ref) - tol).max())
    # the rounding is real: the 16-bit result differs from the FP32 decoder's
    y32 = torch.empty(n, device="cuda")
    fl.fhash_fused_fwd(idx, fl.mlp_desc(width), pos_d, n, tab_d, prm, y32)
    assert not torch.equal(y, y32)
    rel = np.abs(gp - dp_ref).max() / np.abs(dp_ref).max()
    print(f"\n{dt} {width}: {frac:.4f} of hidden units may switch; max |y err| {err.max():.2e}, "
          f"d_params max err {rel:.2e} of max |grad|, bound median "
          f"{np.median(g_err / (np.abs(dp_ref) + 1e-30)):.2e} relative")


def test_decoder16_rejects_unbuilt_shapes(fl):
    """16-bit backward is built for two features per level only."""
    res = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]
    idx, _, _d, _ = fl.fhash_build_index(fl.grid_desc(res, 4), None, [2, 2, 2, 2])
    mlp = fl.mlp_desc([16, 32, 32, 1], fl.BF16)
    prm = torch.zeros(fl.fhash_mlp_num_params(mlp), device="cuda")
    pos = torch.rand(16, 4, device="cuda")
    rows = int(idx.slot_offset[4])
    with pytest.raises(fl.FHashError) as e:
        fl.fhash_fused_bwd(idx, mlp, pos, 16, torch.zeros(rows, 4, device="cuda"), prm,
                           torch.zeros(16, device="cuda"), torch.zeros(rows, 4, device="cuda"),
                           torch.zeros_like(prm))
    assert e.value.code == fl.ENOTSUP


@pytest.mark.parametrize("decoder", ["bf16", "f16"])
def test_mixed_training_with_16bit_decoder_learns_like_fp32(fl, decoder):
    """Mixed precision (FP16 table reads, 16-bit decoder, loss scaling) and the
    FP32 path trained on the same 150 batches of the tiny workload reach the
    same probe PSNR within 0.5 dB, well above the untrained model's."""
    from paper_2507_03836_amd.model import FHashConfig, FHashModel, psnr_on
    from workloads import coreset_ids
    f, mask = tiny_volume()
    T, Sz, Sy, Sx = mask.shape
    dims = [Sx, Sy, Sz, T]
    cfg = FHashConfig(res=_wide_res(16, (32, 32, 32, 8)), n_features=2, hidden=64, n_hidden=3)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    cs = torch.from_numpy(coreset_ids(mask).view(np.int64)).cuda()
    fd = torch.from_numpy(f).cuda()
    probe_p = torch.empty(1 << 14, 4, device="cuda")
    probe_t = torch.empty(1 << 14, device="cuda")
    fl.fhash_sample(4001, 1, 1 << 14, cs, cs.numel(), dims, fd, probe_p, probe_t)
    out = {}
    for name, kw in (("fp32", {}), ("mixed", {"precision": "mixed", "decoder": decoder})):
        model = FHashModel(cfg, bits, dims, init_seed=3001, **kw)
        before = psnr_on(model, probe_p, probe_t)
        pos = torch.empty(4096, 4, device="cuda")
        tgt = torch.empty(4096, device="cuda")
        for k in range(150):
            fl.fhash_sample(2001, k + 1, 4096, cs, cs.numel(), dims, fd, pos, tgt)
            model.train_step(pos, tgt)
        out[name] = (before, psnr_on(model, probe_p, probe_t), model)
    print(f"\n{decoder}: fp32 {out['fp32'][:2]}, mixed {out['mixed'][:2]}")
    assert out["fp32"][1] > out["fp32"][0] + 10
    assert abs(out["mixed"][1] - out["fp32"][1]) < 0.5
    assert out["mixed"][2].skipped == 0
