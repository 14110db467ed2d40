"""fhash_fused_train_static (no workspace, library-owned scratch) against
fhash_fused_train (caller workspace) through the C ABI: two calls in a row,
the second with a smaller batch, each within the FP32 tolerance of the other
(|a - b| <= 2e-5 * mag + 1e-12, mag = the oracle's term magnitudes: both
results lie within 1e-5 * mag of the FP64 value), and both against the
oracle."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import tiny_volume

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-12


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


def _static_call(fl, idx, mlp, pos, tgt, n, table, params, d_table, d_params, loss):
    L = fl.lib()
    fn = L.fhash_fused_train_static
    P = C.c_void_p
    fn.restype = C.c_int
    fn.argtypes = [P, P, P, P, C.c_int64, P, C.c_int, P, P, C.c_float, P, P, P, C.c_uint32, P, P]
    rc = fn(C.byref(idx), C.byref(mlp), C.c_void_p(pos.data_ptr()), C.c_void_p(tgt.data_ptr()),
            n, C.c_void_p(table.data_ptr()), fl.F32, C.c_void_p(params.data_ptr()), None, 1.0,
            C.c_void_p(d_table.data_ptr()), C.c_void_p(d_params.data_ptr()),
            C.c_void_p(loss.data_ptr()), 0, None,
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.fhash_last_error()


@pytest.mark.parametrize("hidden", [[64, 64, 64], [32, 32]])
def test_static_scratch_equals_workspace_call(fl, hidden):
    f, mask = tiny_volume()
    T, Sz, Sy, Sx = mask.shape
    res = _wide_res(16)
    g = O.Grid(np.array(res), 2, mask)
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    idx, counts, _dir, _ = fl.fhash_build_index(fl.grid_desc(res, 2), bits, [Sx, Sy, Sz, T])
    width = [32] + hidden + [1]
    rng = np.random.default_rng(5)
    table = rng.uniform(-1, 1, (g.total_slots, 2)).astype(np.float32)
    params = synth.mlp_init(width, seed=6)
    mlp = fl.mlp_desc(width)
    tab_d, prm_d = torch.from_numpy(table).cuda(), torch.from_numpy(params).cuda()
    for n in (4096 + 7, 999):  # two calls in a row, the second smaller
        print(f"[no-alloc] hidden {hidden}, n = {n}", flush=True)
        pos = synth.probe_points(n, 100 + n).astype(np.float32)
        tgt = rng.random(n).astype(np.float32)
        pos_d, tgt_d = torch.from_numpy(pos).cuda(), torch.from_numpy(tgt).cuda()
        out = []
        for kind in ("workspace", "static"):
            dt = torch.zeros(g.total_slots, 2, device="cuda")
            dp = torch.zeros(len(params), device="cuda")
            loss = torch.zeros(1, dtype=torch.float64, device="cuda")
            if kind == "workspace":
                fl.fhash_fused_train(idx, mlp, pos_d, tgt_d, n, tab_d, prm_d, dt, dp, loss)
            else:
                _static_call(fl, idx, mlp, pos_d, tgt_d, n, tab_d, prm_d, dt, dp, loss)
            torch.cuda.synchronize()
            out.append((dt.cpu().numpy().astype(np.float64), dp.cpu().numpy().astype(np.float64),
                        loss.item()))
        enc, emag = O.encode_fwd(g, pos, table.astype(np.float64))
        y, acts, ymag = O.mlp_fwd(width, params.astype(np.float64), enc, x_mag=emag)
        Lr, dy = O.mse(y[:, 0], tgt.astype(np.float64))
        dym = 2.0 * (ymag[:, 0] + np.abs(tgt)) / n
        dp_ref, denc, dpm, dencm = O.mlp_bwd(width, params.astype(np.float64), acts,
                                             dy.reshape(-1, 1), n, dy_mag=dym.reshape(-1, 1),
                                             x_mag=emag)
        dt_ref, _ = O.encode_bwd(g, pos, denc)
        _, dtm = O.encode_bwd(g, pos, dencm)
        (dt_w, dp_w, l_w), (dt_s, dp_s, l_s) = out
        assert (np.abs(dt_s - dt_w) <= 2 * RTOL * dtm + ATOL).all()
        assert (np.abs(dp_s - dp_w) <= 2 * RTOL * dpm + ATOL).all()
        for dt_x, dp_x in ((dt_w, dp_w), (dt_s, dp_s)):
            assert (np.abs(dt_x - dt_ref) <= RTOL * dtm + ATOL).all()
            assert (np.abs(dp_x - dp_ref) <= RTOL * dpm + ATOL).all()
        assert abs(l_s - l_w) <= 1e-9 * abs(l_w)
        assert np.abs(dp_s).sum() > 0
