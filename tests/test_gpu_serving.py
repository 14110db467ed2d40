"""Continuous-batching server on the device: every result of a mixed stream
(three resident models: FP32, FP16 tables, FP16 tables with the FP16 decoder;
two of them rendering from the coreset's occupancy grid; renders of uneven
sizes and times; point-query batches; batched march and composite launches)
equals, bit for bit, the same request served alone through the plain entry
points (fhash_render from the mask rows, fhash_fused_fwd)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import coreset_ids, render_bound, tiny_volume

pytestmark = pytest.mark.gpu

TINY_RES = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]


@pytest.fixture(scope="module")
def server_models():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd.serving import GpuExecutor, ResidentModel
    fl.lib()
    f, mask = tiny_volume()
    T, Sz, Sy, Sx = mask.shape
    dims = [Sx, Sy, Sz, T]
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    idx, counts, dir_t, _ = fl.fhash_build_index(fl.grid_desc(TINY_RES, 2), bits, dims)
    rows = int(idx.slot_offset[len(TINY_RES)])
    width = [8, 32, 32, 1]
    tf = torch.from_numpy(synth.transfer_function()).cuda()
    models = {}
    for k, (seed, dt, mdt) in enumerate([(11, torch.float32, fl.F32),
                                         (12, torch.float16, fl.F32),
                                         (13, torch.float16, fl.F16)]):
        rng = np.random.default_rng(seed)
        table = torch.from_numpy(rng.uniform(-1, 1, (rows, 2)).astype(np.float32)).cuda()
        params = synth.mlp_init(width, seed=seed)
        params[-1] = 0.5
        # m1 and m2 render from the coreset's occupancy grid, m0 from the mask rows
        occ = fl.fhash_occupancy_grid(bits, dims) if k else None
        models[f"m{k}"] = ResidentModel(index=idx, mlp=fl.mlp_desc(width, mdt),
                                        table=table.to(dt),
                                        params=torch.from_numpy(params).cuda(), mask_bits=bits,
                                        dims=dims, tf=tf, keep=(dir_t,), occ=occ)
    return fl, models, dims


def _requests(dims, rng):
    from paper_2507_03836_amd.serving import Request
    reqs = []
    sizes = [(40, 32), (17, 23), (64, 48), (8, 8), (33, 1)]
    for j in range(14):
        m = f"m{j % 3}"
        if j % 3 != 2:
            W, H = sizes[j % len(sizes)]
            view = synth.orbit_view(dims, rng.uniform(0, 2 * np.pi), rng.uniform(-1, 1), W, H)
            t = float(rng.uniform(0, dims[3] - 1)) if j != 4 else 0.0
            reqs.append(Request(model=m, kind="render", view=view, t=t, W=W, H=H,
                                arrival=j * 2e-4))
        else:
            n = [1, 1000, 4097, 0][j % 4]
            pos = torch.from_numpy(rng.uniform(0, 1, (n, 4)).astype(np.float32)).cuda()
            reqs.append(Request(model=m, kind="points", pos=pos, n=n, arrival=j * 2e-4))
    return reqs


@pytest.mark.parametrize("budget,max_active,policy", [(1 << 14, 64, "oldest_first"),
                                                      (7000, 2, "shared"),
                                                      (1 << 13, 64, "backfill")])
def test_mixed_stream_equals_alone(server_models, budget, max_active, policy):
    fl, models, dims = server_models
    from paper_2507_03836_amd.serving import GpuExecutor, Scheduler
    ex = GpuExecutor(sample_budget=budget)
    for k, m in models.items():
        ex.add_model(k, m)
    sch = Scheduler(ex, sample_budget=budget, mem_budget=1 << 30, max_active=max_active,
                    policy=policy)
    reqs = _requests(dims, np.random.default_rng(budget))
    done = sch.run(reqs, realtime=True)
    assert len(done) == len(reqs)
    assert sch.peak_active <= max_active
    opts = fl.render_opts()
    for r in reqs:
        m = models[r.model]
        if r.kind == "render":
            alone = torch.empty(r.H, r.W, 4, device="cuda")
            fl.fhash_render(m.index, m.mlp, m.table, m.params, m.mask_bits, dims,
                            fl.view_struct(r.view), r.t, m.tf, r.W, r.H, opts, alone)
            assert torch.equal(alone, r.result), (r.rid, r.W, r.H, r.t)
        else:
            alone = torch.empty(r.n, device="cuda")
            if r.n:
                fl.fhash_fused_fwd(m.index, m.mlp, r.pos, r.n, m.table, m.params, alone)
            assert torch.equal(alone, r.result), (r.rid, r.n)
    assert any(float(r.result[..., 3].max()) > 0.3 for r in reqs if r.kind == "render")


def test_served_render_matches_oracle(server_models):
    """One served render of the FP32 model against the oracle's renderer."""
    fl, models, dims = server_models
    from paper_2507_03836_amd.serving import GpuExecutor, Request, Scheduler
    m = models["m0"]
    ex = GpuExecutor(sample_budget=1 << 13)
    ex.add_model("m0", m)
    sch = Scheduler(ex, sample_budget=1 << 13)
    W, H, t = 36, 28, 2.75
    view = synth.orbit_view(dims, 0.9, 0.35, W, H)
    r = Request(model="m0", kind="render", view=view, t=t, W=W, H=H)
    sch.run([r], realtime=False)
    f, mask = tiny_volume()
    g = O.Grid(np.array(TINY_RES), 2, mask)
    tf = synth.transfer_function()
    ref, amb, _, pix = O.render(g, m.table.cpu().numpy().astype(np.float64), [8, 32, 32, 1],
                                m.params.cpu().numpy().astype(np.float64), mask, view, t, tf, W,
                                H, pixel_stats=True)
    bound, amb = render_bound(pix, tf)
    err = np.abs(r.result.cpu().numpy() - ref)
    assert (err <= bound).all(), float((err - bound).max())
