"""GPU renderer parity: images against the oracle, ARM-invariance, the step API."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2507_03836_amd import synth

from workloads import coreset_ids, render_bound, tiny_volume

pytestmark = pytest.mark.gpu

TINY_RES = [[4, 4, 4, 2], [8, 8, 8, 3], [16, 16, 16, 5], [32, 32, 32, 8]]


@pytest.fixture(scope="module")
def scene():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    f, mask = tiny_volume()
    T, Sz, Sy, Sx = mask.shape
    dims = [Sx, Sy, Sz, T]
    g = O.Grid(np.array(TINY_RES), 2, mask)
    rng = np.random.default_rng(1)
    table = rng.uniform(-1.0, 1.0, size=(g.total_slots, 2)).astype(np.float32)
    width = [8, 32, 32, 1]
    params = synth.mlp_init(width, seed=7)
    params[-1] = 0.5  # centre the output in the transfer function's range
    bits = torch.from_numpy(synth.pack_mask_rows(mask).view(np.int64)).cuda()
    idx, counts, dir_t, _ = fl.fhash_build_index(fl.grid_desc(TINY_RES, 2), bits, dims)
    return dict(fl=fl, mask=mask, dims=dims, g=g, table=table, width=width, params=params,
                bits=bits, idx=idx, dir=dir_t, tab_d=torch.from_numpy(table).cuda(),
                prm_d=torch.from_numpy(params).cuda(), mlp=fl.mlp_desc(width),
                tf=synth.transfer_function(), tf_d=torch.from_numpy(synth.transfer_function()).cuda())


def _gpu_render(s, view14, t, W, H, arm_max=64, ds=0.5):
    fl = s["fl"]
    rgba = torch.empty(H, W, 4, device="cuda")
    st, _ = fl.fhash_render(s["idx"], s["mlp"], s["tab_d"], s["prm_d"], s["bits"], s["dims"],
                            fl.view_struct(view14), t, s["tf_d"], W, H,
                            fl.render_opts(ds=ds, arm_max=arm_max), rgba)
    return rgba.cpu().numpy(), st


@pytest.mark.parametrize("az,el,t,W,H", [(0.4, 0.3, 3.5, 48, 40), (2.2, -0.5, 0.0, 37, 29),
                                         (4.0, 0.9, 7.0, 64, 16)])
def test_render_matches_oracle(scene, az, el, t, W, H):
    s = scene
    view = synth.orbit_view(s["dims"], az, el, W, H)
    img, st = _gpu_render(s, view, t, W, H)
    ref, amb, ev, pix = O.render(s["g"], s["table"].astype(np.float64), s["width"],
                                 s["params"].astype(np.float64), s["mask"], view, t, s["tf"], W,
                                 H, pixel_stats=True)
    bound, amb = render_bound(pix, s["tf"])
    err = np.abs(img - ref)
    assert (err <= bound).all(), float((err - bound).max())
    assert amb.mean() < 0.5
    assert ref[..., 3].max() > 0.5  # the scene is not empty
    # pace 1 evaluates exactly the composited samples; a larger pace may also
    # decode samples past a ray's termination point in its last batch (discarded)
    img1, st1 = _gpu_render(s, view, t, W, H, arm_max=1)
    np.testing.assert_array_equal(img1, img)
    assert abs(st1.samples - ev) <= 2 * int(amb.sum())
    assert st.samples >= st1.samples


def test_adaptive_pace_does_not_change_the_image(scene):
    s = scene
    view = synth.orbit_view(s["dims"], 1.1, 0.2, 64, 48)
    a, sa = _gpu_render(s, view, 2.25, 64, 48, arm_max=64)
    b, sb = _gpu_render(s, view, 2.25, 64, 48, arm_max=1)
    np.testing.assert_array_equal(a, b)
    assert sa.samples >= sb.samples and sa.iterations < sb.iterations


def test_step_api_equals_whole_render(scene):
    s = scene
    fl = s["fl"]
    W, H = 40, 32
    view = synth.orbit_view(s["dims"], 5.0, 0.1, W, H)
    whole, _ = _gpu_render(s, view, 4.5, W, H)
    ws = torch.empty(fl.fhash_render_state_bytes(W, H, s["dims"]), dtype=torch.uint8,
                     device="cuda")
    rgba = torch.empty(H, W, 4, device="cuda")
    opts = fl.render_opts()
    st = fl.fhash_render_begin(fl.view_struct(view), 4.5, W, H, s["bits"], s["dims"], ws, rgba)
    pos = torch.empty(W * H, 4, device="cuda")
    y = torch.empty(W * H, device="cuda")
    while st.n_alive > 0:
        pace = fl.fhash_render_pace(W * H, st.n_alive, opts.arm_max)
        ns = fl.fhash_render_march(st, opts, pace, pos, W * H)
        if ns:
            fl.fhash_fused_fwd(s["idx"], s["mlp"], pos[:ns], ns, s["tab_d"], s["prm_d"], y)
        fl.fhash_render_composite(st, y, s["tf_d"], opts, rgba)
    np.testing.assert_array_equal(rgba.cpu().numpy(), whole)


def test_render_empty_mask_is_transparent(scene):
    s = scene
    fl = s["fl"]
    empty = torch.zeros_like(s["bits"])
    W, H = 20, 20
    rgba = torch.full((H, W, 4), 5.0, device="cuda")
    view = synth.orbit_view(s["dims"], 0.0, 0.0, W, H)
    st, _ = fl.fhash_render(s["idx"], s["mlp"], s["tab_d"], s["prm_d"], empty, s["dims"],
                            fl.view_struct(view), 1.0, s["tf_d"], W, H, fl.render_opts(), rgba)
    assert (rgba == 0).all() and st.samples == 0


def test_more_rays_than_one_grid_of_65536_blocks(scene):
    """4200 x 4100 = 17.2e6 rays, more than 65536 blocks of 256 threads: with
    a fully occupied volume, a decoder whose output is the constant 0.6 (TF
    opacity 0.21) and a narrow field of view through the volume's centre,
    every pixel must composite."""
    s = scene
    fl = s["fl"]
    full = torch.from_numpy(
        synth.pack_mask_rows(np.ones_like(s["mask"])).view(np.int64)).cuda()
    params = np.zeros_like(s["params"])
    params[-1] = 0.6
    W, H = 4200, 4100
    view = synth.orbit_view(s["dims"], 0.7, 0.3, W, H, fovy_deg=4.0)
    rgba = torch.empty(H, W, 4, device="cuda")
    st, ws = fl.fhash_render(s["idx"], s["mlp"], s["tab_d"], torch.from_numpy(params).cuda(),
                             full, s["dims"], fl.view_struct(view), 2.5, s["tf_d"], W, H,
                             fl.render_opts(), rgba)
    del ws
    a = rgba[..., 3]
    assert bool((a >= 0.99).all()), int((a < 0.99).sum())
    assert st.samples >= W * H


def test_batched_steps_equal_single_renders(scene):
    """fhash_render_march_batch / fhash_render_composite_batch over several
    requests (uneven sizes, times and paces, samples interleaved in one
    buffer at a non-zero base) give every request the image, sample count
    and iteration count of its own fhash_render, bit for bit."""
    s = scene
    fl = s["fl"]
    opts = fl.render_opts()
    cases = [(40, 32, 4.5, 5.0), (17, 23, 0.0, 1.3), (64, 48, 6.75, 2.6), (8, 8, 2.0, 0.2),
             (33, 1, 7.0, 3.9), (3, 2, 1.5, 4.4)]
    reqs = []
    for W, H, t, az in cases:
        view = synth.orbit_view(s["dims"], az, 0.25, W, H)
        whole, stats = _gpu_render(s, view, t, W, H)
        ws = torch.empty(fl.fhash_render_state_bytes(W, H, s["dims"]), dtype=torch.uint8,
                         device="cuda")
        rgba = torch.empty(H, W, 4, device="cuda")
        st = fl.fhash_render_begin(fl.view_struct(view), t, W, H, s["bits"], s["dims"], ws, rgba)
        reqs.append(dict(W=W, H=H, whole=whole, stats=stats, ws=ws, rgba=rgba, st=st))
    base = 7
    cap = base + sum(r["W"] * r["H"] for r in reqs) * opts.arm_max
    pos = torch.empty(cap, 4, device="cuda")
    y = torch.full((cap,), float("nan"), device="cuda")
    counts = torch.empty(1 + fl.RENDER_BATCH_MAX, dtype=torch.int32, device="cuda")
    launches = 0
    while True:
        act = [r for r in reqs if r["st"].n_alive > 0]
        if not act:
            break
        paces = [fl.fhash_render_pace(r["W"] * r["H"], r["st"].n_alive, opts.arm_max)
                 for r in act]
        ns = fl.fhash_render_march_batch([r["st"] for r in act], paces, opts, pos, base, cap,
                                         counts)
        total = sum(ns)
        if total:
            fl.fhash_fused_fwd(s["idx"], s["mlp"], pos[base: base + total], total, s["tab_d"],
                               s["prm_d"], y[base: base + total])
        alive = fl.fhash_render_composite_batch([r["st"] for r in act], y, [s["tf_d"]] * len(act),
                                                opts, [r["rgba"] for r in act], counts)
        assert alive == [r["st"].n_alive for r in act]
        launches += 1
    assert launches == max(r["stats"].iterations for r in reqs)
    for r in reqs:
        np.testing.assert_array_equal(r["rgba"].cpu().numpy(), r["whole"])
        assert r["st"].samples == r["stats"].samples
        assert r["st"].iterations == r["stats"].iterations


def test_render_from_occupancy_grid_equals_mask_rows(scene):
    """A render that starts from the coreset's occupancy grid
    (fhash_render_begin_grid) is the render from the mask rows, bit for bit,
    at key and in-between times, on a volume whose x extent is not a multiple
    of the brick or word width."""
    s = scene
    fl = s["fl"]
    opts = fl.render_opts()
    rng = np.random.default_rng(8)
    for dims, mask, bits in [(s["dims"], s["mask"], s["bits"])] + [
            _random_mask(rng, (3, 13, 21, 150)), _random_mask(rng, (2, 6, 5, 67))]:
        occ = fl.fhash_occupancy_grid(bits, dims)
        for az, t in ((0.3, 0.0), (2.0, 0.5 * (dims[3] - 1)), (4.1, float(dims[3] - 1) - 0.25)):
            W, H = 29, 21
            view = fl.view_struct(synth.orbit_view(dims, az, 0.3, W, H))
            imgs, stats = [], []
            for grid in (False, True):
                ws = torch.empty(fl.fhash_render_state_bytes(W, H, dims), dtype=torch.uint8,
                                 device="cuda")
                rgba = torch.empty(H, W, 4, device="cuda")
                begin = fl.fhash_render_begin_grid if grid else fl.fhash_render_begin
                st = begin(view, t, W, H, occ if grid else bits, dims, ws, rgba)
                pos = torch.empty(W * H * 64, 4, device="cuda")
                y = torch.empty(W * H * 64, device="cuda")
                while st.n_alive > 0:
                    pace = fl.fhash_render_pace(W * H, st.n_alive, opts.arm_max)
                    ns = fl.fhash_render_march(st, opts, pace, pos, W * H * 64)
                    if ns:
                        # a decoder stand-in that depends on the sample: the
                        # position's coordinates (any difference in the samples
                        # taken shows up in the image)
                        y[:ns] = pos[:ns, :3].sum(1) / 3.0
                    fl.fhash_render_composite(st, y, s["tf_d"], opts, rgba)
                imgs.append(rgba.cpu().numpy())
                stats.append((st.samples, st.iterations))
            np.testing.assert_array_equal(imgs[0], imgs[1])
            assert stats[0] == stats[1]


def _random_mask(rng, shape):
    from paper_2507_03836_amd import synth as S
    T, Sz, Sy, Sx = shape
    m = (rng.random(shape) < 0.15).astype(np.uint8)
    bits = torch.from_numpy(S.pack_mask_rows(m).view(np.int64)).cuda()
    return [Sx, Sy, Sz, T], m, bits
