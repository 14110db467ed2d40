"""GPU parity of the coreset-selection calls (Sec. 3.1) against the numpy
oracle: every output is integer or bit work, so every comparison is exact,
padding bits included.  Shapes span several 64-voxel words with a ragged
last word, bricks that overhang the volume, empty frames and empty masks."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import coreset as OC
from paper_2507_03836_amd import synth

from workloads import coreset_ids, tiny_volume

SHAPES = [(70, 5, 3, 2), (130, 9, 4, 3), (64, 4, 4, 2), (65, 3, 2, 2), (2, 2, 2, 2)]
# rows of a multiple of 4 voxels take the float4 extraction pass: a partial
# 256-voxel segment (300: words 4..7 of the second segment, only word 4 real),
# whole segments (256, 512) and more words than one segment (1028)
SHAPES4 = [(300, 7, 5, 3), (256, 3, 2, 2), (512, 2, 3, 2), (1028, 3, 2, 2), (4, 3, 3, 2)]


def _fl():
    from paper_2507_03836_amd import _lib as fl
    fl.lib()
    return fl


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return _fl()


def _np_field(dims, seed):
    Sx, Sy, Sz, T = dims
    return np.random.default_rng(seed).random((T, Sz, Sy, Sx), dtype=np.float32)


def _words(t):
    return t.cpu().numpy().view(np.uint64)


def _mask_dev(mask):
    return torch.from_numpy(OC.pack_rows(mask).view(np.int64).ravel().copy()).cuda()


@pytest.mark.gpu
@pytest.mark.parametrize("dims", SHAPES + SHAPES4)
def test_feature_interval_parity(fl, dims):
    print(f"[coreset] interval {dims}", flush=True)
    f = _np_field(dims, 1)
    f.ravel()[::7] = 0.25  # values on the lower bound stay out, on the upper bound stay in
    f.ravel()[3::11] = 0.75
    bits = fl.fhash_feature_mask(torch.from_numpy(f).cuda(), dims, fl.FEATURE_INTERVAL, 0.25, 0.75)
    torch.cuda.synchronize()
    want = OC.pack_rows(OC.feature_interval(f, 0.25, 0.75)).ravel()
    assert np.array_equal(_words(bits), want)


@pytest.mark.gpu
@pytest.mark.parametrize("dims", SHAPES + SHAPES4)
def test_feature_isosurface_parity(fl, dims):
    print(f"[coreset] isosurface {dims}", flush=True)
    f = _np_field(dims, 2)
    f.ravel()[::5] = 0.5  # corners exactly on the level count as above it
    bits = fl.fhash_feature_mask(torch.from_numpy(f).cuda(), dims, fl.FEATURE_ISOSURFACE, 0.5)
    torch.cuda.synchronize()
    want = OC.pack_rows(OC.feature_isosurface(f, 0.5)).ravel()
    assert np.array_equal(_words(bits), want)


@pytest.mark.gpu
@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("r", [0, 1, 2, 5, 63])
def test_dilate_parity(fl, dims, r):
    print(f"[coreset] dilate {dims} r={r}", flush=True)
    Sx, Sy, Sz, T = dims
    m = np.random.default_rng(3 + r).random((T, Sz, Sy, Sx)) < 0.02
    m[0, 0, 0, Sx - 1] = True  # a voxel at the row end: padding must stay clear
    out = fl.fhash_dilate_mask(_mask_dev(m), dims, r)
    torch.cuda.synchronize()
    assert np.array_equal(_words(out), OC.pack_rows(OC.dilate(m, r)).ravel())


@pytest.mark.gpu
@pytest.mark.parametrize("r", [1, 2])
def test_dilate_parity_large_slice(fl, r):
    """A (t, z) slice of 130 rows x 64 words (8,320 words, above the 8,192 that
    the LDS form holds) takes the direct form; 128 rows x 64 words the LDS form."""
    for dims in [(4096, 130, 3, 2), (4096, 128, 3, 2)]:
        print(f"[coreset] dilate {dims} r={r}", flush=True)
        Sx, Sy, Sz, T = dims
        m = np.random.default_rng(30 + r).random((T, Sz, Sy, Sx)) < 0.001
        out = fl.fhash_dilate_mask(_mask_dev(m), dims, r)
        torch.cuda.synchronize()
        assert np.array_equal(_words(out), OC.pack_rows(OC.dilate(m, r)).ravel())


@pytest.mark.gpu
@pytest.mark.parametrize("dims", SHAPES + [(300, 17, 9, 5)])
def test_boxes_parity(fl, dims):
    print(f"[coreset] boxes {dims}", flush=True)
    Sx, Sy, Sz, T = dims
    m = np.random.default_rng(4).random((T, Sz, Sy, Sx)) < 0.003
    m[-1] = False  # an empty frame
    if T > 2:
        m[1, Sz - 1, Sy - 1, Sx - 1] = True  # far corner
    box = fl.fhash_feature_boxes(_mask_dev(m), dims)
    torch.cuda.synchronize()
    assert np.array_equal(box.cpu().numpy().astype(np.int64), OC.feature_boxes(m))
    empty = fl.fhash_feature_boxes(_mask_dev(np.zeros_like(m)), dims)
    torch.cuda.synchronize()
    assert np.array_equal(empty.cpu().numpy().astype(np.int64),
                          OC.feature_boxes(np.zeros_like(m)))


@pytest.mark.gpu
@pytest.mark.parametrize("dims", SHAPES + [(131, 10, 7, 3)])
def test_occupancy_parity(fl, dims):
    print(f"[coreset] occupancy {dims}", flush=True)
    Sx, Sy, Sz, T = dims
    m = np.random.default_rng(6).random((T, Sz, Sy, Sx)) < 0.3
    occ = fl.fhash_occupancy_grid(_mask_dev(m), dims)
    torch.cuda.synchronize()
    assert np.array_equal(_words(occ), OC.occupancy_grid(m).ravel())


@pytest.mark.gpu
@pytest.mark.parametrize("dims", SHAPES + [(700, 40, 30, 3)])
def test_coreset_parity(fl, dims):
    """(700, 40, 30, 3): 39,600 mask words, ten chunks of the count/emit pass."""
    print(f"[coreset] ids {dims}", flush=True)
    Sx, Sy, Sz, T = dims
    m = np.random.default_rng(8).random((T, Sz, Sy, Sx)) < 0.1
    ids = fl.fhash_coreset(_mask_dev(m), dims)
    assert np.array_equal(_words(ids), OC.coreset_ids(m))
    none = fl.fhash_coreset(_mask_dev(np.zeros_like(m)), dims)
    assert none.numel() == 0


@pytest.mark.gpu
def test_pipeline_reproduces_the_tiny_workload(fl):
    """Feature value > 0.1 dilated by one voxel: the tiny workload's mask and
    coreset, from the product calls alone."""
    print("[coreset] tiny pipeline", flush=True)
    f, mask = tiny_volume()
    dims = (f.shape[3], f.shape[2], f.shape[1], f.shape[0])
    feat = fl.fhash_feature_mask(torch.from_numpy(f).cuda(), dims, fl.FEATURE_INTERVAL, 0.1,
                                 float("inf"))
    d = fl.fhash_dilate_mask(feat, dims, 1)
    ids = fl.fhash_coreset(d, dims)
    assert np.array_equal(_words(d), OC.pack_rows(mask.astype(bool)).ravel())
    assert np.array_equal(_words(ids), OC.coreset_ids(mask))
    box = fl.fhash_feature_boxes(d, dims)
    torch.cuda.synchronize()
    assert np.array_equal(box.cpu().numpy().astype(np.int64), OC.feature_boxes(mask))


@pytest.mark.gpu
def test_pipeline_at_production_shape(fl):
    """480 x 720 x 120 spatial, 4 timesteps (166 M voxels): gradient magnitude
    above its 80th percentile, dilated by 2, through the product calls
    (paper_2507_03836_amd.volume), against oracle/coreset.py on the same
    attribute field: mask, coreset ids, frame boxes + FBB and occupancy grid
    bit for bit."""
    import time
    from paper_2507_03836_amd import volume
    dims = (480, 720, 120, 4)
    print(f"[coreset] production pipeline {dims}", flush=True)
    gen = synth.production_field_gpu(dims, seed=5, keep_field=False)
    attr, thr = gen.pop("grad"), gen["threshold"]
    sel = volume.select_coreset(attr, dims, thr, radius=synth.PRODUCTION_DILATION)
    d = sel["bits"].reshape(-1)
    occ = fl.fhash_occupancy_grid(d, dims)
    box = fl.fhash_feature_boxes(d, dims)
    torch.cuda.synchronize()
    t0 = time.time()
    g = attr.cpu().numpy()
    del attr
    m = OC.dilate(OC.feature_interval(g, thr, np.inf), synth.PRODUCTION_DILATION)
    print(f"[coreset] oracle mask in {time.time() - t0:.1f} s", flush=True)
    assert np.array_equal(_words(d), OC.pack_rows(m).ravel())
    assert np.array_equal(_words(sel["coreset"]), OC.coreset_ids(m))
    assert np.array_equal(box.cpu().numpy().astype(np.int64), OC.feature_boxes(m))
    assert np.array_equal(_words(occ), OC.occupancy_grid(m).ravel())


def test_coreset_calls_reject_bad_arguments():
    """Host-side validation returns before any launch (no device needed)."""
    fl = _fl()
    L = fl.lib()
    dims = (C.c_int64 * 4)(70, 5, 3, 2)
    fake = C.c_void_p(1 << 20)
    assert L.fhash_dilate_mask(fake, dims, 64, C.c_void_p(1 << 30), None) == fl.EINVAL
    assert L.fhash_dilate_mask(fake, dims, -1, C.c_void_p(1 << 30), None) == fl.EINVAL
    assert L.fhash_dilate_mask(fake, dims, 1, fake, None) == fl.EINVAL  # in place
    big_t = (C.c_int64 * 4)(70, 5, 3, 65536)
    assert L.fhash_feature_boxes(fake, big_t, fake, None) == fl.EINVAL
    assert L.fhash_occupancy_words(big_t) == -1
    assert L.fhash_occupancy_words(dims) == 2 * 1 * 2 * 18
    assert L.fhash_feature_mask(fake, dims, 7, 0.0, 1.0, fake, None, None, None) == fl.EINVAL
    nb = C.c_size_t(0)
    assert L.fhash_feature_mask(None, dims, 1, 0.5, 0.0, None, None, C.byref(nb), None) == fl.OK
    assert nb.value == 2 * 3 * 5 * 2 * 8
    cnt = C.c_int64(0)
    assert L.fhash_coreset(fake, dims, None, 0, None, C.byref(nb), C.byref(cnt), None) == fl.OK
    assert nb.value >= 16
