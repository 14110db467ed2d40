"""Test-side workloads: the seeded synthetic fields (synth, inputs only) with
their feature masks and coresets taken from the oracle (oracle/coreset.py), so
every mask and coreset a parity test feeds to the HIP path comes from the
plain definition, never from the HIP coreset kernels."""
import numpy as np

from oracle import coreset as OC
from paper_2507_03836_amd import synth


def tiny_volume():
    """(field float32 [T][Sz][Sy][Sx], mask uint8 of the same shape): value > 0.1,
    dilated by 1 (the tiny parity workload)."""
    f = synth.tiny_field()
    m = OC.dilate(OC.feature_interval(f, synth.TINY_FEATURE_LO, np.inf), synth.TINY_DILATION)
    return f, m.astype(np.uint8)


def production_volume_host(shape, seed):
    """Small-shape production workload: field, mask (|grad| above its 80th
    percentile, dilated by 2)."""
    f, g, thr = synth.production_field_host(shape, seed)
    m = OC.dilate(OC.feature_interval(g, thr, np.inf), synth.PRODUCTION_DILATION)
    return f, m.astype(np.uint8)


def coreset_ids(mask):
    """Increasing uint64 linear voxel ids of the mask (Eq. (3) union)."""
    return OC.coreset_ids(np.asarray(mask, bool))


def render_bound(pix, tf, rtol=1e-5, atol=1e-12, alpha_stop=0.99):
    """Per-pixel bound on |image - oracle image| for a renderer that decodes in
    FP32 and composites in FP32, from the oracle's per-pixel statistics pix
    ([H][W][3]: composited samples n, sum of their output magnitudes, smallest
    |A - alpha_stop|).  Each decoded value is within rtol * magnitude + atol of
    the oracle's; the transfer function is piecewise linear with slope at most
    s = 255 max |tf[i+1] - tf[i]|, so colour and opacity move by at most s times
    that, plus a few FP32 roundings of its evaluation; front-to-back
    compositing (partial derivatives of A and C by any sample's colour or
    opacity are at most 1 in magnitude) adds the per-sample changes of opacity
    twice and of colour once, plus four FP32 roundings per step.  Pixels whose
    opacity came within the opacity bound of alpha_stop may stop one sample
    apart (ambiguous): the sample composited by one side and not the other
    adds (1 - A) a c <= 1 - alpha_stop + (the opacity bound) to each channel,
    which their bound includes.  Returns (bound [H][W][1], ambiguous [H][W])."""
    u = 2.0 ** -24
    tf = np.asarray(tf, np.float64)
    s = 255.0 * np.abs(np.diff(tf, axis=0)).max()
    n, ymag, margin = pix[..., 0], pix[..., 1], pix[..., 2]
    dval = s * (rtol * ymag + atol * n) + 3 * u * n
    d_alpha = dval + 4 * u * n
    bound = 3 * dval + 4 * u * n + 1e-7
    ambiguous = margin <= d_alpha
    bound = np.where(ambiguous, bound + (1.0 - float(np.float32(alpha_stop))) + d_alpha, bound)
    return bound[..., None], ambiguous
