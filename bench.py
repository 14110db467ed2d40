#!/usr/bin/env python3
"""Benchmarks of the F-Hash hot path on one MI355X.

Default (the headline metric: training samples/s fwd+bwd, FP32 vs mixed
precision at equal PSNR, and render p50/p99): the differentiated
mixed-precision training workload.  A seeded synthetic 432^3 x 60 float32
volume (64 advected Gaussian blobs + 3-octave value-noise turbulence, min-max
normalised), feature = gradient magnitude above its 80th percentile, dilated
by 2, coreset = feature voxels (all through the coreset-selection calls);
16 levels (spatial 16..512 clamped to 432, temporal 4..60), 2 features per
level, decoder 32-64-64-64-1, batch 2^20 coreset draws per step, Adam lr 0.01.

* FP32 path: FP32 tables and FP32-MFMA decoder; mixed path: BF16-MFMA decoder
  with FP32 accumulation, FP32 master tables / moments, dynamic loss scaling;
  its table reads are FP32 by default (--mixed-table-reads f16: an FP16 copy
  written by Adam).  Each path: W warm-up steps,
  K timed steps (HIP events per phase on the launch stream), then training on
  to the common probe-PSNR target (40 dB on 2^22 coreset draws), wall time from
  the first step.
* Render serving with the mixed model (FP16 tables, BF16 decoder): requests of
  side 256/512/1024, fractional t, orbit cameras, ds = 1/2 voxel, ARM max 64,
  alpha stop 0.99; saturation, then Poisson arrivals at 0.25/0.5/0.9 x
  saturation, continuous batching against one request at a time.
* roofline: the dominant kernel of the reported path's step (the fused
  training kernel), with the algorithmic bytes per sample and the compulsory
  128-byte lines of the timed batch (directory, table and gradient lines its
  corners touch, counted with fhash_corner_rows).

Other modes: --workload train (the 480 x 720 x 120 x 100 training
configuration and its variants), --serve, --serve-multi, --key-frames,
--coreset.  Inputs are resident in HBM before timing starts.  Prints ONE JSON
line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Dense Adam moves 24 B per parameter (read p, m, v; write p, m, v), plus 4 B for every
# gradient float it must read: all of them untracked, only those in flagged 64-B segments
# under touched-segment tracking (plus one flag byte per tracked segment); the gradient
# reset is not counted.  The FP16 shadow adds 2 B per parameter.
ADAM_RW_BYTES_PER_PARAM = 24
# HBM bytes of one adam_kernel launch at the default workload (FP32, tracked), from
# rocprofv3 FETCH_SIZE (x2.000) and WRITE_SIZE (x1.000) passes scaled by a plain streaming
# copy of known size; valid only for the parameter count, optimiser state layout and
# optimizer source they were taken on.
ADAM_TRAFFIC = {"bytes": 160.80e9, "params": 6390343593, "moments": "with-params",
                "source_md5": "f6d69b782465363a0baa0efdebaf6158"}

# Catch-up of the deferred Adam (one launch per step), algorithmic bytes: the claim flags of
# the whole range are read (1 B per segment of 16 floats); every flagged segment reads and
# writes its 8-B state word (16 B); a segment stepped before reads and writes p, m, v
# (6 x 64 B); a pending gradient is read and reset (2 x 64 B); the FP16 shadow adds 32 B
# written.
LAZY_ENTRY_BYTES, LAZY_LOADED_BYTES, LAZY_PENDING_BYTES, LAZY_SHADOW_BYTES = 16, 384, 128, 32
# HBM bytes of one lazy_catchup_kernel launch of the training workload (480x720x120x100,
# FP32, 200 timed steps), from rocprofv3 FETCH_SIZE and WRITE_SIZE passes
# (copy-calibrated, per launch, averaged over the timed steps); valid only for the
# sources, optimiser state layout, parameter count, batch and step count they were
# taken on.
CATCHUP_TRAFFIC = {"bytes": 9.084e9, "raw_bytes": 6.464e9, "params": 6390343593,
                   "batch": 1 << 18, "steps": 200, "moments": "with-params",
                   "source_md5": "15eec88035e7f0c606f4974f8402c0d0"}

# HBM bytes of one feature-extraction launch on the 480x720x120x100 volume from the two
# counter passes (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, the copy-calibrated factors);
# valid only while the source text of classify4_kernel (hashed alone by _kernel_md5) and
# the volume shape equal those the counters were taken on.
CLASSIFY_TRAFFIC = {"bytes": 17141931808.0, "shape": [480, 720, 120, 100],
                    "kernel_md5": "069f488afcee6ec399a6892a53ef8c05"}


def _layout_kw(args, lazy=True):
    """Model keywords of the optimiser state layout chosen by --moments (the
    layout with parameters is built for the deferred update's models)."""
    return {"paired_moments": args.moments == "paired" or (args.moments == "with-params"
                                                         and not lazy),
            "moments_with_params": args.moments == "with-params" and lazy}


def _reads_kw(args, precision):
    """Model keywords of the mixed path's table reads and decoder arithmetic
    (--mixed-table-reads, --mixed-decoder)."""
    if precision != "mixed":
        return {"table_reads": "f32"}
    return {"table_reads": args.mixed_table_reads, "decoder": args.mixed_decoder}


def _kernel_md5(path, name):
    """md5 of one kernel's source text: from the line holding `name(` back to
    the preceding __global__, through the brace that closes its body."""
    import hashlib
    src = open(path).read()
    i = src.index(name + "(")
    i = src.rindex("__global__", 0, i)
    j = src.index("{", src.index(name + "(", i))
    depth = 0
    for k in range(j, len(src)):
        depth += {"{": 1, "}": -1}.get(src[k], 0)
        if depth == 0:
            return hashlib.md5(src[i:k + 1].encode()).hexdigest()
    raise ValueError(name)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["headline", "train"], default="headline",
                    help="headline: 432^3 x 60 FP32 vs mixed + render serving; train: the "
                         "single-path training benchmark selected by the options below")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=1 << 18)
    ap.add_argument("--shape", type=str, default="480,720,120,100")
    ap.add_argument("--levels", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1 << 12)
    ap.add_argument("--precision", choices=["fp32", "mixed"], default="fp32",
                    help="mixed: FP16 table reads (Adam-written shadow) + dynamic loss scaling")
    ap.add_argument("--optimizer", choices=["lazy", "tracked", "dense"], default="lazy",
                    help="Adam over the large levels: deferred (same values, bit for bit), "
                         "dense with touched-segment gradient reads, or plain dense")
    ap.add_argument("--key-frames", type=int, default=0,
                    help="K > 1: train on K key frames evenly spaced over the timesteps "
                         "(finest temporal resolution = K) and report PSNR on seen and "
                         "unseen frames next to a model trained on every frame")
    ap.add_argument("--hash-bits", type=int, default=0,
                    help="b > 0: the spatial-hash comparison index instead of F-Hash (levels "
                         "of more than 2^b vertices hash into 2^b rows, collisions allowed)")
    ap.add_argument("--fold-sweep", action="store_true",
                    help="dense FBB model with fold-policy levels: embedding size x fold sweep")
    ap.add_argument("--dense-index", action="store_true",
                    help="index every vertex of the box (the F-Hash equation, no feature mask) "
                         "instead of the vertices of active cells; samples still come from "
                         "the coreset")
    ap.add_argument("--hidden-layers", type=int, default=2)
    ap.add_argument("--moments", choices=["with-params", "paired", "separate"],
                    default="with-params",
                    help="optimiser state layout of the deferred-Adam models: a segment's 16 "
                         "parameters and their m in one 128-byte line and its gradients and v "
                         "in another (with-params), m and v in one line (paired), or four "
                         "arrays")
    ap.add_argument("--layout", choices=["rows", "bricks"], default="rows",
                    help="slot order of the active index: the F-Hash equation's rows, or "
                         "2x2x2x2 vertex bricks (Sec. 3.2.3 allows other linearisations)")
    ap.add_argument("--mixed-table-reads", choices=["f16", "f32"], default="f32",
                    help="what the mixed path's fused kernels gather from the tables: the FP32 "
                         "master (f32), or an FP16 copy that the Adam update writes beside it "
                         "(f16: one more scattered store per updated segment, and the fused "
                         "kernel, bound by its atomics, gains nothing from the smaller reads); "
                         "the decoder runs on BF16 MFMA either way")
    ap.add_argument("--mixed-decoder", choices=["f16", "bf16"], default="f16",
                    help="the 16-bit MFMA type of the mixed path's decoder (FP32 accumulation; "
                         "f16 keeps 3 more mantissa bits and tracks the FP32 path's PSNR "
                         "closely under the dynamic loss scale)")
    ap.add_argument("--paths", choices=["fp32,mixed", "mixed,fp32"], default="fp32,mixed",
                    help="headline: the order in which the two training paths run")
    ap.add_argument("--no-sort", dest="sort", action="store_false",
                    help="train on batches in draw order instead of sorting each batch by a "
                         "4D Morton key before the fused step (sorted, the lanes of one "
                         "scatter instruction that add into one 64-byte chunk share one "
                         "atomic request, and the gathers share lines)")
    ap.add_argument("--no-coarse-lds", dest="coarse_lds", action="store_false",
                    help="add the coarse levels' encoding gradient in the fused kernel instead of "
                         "summing it in LDS per chunk of the batch before its atomics "
                         "(FHASH_COARSE_LDS, the default)")
    ap.add_argument("--sort-reduce", action="store_true",
                    help="with sorted batches: at the coarse levels, sum a corner across the "
                         "samples of a scatter instruction before one atomic when they all "
                         "share its slot (FHASH_SAMPLES_SORTED)")
    ap.add_argument("--field-seed", type=int, default=1002)
    ap.add_argument("--sampler-seed", type=int, default=2002)
    ap.add_argument("--psnr-target", type=float, default=0.0,
                    help="after the timed steps, keep training until the probe PSNR reaches this")
    ap.add_argument("--max-steps", type=int, default=2000)
    ap.add_argument("--eval-every", type=int, default=5)
    ap.add_argument("--serve", action="store_true",
                    help="render-serving benchmark instead of training (p50/p99 at 3 rates)")
    ap.add_argument("--serve-shape", type=str, default="432,432,432,60")
    ap.add_argument("--serve-train-steps", type=int, default=300)
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-sizes", type=str, default="256,512,1024")
    ap.add_argument("--serve-rates", type=str, default="0.25,0.5,0.9",
                    help="Poisson rates as fractions of the saturation request rate")
    ap.add_argument("--serve-decoder", choices=["f32", "f16"], default="f32",
                    help="decoder arithmetic of the served models (FP32 or FP16 MFMA)")
    ap.add_argument("--serve-multi", action="store_true",
                    help="multi-model serving: 6 resident models, mixed renders + point queries")
    ap.add_argument("--coreset", action="store_true",
                    help="coreset-selection benchmark: feature extraction, dilation, boxes, "
                         "occupancy grid and coreset list over the whole volume")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 4 GiB device copy first (counter calibration)")
    return ap.parse_args()


def cpu_baseline(model, gen, dims, batch, n_cpu, seed):
    """Time the FP64 oracle, as it stands, on a bounded sample of the workload.

    Sample: n_cpu coreset draws (the oracle's own Philox sampler) through the
    oracle's encoding + decoder forward, MSE and backward with the same level
    structure (dense-box index: slot = F-Hash equation; the per-sample work is
    the same 16 levels x 16 corners), plus the oracle's Adam on a 2^22-parameter
    chunk.  Scaled to one full step: fwd+bwd time x batch/n_cpu + Adam time x
    (parameter count / chunk)."""
    import numpy as np

    import oracle as O

    M = gen["M"]
    ids = O.sample_ids(seed, 1, n_cpu, M)
    ids_t = torch.from_numpy(ids.view(np.int64)).cuda()
    lin = gen["coreset"][ids_t].cpu().numpy().view(np.uint64)
    tgt = gen["field"].view(-1)[torch.from_numpy(lin.view(np.int64)).cuda()].cpu().numpy()
    pos = O.voxel_positions(lin, dims)
    cfg = model.cfg
    g = O.Grid(np.array(cfg.res), cfg.n_features, None)
    rows = g.total_slots
    table = np.zeros((rows, cfg.n_features))  # lazily committed pages
    width = cfg.width
    params = model.mlp_params.double().cpu().numpy()
    t0 = time.perf_counter()
    enc, _ = O.encode_fwd(g, pos, table)
    y, acts, _ = O.mlp_fwd(width, params, enc)
    L, dy = O.mse(y[:, 0], tgt.astype(np.float64))
    dp, denc, _, _ = O.mlp_bwd(width, params, acts, dy.reshape(-1, 1), n_cpu)
    dt, _ = O.encode_bwd(g, pos, denc)
    t_fb = time.perf_counter() - t0
    del table, dt
    chunk = 1 << 22
    p = np.zeros(chunk)
    gr = np.random.default_rng(0).normal(size=chunk)
    m = np.zeros(chunk)
    v = np.zeros(chunk)
    t0 = time.perf_counter()
    O.adam(p, gr, m, v, 0.01, 0.9, 0.999, 1e-8, 1)
    t_adam = time.perf_counter() - t0
    t_step = t_fb * batch / n_cpu + t_adam * model.n_params / chunk
    return {"value": batch / t_step, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": (f"{n_cpu} coreset draws fwd+bwd ({t_fb:.2f} s) scaled to {batch}, "
                       f"+ Adam on {chunk} params ({t_adam:.3f} s) scaled to {model.n_params}; "
                       "dense-box index, FP64, single thread")}


def time_to_psnr(args, model, step, gen, dims, t_train0, k_done):
    """Keep training after the timed steps until the probe PSNR reaches the
    target (or max steps).  Probe: 2^22 coreset draws (sampler seed + 2000).
    Wall time counts every training step since the first warm-up step plus
    the probe evaluations."""
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd.model import psnr_on
    P = 1 << 22
    ppos = torch.empty(P, 4, device="cuda")
    ptgt = torch.empty(P, device="cuda")
    fl.fhash_sample(args.sampler_seed + 2000, 1, P, gen["coreset"], gen["M"], dims,
                    gen["field"], ppos, ptgt)
    k = k_done
    hist = []
    reached = None
    near = False  # within 1 dB of the target: evaluate after every step
    while True:
        if near or (k - k_done) % args.eval_every == 0 or k >= args.max_steps:
            ps = psnr_on(model, ppos, ptgt)
            el = time.perf_counter() - t_train0
            hist.append((k, round(el, 3), round(ps, 3)))
            log(f"[bench] step {k}: probe PSNR {ps:.3f} dB at {el:.1f} s")
            if ps >= args.psnr_target:
                reached = (k, el, ps)
                break
            if k >= args.max_steps:
                break
            near = ps >= args.psnr_target - 1.0
        k += 1
        step(k)
    return {"target_db": args.psnr_target, "reached": reached is not None,
            "steps": reached[0] if reached else None,
            "seconds": reached[1] if reached else None,
            "final_psnr_db": hist[-1][2], "history": hist,
            "probe": "2^22 coreset draws, PSNR over data range 1, FP64 sum on the device"}


def key_frame_bench(args):
    """Key-frame training with temporal super-resolution (Sec. 3.2.2): n_kf key
    frames evenly spaced over the T frames (first and last included, frame
    round(k (T-1) / (n_kf-1))); samples only from their coreset
    (fhash_coreset_frames); the time coordinate of every frame from
    fhash_key_frame_times, so key frames sit on the vertices of the finest
    temporal level (n_kf vertices, geometric temporal range 4..n_kf); PSNR on
    coreset draws at the key frames (seen) and at the other frames (unseen,
    reached only through the temporal interpolation), next to the same model
    trained on every frame (finest temporal level T) for the same steps."""
    import numpy as np
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import volume
    from paper_2507_03836_amd.model import (FHashConfig, FHashModel, geometric_resolutions,
                                            psnr_on)
    fl.lib()
    dims = [int(x) for x in args.shape.split(",")]
    T = dims[3]
    n_kf = args.key_frames
    key = sorted({int(round(k * (T - 1) / (n_kf - 1))) for k in range(n_kf)})
    unseen = [n for n in range(T) if n not in key]
    gen = volume.production_volume(dims, seed=args.field_seed)
    frame_t = torch.from_numpy(fl.fhash_key_frame_times(T, key)).cuda()
    cs_key = fl.fhash_coreset_frames(gen["bits"], dims, key)
    cs_unseen = fl.fhash_coreset_frames(gen["bits"], dims, unseen)
    P = 1 << 22
    B = args.batch
    out = {"metric": "probe PSNR (dB) on seen and unseen frames after key-frame training",
           "unit": "dB", "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"F-Hash key-frame training, {'x'.join(map(str, dims))} "
                                  f"synthetic volume, {len(key)} key frames of {T}, batch "
                                  f"2^{int(np.log2(B))}, {args.steps} steps",
                      "key_frames": key, "key_voxels": int(cs_key.numel()),
                      "unseen_voxels": int(cs_unseen.numel())},
           "runs": {}}
    pos = torch.empty(B, 4, device="cuda")
    tgt = torch.empty(B, device="cuda")
    for label, cs, rt, ft in (("key_frames", cs_key, len(key), frame_t),
                              ("all_frames", gen["coreset"], T, None)):
        probes = {}
        for name, c, seed in (("seen", cs_key, 7001), ("unseen", cs_unseen, 7002)):
            pp = torch.empty(P, 4, device="cuda")
            pt = torch.empty(P, device="cuda")
            fl.fhash_sample(seed, 1, P, c, c.numel(), dims, gen["field"], pp, pt, frame_t=ft)
            probes[name] = (pp, pt)
        res = geometric_resolutions(args.levels, 16, 512, 4, rt, dims)
        cfg = FHashConfig(res=res, n_features=2, hidden=64, n_hidden=args.hidden_layers,
                          layout=LAYOUTS[args.layout])
        model = FHashModel(cfg, gen["bits"], dims, init_seed=3000, lazy=True,
                           **_layout_kw(args),
                           max_steps=args.steps + 8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            fl.fhash_sample(args.sampler_seed, k + 1, B, cs, cs.numel(), dims, gen["field"], pos,
                            tgt, frame_t=ft)
            model.fwd_bwd(pos, tgt)
            model.optimizer_step()
        model.flush()
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        r = {"train_s": secs, "params": model.n_params, "temporal_res_finest": res[-1][3]}
        for name, (pp, pt) in probes.items():
            r[f"psnr_{name}_db"] = psnr_on(model, pp, pt)
        out["runs"][label] = r
        log(f"[keyframes] {label}: {r}")
        model.params = model.grads = model.m = model.v = model.mv = model.pm = model.gv = None
        del model, probes
        torch.cuda.empty_cache()
    out["value"] = out["runs"]["key_frames"]["psnr_unseen_db"]
    print(json.dumps(out), flush=True)


def fold_sweep_bench(args):
    """The paper's published mode on the product path: a dense model over the
    feature bounding box (Sec. 3.1: FBB of the key frames' feature, positions
    translated and scaled to it), fold-policy levels (Sec. 3.2.1-3.2.2:
    fhash_fold_resolutions of the FBB size and the key-frame count), trained on
    the key frames' coreset; embedding size F in {1, 2, 4} x fold in {2, 4, 6}
    (the shape of the paper's Table 1).  Per cell: levels, parameters, ms per
    step with the deferred Adam (batch as --batch), the fused kernel's share,
    one dense Adam sweep over every parameter, and probe PSNR after --steps
    steps.  Cells whose decoder input L x F exceeds 32 are not built for the
    fused kernels and are reported as such."""
    import numpy as np
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import volume
    from paper_2507_03836_amd.model import FHashConfig, FHashModel, psnr_on
    fl.lib()
    dims = [int(x) for x in args.shape.split(",")]
    T = dims[3]
    n_kf = 10
    key = sorted({int(round(k * (T - 1) / (n_kf - 1))) for k in range(n_kf)})
    gen = volume.production_volume(dims, seed=args.field_seed)
    boxes = fl.fhash_feature_boxes(gen["bits"], dims).cpu().numpy()[key]
    fbb = [int(boxes[:, d].min()) for d in range(3)] + [int(boxes[:, 3 + d].max())
                                                        for d in range(3)]
    size = [fbb[3 + d] - fbb[d] + 1 for d in range(3)] + [len(key)]
    frame_t = torch.from_numpy(fl.fhash_key_frame_times(T, key)).cuda()
    cs = fl.fhash_coreset_frames(gen["bits"], dims, key)
    B = args.batch
    pos = torch.empty(B, 4, device="cuda")
    tgt = torch.empty(B, device="cuda")
    P = 1 << 21
    ppos = torch.empty(P, 4, device="cuda")
    ptgt = torch.empty(P, device="cuda")
    fl.fhash_sample(7003, 1, P, cs, cs.numel(), dims, gen["field"], ppos, ptgt, frame_t=frame_t,
                    box=fbb)
    stream = torch.cuda.current_stream()
    cells = []
    for fold in (2, 4, 6):
        res = fl.fhash_fold_resolutions(size, fold)
        for F in (1, 2, 4):
            cell = {"fold": fold, "F": F, "levels": len(res), "res_finest": res[-1]}
            if len(res) * F > 32:
                cell["built"] = False
                cells.append(cell)
                log(f"[fold] fold {fold} F {F}: {len(res)} levels x {F} > 32 inputs, not built")
                continue
            cfg = FHashConfig(res=res, n_features=F, hidden=64, n_hidden=2)
            model = FHashModel(cfg, None, dims, init_seed=3000, lazy=True,
                               **_layout_kw(args, lazy=False),
                               max_steps=args.steps + 8)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            fb_ms = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                fl.fhash_sample(args.sampler_seed, k + 1, B, cs, cs.numel(), dims, gen["field"],
                                pos, tgt, frame_t=frame_t, box=fbb)
                model.prepare(pos)
                ev[0].record(stream)
                model.fwd_bwd(pos, tgt, prepared=True)
                ev[1].record(stream)
                model.optimizer_step()
                ev[1].synchronize()
                fb_ms.append(ev[0].elapsed_time(ev[1]))
            model.flush()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            psnr = psnr_on(model, ppos, ptgt)
            # one dense Adam sweep over every parameter (the optimiser of the paper)
            opt = model.adam_desc(args.steps + 1)
            n = model.n_params
            ev[2].record(stream)
            fl.fhash_step(opt, model.params[:n], model.grads[:n], model.m[:n], model.v[:n])
            ev[3].record(stream)
            torch.cuda.synchronize()
            cell.update({"built": True, "params": n, "ms_per_step": ms,
                         "fused_fwd_bwd_ms": float(np.median(fb_ms)),
                         "dense_adam_ms": ev[2].elapsed_time(ev[3]), "psnr_db": psnr})
            cells.append(cell)
            log(f"[fold] fold {fold} F {F}: {cell}")
            model.params = model.grads = model.m = model.v = None
            model.mv = model.pm = model.gv = model.lazy = None
            del model
            torch.cuda.empty_cache()
    out = {"metric": "training ms/step and probe PSNR over embedding size x fold (dense FBB)",
           "unit": "ms/step", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"F-Hash dense FBB model, {'x'.join(map(str, dims))} synthetic "
                                  f"volume, {len(key)} key frames, FBB {size[:3]}, decoder "
                                  f"L*F-64-64-1, batch 2^{int(np.log2(B))}, {args.steps} steps",
                      "key_frames": key, "fbb": fbb, "coreset": int(cs.numel())},
           "cells": cells}
    print(json.dumps(out), flush=True)


def serve_multi_bench(args):
    """Six resident models (480x720x120x100, 640x256x256x100 and 432^3x60, two
    field seeds each; 16 levels, MLP 32-64-64-64-1, FP16 tables), each trained
    for --serve-train-steps steps at batch 2^20, then a Poisson stream of
    requests to random models: every 4th a render (side uniform over
    {256, 512, 1024}, fractional t, orbit camera), the others point-query
    batches of 2^k points, k ~ U{10..20}.  Requests are admitted by device
    bytes next to the resident models.  Continuous batching (backfill) vs one
    request at a time, same arrivals, at 0.5 x the saturation rate."""
    import numpy as np

    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import synth, volume
    from paper_2507_03836_amd.model import FHashConfig, FHashModel, geometric_resolutions, psnr_on
    from paper_2507_03836_amd.serving import (GpuExecutor, Request, ResidentModel, Scheduler,
                                              latency_stats, poisson_arrivals)

    fl.lib()
    torch.cuda.set_device(0)
    C = 1 << 22
    shapes = [[480, 720, 120, 100], [640, 256, 256, 100], [432, 432, 432, 60]]
    tf = torch.from_numpy(synth.transfer_function()).cuda()
    models, info = {}, []
    for i, dims in enumerate(shapes):
        for seed in (1005 + 10 * i, 1006 + 10 * i):
            t0 = time.time()
            gen = volume.production_volume(dims, seed=seed)
            res = geometric_resolutions(16, 16, 512, 4, dims[3], dims)
            cfg = FHashConfig(res=res, n_features=2, hidden=64, n_hidden=3,
                              layout=LAYOUTS[args.layout])
            model = FHashModel(cfg, gen["bits"], dims, init_seed=seed + 2000, lazy=True,
                               **_layout_kw(args),
                               max_steps=args.serve_train_steps + 8)
            B = 1 << 20
            pos = torch.empty(B, 4, device="cuda")
            tgt = torch.empty(B, device="cuda")
            for k in range(args.serve_train_steps):
                fl.fhash_sample(seed + 1000, k + 1, B, gen["coreset"], gen["M"], dims,
                                gen["field"], pos, tgt)
                model.fwd_bwd(pos, tgt)
                model.optimizer_step()
            fl.fhash_sample(seed + 3000, 1, B, gen["coreset"], gen["M"], dims, gen["field"],
                            pos, tgt)
            psnr = psnr_on(model, pos, tgt)
            model.flush()
            table16 = torch.empty(model.n_table, dtype=torch.float16, device="cuda")
            fl.fhash_cast(model.table, table16)
            name = f"{'x'.join(map(str, dims))}/s{seed}"
            mlp = fl.mlp_desc(cfg.width, fl.F16 if args.serve_decoder == "f16" else fl.F32)
            models[name] = ResidentModel(index=model.index, mlp=mlp, table=table16,
                                         params=model.mlp_params.clone(), mask_bits=gen["bits"],
                                         dims=dims, tf=tf, keep=(model._dir,),
                                         occ=fl.fhash_occupancy_grid(gen["bits"], dims))
            info.append({"model": name, "params": model.n_params, "probe_psnr_db": psnr,
                         "resident_bytes": models[name].nbytes()})
            del gen, pos, tgt
            model.params = model.grads = model.m = model.v = model.mv = model.pm = model.gv = None
            del model
            torch.cuda.empty_cache()
            log(f"[multi] {name}: {info[-1]['params']} params, PSNR {psnr:.1f} dB, resident "
                f"{info[-1]['resident_bytes'] / 2**30:.1f} GiB ({time.time() - t0:.1f} s)")
    names = list(models)
    rng = np.random.default_rng(5007)
    g = torch.Generator(device="cuda")
    g.manual_seed(5007)
    sizes = [int(x) for x in args.serve_sizes.split(",")]
    n_req = 4 * args.serve_requests
    spec = []
    for i in range(n_req):
        m = names[int(rng.integers(0, len(names)))]
        dims = models[m].dims
        if i % 4 == 0:
            S = int(rng.choice(sizes))
            view = synth.orbit_view(dims, float(rng.uniform(0, 2 * np.pi)),
                                    float(rng.uniform(-np.pi / 3, np.pi / 3)), S, S)
            spec.append(("render", m, S, view, float(rng.uniform(0, dims[3] - 1))))
        else:
            n = 1 << int(rng.integers(10, 21))
            spec.append(("points", m, torch.rand(n, 4, device="cuda", generator=g)))

    def requests(arr):
        out = []
        for sp, a in zip(spec, arr):
            if sp[0] == "render":
                _, m, S, v, t = sp
                out.append(Request(model=m, kind="render", view=v, t=t, W=S, H=S,
                                   arrival=float(a)))
            else:
                out.append(Request(model=sp[1], kind="points", pos=sp[2], n=sp[2].shape[0],
                                   arrival=float(a)))
        return out

    def serve(arr, realtime, **kw):
        ex = GpuExecutor(sample_budget=C)
        for k, m in models.items():
            ex.add_model(k, m)
        free, _ = torch.cuda.mem_get_info()
        sch = Scheduler(ex, sample_budget=C, mem_budget=int(free * 0.8), **kw)
        torch.cuda.synchronize()
        done = sch.run(requests(arr), realtime=realtime)
        return {"all": latency_stats(done),
                "render": latency_stats([r for r in done if r.kind == "render"]),
                "points": latency_stats([r for r in done if r.kind == "points"]),
                "iterations": sch.iterations, "peak_active": sch.peak_active,
                "peak_request_bytes": sch.peak_mem, "mem_budget": sch.mem_budget,
                "resident_bytes": ex.resident_bytes()}

    serve([0.0] * 4, realtime=False)  # warm-up (first 4 requests)
    sat = serve([0.0] * n_req, realtime=False)
    rate = 0.5 * sat["all"]["requests_per_s"]
    arr = poisson_arrivals(rate, n_req, seed=5008)
    cb = serve(arr, realtime=True)
    one = serve(arr, realtime=True, max_active=1)
    for name, x in (("continuous_backfill", cb), ("one_at_a_time", one)):
        log(f"[multi] {rate:.2f}/s {name}: render p50 {x['render']['p50_ms']:.1f} p99 "
            f"{x['render']['p99_ms']:.1f} ms; points p50 {x['points']['p50_ms']:.1f} p99 "
            f"{x['points']['p99_ms']:.1f} ms")
    out = {
        "metric": "multi-model serving p50/p99 ms (renders and point queries), 0.5 x saturation",
        "value": sat["all"]["requests_per_s"], "unit": "requests/s at saturation", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None,
        "dtype": f"f16 tables, {args.serve_decoder} MLP", "data": "synthetic",
        "config": {"workload": "6 resident models (480x720x120x100, 640x256x256x100, "
                   "432x432x432x60; 2 seeds each), 16 levels, MLP 32-64-64-64-1, FP16 tables; "
                   "1 in 4 requests a render, the rest 2^10-2^20 point queries",
                   "requests": n_req, "sample_budget": C, "models": info},
        "saturation": sat, "rate_per_s": rate, "continuous_backfill": cb, "one_at_a_time": one,
    }
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Render serving: a trained model (432^3 x 60 volume, 16 levels, MLP
    32-64-64-64-1, FP16 tables) answers ray-march requests of sizes uniform
    over {256^2, 512^2, 1024^2}, t ~ U[0, T-1] (fractional), orbit cameras
    (azimuth U[0, 2pi), elevation U[-60, 60] deg, distance 2x the half
    diagonal, fovy 45 deg), ds = 1/2 voxel, alpha stop 0.99, ARM max 64.

    Saturation: every request submitted at once, continuous batching.  Then
    Poisson arrivals at 0.25 / 0.5 / 0.9 x the saturation request rate, served
    by continuous batching and by a one-request-at-a-time server (same
    arrivals).  ARM off (pace 1) is timed at saturation too."""
    import numpy as np

    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import synth, volume
    from paper_2507_03836_amd.model import FHashConfig, FHashModel, geometric_resolutions, psnr_on
    from paper_2507_03836_amd.serving import (GpuExecutor, Request, ResidentModel, Scheduler,
                                              latency_stats, poisson_arrivals)

    fl.lib()
    torch.cuda.set_device(0)
    dims = [int(x) for x in args.serve_shape.split(",")]
    t0 = time.time()
    gen = volume.production_volume(dims, seed=1003)
    log(f"[serve] volume {dims} in {time.time() - t0:.1f} s; coreset {gen['M']}")
    res = geometric_resolutions(16, 16, 512, 4, dims[3], dims)
    cfg = FHashConfig(res=res, n_features=2, hidden=64, n_hidden=3,
                      layout=LAYOUTS[args.layout])
    model = FHashModel(cfg, gen["bits"], dims, init_seed=3003, lazy=True,
                       **_layout_kw(args),
                       max_steps=args.serve_train_steps + 8)
    log(f"[serve] model: {model.rows} active vertices, {model.n_params} params")
    B = 1 << 20
    pos = torch.empty(B, 4, device="cuda")
    tgt = torch.empty(B, device="cuda")
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(args.serve_train_steps):
        fl.fhash_sample(2003, k + 1, B, gen["coreset"], gen["M"], dims, gen["field"], pos, tgt)
        model.fwd_bwd(pos, tgt)
        model.optimizer_step()
    torch.cuda.synchronize()
    t_train = time.time() - t0
    probe = 1 << 22
    ppos = torch.empty(probe, 4, device="cuda")
    ptgt = torch.empty(probe, device="cuda")
    fl.fhash_sample(4003, 1, probe, gen["coreset"], gen["M"], dims, gen["field"], ppos, ptgt)
    psnr = psnr_on(model, ppos, ptgt)
    log(f"[serve] trained {args.serve_train_steps} steps in {t_train:.1f} s; probe PSNR {psnr:.2f} dB")
    model.flush()
    table16 = torch.empty(model.n_table, dtype=torch.float16, device="cuda")
    fl.fhash_cast(model.table, table16)
    params = model.mlp_params.clone()
    bits = gen["bits"]
    del gen, pos, tgt, ppos, ptgt
    model.params = model.grads = model.m = model.v = model.mv = model.pm = model.gv = None
    torch.cuda.empty_cache()
    tf = torch.from_numpy(synth.transfer_function()).cuda()
    mlp = fl.mlp_desc(cfg.width, fl.F16 if args.serve_decoder == "f16" else fl.F32)
    rm = ResidentModel(index=model.index, mlp=mlp, table=table16, params=params,
                       mask_bits=bits, dims=dims, tf=tf, keep=(model._dir,),
                       occ=fl.fhash_occupancy_grid(bits, dims))
    C = 1 << 22
    sizes = [int(x) for x in args.serve_sizes.split(",")]
    rng = np.random.default_rng(5004)
    spec = []
    for i in range(args.serve_requests):
        S = int(rng.choice(sizes))
        az = float(rng.uniform(0, 2 * np.pi))
        el = float(rng.uniform(-np.pi / 3, np.pi / 3))
        t = float(rng.uniform(0, dims[3] - 1))
        spec.append((S, synth.orbit_view(dims, az, el, S, S), t))

    def requests(arr):
        return [Request(model="m", kind="render", view=v, t=t, W=S, H=S, arrival=float(a))
                for (S, v, t), a in zip(spec, arr)]

    def serve(reqs, realtime, max_active=64, arm_max=64, policy="backfill"):
        ex = GpuExecutor(sample_budget=C, arm_max=arm_max)
        ex.add_model("m", rm)
        free, _ = torch.cuda.mem_get_info()
        sch = Scheduler(ex, sample_budget=C, mem_budget=int(free * 0.8), max_active=max_active,
                        arm_max=arm_max, policy=policy)
        torch.cuda.synchronize()
        done = sch.run(reqs, realtime=realtime)
        st = latency_stats(done)
        st["iterations"] = sch.iterations
        st["samples"] = sch.samples
        st["peak_active"] = sch.peak_active
        return st

    serve(requests([0.0] * 2), realtime=False)  # warm-up
    sat = serve(requests([0.0] * len(spec)), realtime=False)
    log(f"[serve] saturation: {sat}")
    rate_sat = sat["requests_per_s"]
    arm_off = serve(requests([0.0] * len(spec)), realtime=False, arm_max=1)
    log(f"[serve] ARM off: {arm_off}")
    sat_one = serve(requests([0.0] * len(spec)), realtime=False, max_active=1)
    log(f"[serve] one at a time, all submitted at once: {sat_one}")
    rates = []
    for frac in [float(x) for x in args.serve_rates.split(",") if x]:
        rate = frac * rate_sat
        arr = poisson_arrivals(rate, len(spec), seed=5004)
        row = {"rate_frac": frac, "rate_per_s": rate}
        for name, kw in (("continuous_oldest_first", {"policy": "oldest_first"}),
                         ("continuous_shared_pace", {"policy": "shared"}),
                         ("continuous_backfill", {}),
                         ("one_at_a_time", {"max_active": 1})):
            row[name] = serve(requests(arr), realtime=True, **kw)
            log(f"[serve] rate {rate:.3f}/s {name}: p50 {row[name]['p50_ms']:.1f} ms, "
                f"p99 {row[name]['p99_ms']:.1f} ms, {row[name]['rays_per_s'] / 1e6:.2f} Mrays/s")
        rates.append(row)

    # mixed stream: every 4th request a render, the others point-query batches of
    # 2^k points, k ~ U{10..20}, positions U[0,1)^4
    g = torch.Generator(device="cuda")
    g.manual_seed(5005)
    krng = np.random.default_rng(5005)
    pts = [torch.rand(1 << int(krng.integers(10, 21)), 4, device="cuda", generator=g)
           for _ in range(3 * len(spec))]

    def mixed(arr):
        reqs, j = [], 0
        for i, a in enumerate(arr):
            if i % 4 == 0:
                S, v, t = spec[(i // 4) % len(spec)]
                reqs.append(Request(model="m", kind="render", view=v, t=t, W=S, H=S,
                                    arrival=float(a)))
            else:
                reqs.append(Request(model="m", kind="points", pos=pts[j], n=pts[j].shape[0],
                                    arrival=float(a)))
                j += 1
        return reqs

    def serve_mixed(arr, realtime, **kw):
        ex = GpuExecutor(sample_budget=C)
        ex.add_model("m", rm)
        free, _ = torch.cuda.mem_get_info()
        sch = Scheduler(ex, sample_budget=C, mem_budget=int(free * 0.8), **kw)
        torch.cuda.synchronize()
        done = sch.run(mixed(arr), realtime=realtime)
        return {"all": latency_stats(done),
                "render": latency_stats([r for r in done if r.kind == "render"]),
                "points": latency_stats([r for r in done if r.kind == "points"]),
                "iterations": sch.iterations, "samples": sch.samples}

    n_mix = 4 * len(spec)
    mix_sat = serve_mixed([0.0] * n_mix, realtime=False)
    mix_rate = 0.5 * mix_sat["all"]["requests_per_s"]
    arr = poisson_arrivals(mix_rate, n_mix, seed=5006)
    mix = {"saturation": mix_sat, "rate_per_s": mix_rate,
           "continuous_backfill": serve_mixed(arr, realtime=True),
           "one_at_a_time": serve_mixed(arr, realtime=True, max_active=1)}
    for name in ("continuous_backfill", "one_at_a_time"):
        m = mix[name]
        log(f"[serve] mixed {mix_rate:.2f}/s {name}: render p50 {m['render']['p50_ms']:.1f} "
            f"p99 {m['render']['p99_ms']:.1f} ms; points p50 {m['points']['p50_ms']:.1f} "
            f"p99 {m['points']['p99_ms']:.1f} ms")
    out = {
        "metric": "render p50/p99 ms at 0.25/0.5/0.9 x saturation (Poisson), rays/s at saturation",
        "value": sat["rays_per_s"], "unit": "rays/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None,
        "dtype": f"f16 tables, {args.serve_decoder} MLP", "data": "synthetic",
        "config": {"workload": f"render serving, {'x'.join(map(str, dims))} volume, 16 levels, "
                   "MLP 32-64-64-64-1, images {" + ",".join(f"{x}^2" for x in sizes) + "}",
                   "requests_per_rate": len(spec), "sample_budget": C,
                   "train_steps": args.serve_train_steps, "probe_psnr_db": psnr,
                   "params": model.n_params},
        "saturation": sat, "arm_off_saturation": arm_off, "one_at_a_time_saturation": sat_one,
        "rates": rates, "mixed_points_and_renders": mix,
    }
    print(json.dumps(out), flush=True)


def coreset_bench(args):
    """Feature-based coreset selection (Sec. 3.1) over the whole production
    volume: gradient-magnitude interval feature, dilation by 2, per-frame boxes
    and FBB, Morton occupancy grid, coreset ids.  Each call is timed with HIP
    events on the stream it runs on, over `--steps` repetitions."""
    import ctypes as C

    import numpy as np

    from oracle import coreset as OC
    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import synth, volume

    fl.lib()
    torch.cuda.set_device(0)
    dims = [int(x) for x in args.shape.split(",")]
    Sx, Sy, Sz, T = dims
    N = Sx * Sy * Sz * T
    gen = synth.production_field_gpu(dims, args.field_seed, keep_field=False)
    g, thr = gen.pop("grad"), gen["threshold"]
    words = fl.mask_words(dims) * 8
    feat = torch.empty(words // 8, dtype=torch.int64, device="cuda")
    dil = torch.empty_like(feat)
    occ = torch.empty(fl.fhash_occupancy_words(dims), dtype=torch.int64, device="cuda")
    box = torch.empty((T + 1, 6), dtype=torch.int32, device="cuda")
    calls = {
        "feature_mask": (lambda: fl.fhash_feature_mask(g, dims, fl.FEATURE_INTERVAL, thr,
                                                       float("inf"), feat), 4 * N + words),
        "dilate_r2": (lambda: fl.fhash_dilate_mask(feat, dims, 2, dil), 2 * words),
        "feature_boxes": (lambda: fl.fhash_feature_boxes(dil, dims, box), words),
        "occupancy_grid": (lambda: fl.fhash_occupancy_grid(dil, dims, occ), words + occ.numel() * 8),
    }
    out = {}
    for name, (fn, nbytes) in calls.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out[name] = {"ms": ms, "algorithmic_bytes": nbytes, "GB_s": nbytes / ms / 1e6,
                     "frac": nbytes / ms / 1e6 / 8000.0}
        log(f"[coreset] {name}: {ms:.3f} ms, {nbytes / ms / 1e6:.0f} GB/s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ids = fl.fhash_coreset(dil, dims)
    torch.cuda.synchronize()  # the last call's emit pass is still in flight
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    M = ids.numel()
    out["coreset_ids"] = {"ms": ms, "algorithmic_bytes": 2 * words + 8 * M,
                          "GB_s": (2 * words + 8 * M) / ms / 1e6, "note": "wall clock, 3 calls "
                          "(size query, count, emit) with two host synchronisations"}
    log(f"[coreset] coreset ids: {ms:.3f} ms ({M} voxels)")
    total_ms = sum(v["ms"] for v in out.values())
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on one timestep of the same volume (one thread of numpy)
        f1 = g[0].cpu().numpy()
        t0 = time.perf_counter()
        m1 = OC.dilate(OC.feature_interval(f1[None], thr, np.inf), 2)
        OC.feature_boxes(m1)
        OC.occupancy_grid(m1)
        OC.coreset_ids(m1)
        sec = time.perf_counter() - t0
        cpu = {"value": f1.size / sec, "unit": "voxels/s", "cores": 1, "kind": "oracle",
               "sample": f"one timestep ({f1.size} voxels) through the numpy oracle, {sec:.2f} s"}
    dom = out["feature_mask"]
    src = os.path.join(ROOT, "paper_2507_03836_amd", "csrc", "coreset.hip")
    same = (_kernel_md5(src, "classify4_kernel") == CLASSIFY_TRAFFIC["kernel_md5"]
            and dims == CLASSIFY_TRAFFIC["shape"] and Sx % 4 == 0)
    print(json.dumps({
        "metric": "coreset selection voxels/s (feature mask, dilation, boxes, occupancy, ids)",
        "value": N / (total_ms / 1e3), "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": total_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"coreset selection, {Sx}x{Sy}x{Sz}x{T} synthetic volume, "
                               "gradient-magnitude feature above its 80th percentile, "
                               "dilation by 2", "shape": dims, "coreset": M},
        "breakdown": out,
        "roofline": {"kernel": "classify4_kernel" if Sx % 4 == 0 else "classify_kernel",
                     "bound": "hbm", "achieved": dom["GB_s"],
                     "peak": 8000.0, "unit": "GB/s", "frac": dom["frac"],
                     "traffic": CLASSIFY_TRAFFIC["bytes"] if same else None,
                     "algorithmic_bytes": dom["algorithmic_bytes"], "kernel_ms": dom["ms"]},
        "cpu_baseline": cpu}))


LAYOUTS = {"rows": 0, "bricks": 1}


# ------------------------------------------------------------------ headline
HEADLINE_DIMS = [432, 432, 432, 60]
# Memory-side atomic requests per second of the chip on a footprint far beyond
# the caches (random 16-byte float-atomic groups over 24 GiB, the probe
# paper_2507_03836_amd/probe/random_access): the bound of the scatter-add.
ATOMIC_CEILING_GPS = 16.8
# HBM bytes of one fused training launch and its coarse-level LDS scatter
# (mixed path, 432^3 x 60, batch 2^20)
# from rocprofv3 FETCH_SIZE (x2.000) and WRITE_SIZE (x1.000) passes scaled by a
# plain streaming copy of known size; valid only while the kernel sources
# hashed in _fused_src_md5(), the optimiser state layout, the batch order, the
# table reads and the decoder type are those the counters were taken with.
FUSED_TRAFFIC = {"bytes": 20075089224, "raw_bytes": 11912743544, "moments": "with-params",
                 "sorted": True, "table_reads": "f32", "decoder": "f16", "coarse_lds": True,
                 "source_md5": "14b8d4d63f82b0e95aecefef307e9e53"}


def _fused_src_md5():
    import hashlib
    csrc = os.path.join(ROOT, "paper_2507_03836_amd", "csrc")
    names = ("fused_impl.h", "encode_dev.h", "mlp_dev.h", "mlp_train_dev.h", "common.h",
             "fused_train.hip", "fused_train16.hip", "coarse.hip")
    return hashlib.md5(b"".join(open(os.path.join(csrc, n), "rb").read()
                                for n in names)).hexdigest()


def _cpu_worker(task):
    """One process of the all-core CPU baseline: the FP64 oracle, as it
    stands, on its share of the sample draws (fwd+bwd) or on an Adam chunk."""
    import numpy as np

    import oracle as O
    kind = task[0]
    if kind == "fb":
        _, res, F, width, params, pos, tgt = task
        g = O.Grid(np.array(res), F, None)
        table = np.zeros((g.total_slots, F))  # zero pages, committed only where written
        t0 = time.perf_counter()
        enc, _ = O.encode_fwd(g, pos, table)
        y, acts, _ = O.mlp_fwd(width, params, enc)
        L, dy = O.mse(y[:, 0], tgt.astype(np.float64))
        dp, denc, _, _ = O.mlp_bwd(width, params, acts, dy.reshape(-1, 1), pos.shape[0])
        dt, _ = O.encode_bwd(g, pos, denc)
        return time.perf_counter() - t0
    _, n = task
    rng = np.random.default_rng(n)
    p, gr, m, v = np.zeros(n), rng.normal(size=n), np.zeros(n), np.zeros(n)
    t0 = time.perf_counter()
    O.adam(p, gr, m, v, 0.01, 0.9, 0.999, 1e-8, 1)
    return time.perf_counter() - t0


def _cpu_worker_init():
    """Worker start-up: no transparent huge pages in this process.  The oracle
    works on full-size zero tables and counts on pages being committed only
    where it writes; with huge pages each scattered write would commit 2 MiB."""
    import ctypes
    try:
        ctypes.CDLL(None, use_errno=True).prctl(41, 1, 0, 0, 0)  # PR_SET_THP_DISABLE
    except (OSError, AttributeError):
        pass


def cpu_baseline_all_cores(model, gen, dims, batch, n_cpu, seed):
    """The FP64 oracle, as it stands, on every host core the box gives this
    job (one process per core, at most 16): n_cpu coreset draws split over the
    processes through the oracle's encoding, decoder, MSE and backward with the
    same level structure (dense-box index, same 16 x 16 corner work per
    sample), and the oracle's Adam on one 2^21-parameter chunk per process.
    Scaled to one full step: wall time of the parallel fwd+bwd x batch/n_cpu +
    wall time of the parallel Adam x parameters / (processes x chunk)."""
    import multiprocessing as mp

    import numpy as np

    import oracle as O
    nproc = os.cpu_count() or 1
    workers = max(1, min(16, nproc))
    ids = O.sample_ids(seed, 1, n_cpu, gen["M"])
    ids_t = torch.from_numpy(ids.view(np.int64)).cuda()
    lin = gen["coreset"][ids_t].cpu().numpy().view(np.uint64)
    tgt = gen["field"].view(-1)[torch.from_numpy(lin.view(np.int64)).cuda()].cpu().numpy()
    pos = O.voxel_positions(lin, dims)
    cfg = model.cfg
    params = model.mlp_params.double().cpu().numpy()
    chunks = np.array_split(np.arange(n_cpu), workers)
    fb = [("fb", cfg.res, cfg.n_features, cfg.width, params, pos[c], tgt[c]) for c in chunks]
    chunk = 1 << 21
    cpu_model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ctx = mp.get_context("spawn")
    log(f"[cpu] oracle on {workers} processes ({nproc} host CPUs, {cpu_model})")
    with ctx.Pool(workers, initializer=_cpu_worker_init) as pool:
        pool.map(_cpu_worker, [("adam", 1024)] * workers)  # start-up outside the timing
        t0 = time.perf_counter()
        pool.map(_cpu_worker, fb)
        t_fb = time.perf_counter() - t0
        log(f"[cpu] fwd+bwd of {n_cpu} draws: {t_fb:.2f} s")
        t0 = time.perf_counter()
        pool.map(_cpu_worker, [("adam", chunk)] * workers)
        t_adam = time.perf_counter() - t0
        log(f"[cpu] Adam on {workers} x {chunk} parameters: {t_adam:.3f} s")
    t_step = t_fb * batch / n_cpu + t_adam * model.n_params / (workers * chunk)
    return {"value": batch / t_step, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "nproc": nproc, "cpu_model": cpu_model,
            "sample": (f"{n_cpu} coreset draws fwd+bwd over {workers} processes ({t_fb:.2f} s "
                       f"wall) scaled to {batch}, + Adam on {workers} x {chunk} params "
                       f"({t_adam:.3f} s wall) scaled to {model.n_params}; dense-box index, "
                       "FP64, one process per core")}


def _train_timed(model, gen, dims, B, steps, warmup, sampler_seed, pos, tgt, sort=True,
                 sort_reduce=False):
    """warmup + steps training steps; per-phase HIP events on the launch stream
    over the timed steps; the timed region ends with the deferred update
    flushed.  sort: each batch is put in 4D Morton order (fhash_sort_samples)
    after it is drawn.  Returns the breakdown and the step closure."""
    import numpy as np

    from paper_2507_03836_amd import _lib as fl
    stream = torch.cuda.current_stream()
    coreset, M, field = gen["coreset"], gen["M"], gen["field"]
    sort_ws = [None]

    def step(k, ev=None):
        fl.fhash_sample(sampler_seed, k, B, coreset, M, dims, field, pos, tgt)
        if sort:
            sort_ws[0] = fl.fhash_sort_samples(pos, tgt, B, sort_ws[0])
        if ev is not None:
            ev[0].record(stream)
        model.prepare(pos, fl.LAZY_MARK)
        if ev is not None:
            ev[1].record(stream)
        model.prepare(pos, fl.LAZY_CATCH_UP)
        if ev is not None:
            ev[2].record(stream)
        model.fwd_bwd(pos, tgt, prepared=True, sorted_batch=sort and sort_reduce)
        if ev is not None:
            ev[3].record(stream)
        model.optimizer_step()
        if ev is not None:
            ev[4].record(stream)

    t_first = time.perf_counter()
    for k in range(warmup):
        step(k + 1)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    fev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    st0 = fl.fhash_lazy_stats(model.lazy)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(warmup + k + 1, evs[k])
    st1 = fl.fhash_lazy_stats(model.lazy)
    fev[0].record(stream)
    model.flush()
    fev[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mean = lambda i, j: float(np.mean([e[i].elapsed_time(e[j]) for e in evs]))
    out = {"ms_per_step": wall * 1e3 / steps, "samples_per_s": B / (wall / steps),
           "breakdown_ms": {"lazy_mark": mean(0, 1), "lazy_catch_up": mean(1, 2),
                            "fused_fwd_bwd": mean(2, 3), "adam_dense_part": mean(3, 4),
                            "final_flush_per_step": fev[0].elapsed_time(fev[1]) / steps},
           "lazy_per_step": {k: (st1[k] - st0[k]) / steps for k in st1},
           "mean_loss": model.loss_sum.item() / (B * (warmup + steps))}
    out["breakdown_ms"]["sampler_sort_and_other" if sort else "sampler_and_other"] = (
        out["ms_per_step"] - sum(out["breakdown_ms"].values()))
    return out, step, t_first


def _to_psnr(model, step, k_done, t_first, ppos, ptgt, target, eval_every, max_steps):
    """Train on until the probe PSNR reaches the target: evaluated every
    eval_every steps, and after every step once it is within 1 dB of the
    target, so that the step count is exact."""
    from paper_2507_03836_amd.model import psnr_on
    k, hist, reached, near = k_done, [], None, False
    while True:
        if near or (k - k_done) % eval_every == 0 or k >= max_steps:
            ps = psnr_on(model, ppos, ptgt)
            el = time.perf_counter() - t_first
            hist.append((k, round(el, 3), round(ps, 3)))
            log(f"[headline] step {k}: probe PSNR {ps:.3f} dB at {el:.2f} s")
            if ps >= target:
                reached = (k, el, ps)
                break
            if k >= max_steps:
                break
            near = ps >= target - 1.0
        k += 1
        step(k)
    return {"target_db": target, "reached": reached is not None,
            "steps": reached[0] if reached else None,
            "seconds": reached[1] if reached else None,
            "final_psnr_db": hist[-1][2], "history": hist}


def coarse_levels(res, n):
    """Levels that FHASH_COARSE_LDS sends through the LDS scatter: from the
    coarsest on, those with at most one cell per sample of the batch."""
    lc = 0
    for r in res:
        if (r[0] - 1) * (r[1] - 1) * (r[2] - 1) * (r[3] - 1) > n:
            break
        lc += 1
    return lc


def compulsory_lines(model, pos, line=128):
    """Distinct `line`-byte lines of directory, table and table gradient that
    the fused training kernel must move for this batch (the corners of every
    sample at every level, fhash_corner_rows), in bytes: directory and table
    lines are read once, gradient lines read and written once; plus 20 bytes
    of sample I/O per sample.  With the moments stored beside the parameters,
    a 16-float segment's parameters (FP32 path) and its gradient each take a
    128-byte line of their own (the other half holds m or v): 8 bytes of line
    address per value."""
    from paper_2507_03836_amd import _lib as fl
    n = pos.shape[0]
    F = model.cfg.n_features
    runs = getattr(model, "moments_with_params", False)
    tb = 2 if model.shadow is not None else (8 if runs else 4)
    gb = 8 if runs else 4
    dir_lines, tab_lines, grad_lines = [], [], []
    requests = {}
    for s in range(0, n, 1 << 16):
        e = min(n, s + (1 << 16))
        d, sl = fl.fhash_corner_rows(model.index, pos[s:e], e - s)
        d = d.view(-1)
        d = d[d >= 0]
        dir_lines.append(torch.unique(d * 16 // line))
        # the scatter-add's atomic requests, per level: as issued, and as they would
        # be if equal slots of a block were summed first (whole blocks on one slot,
        # or every run of neighbours on one slot)
        c = sl
        pad = (-(e - s)) % 16
        if pad:
            c = torch.cat([c, torch.full((pad,) + tuple(c.shape[1:]), -1, dtype=c.dtype,
                                         device=c.device)])
        c = c.view(-1, 16, c.shape[1], 8, 2).permute(0, 2, 3, 1, 4)  # block, level, pair, i, e
        for name, v in (("issued", c), ("uniform", _merge_uniform(c)), ("runs", _merge_runs(c))):
            per_level = _atomic_requests(v, F)
            requests[name] = per_level if name not in requests else requests[name] + per_level
        del c
        sl = sl.view(-1)
        sl = sl[sl >= 0]
        tab_lines.append(torch.unique(sl * (F * tb) // line))
        grad_lines.append(torch.unique(sl * (F * gb) // line))
        del d, sl
    u = lambda xs: int(torch.unique(torch.cat(xs)).numel())
    nd, nt, ng = u(dir_lines), u(tab_lines), u(grad_lines)
    return {"line_bytes": line, "directory_lines": nd, "table_lines": nt, "gradient_lines": ng,
            "bytes": line * (nd + nt + 2 * ng) + 20 * n,
            "atomic_requests": int(requests["issued"].sum()),
            "atomic_requests_per_level": requests["issued"].tolist(),
            "atomic_requests_if_summed": {k: requests[k].tolist() for k in ("uniform", "runs")}}


def _atomic_requests(c, F):
    """Memory-side atomic requests of the scatter-add, per level.  c: slots
    (block, level, pair, sample, pair element), -1 for none.  One scatter
    instruction covers one corner pair of one level for the 16 samples of a
    block; lanes that add into distinct floats of one 64-byte chunk share a
    request, lanes that add into the same float cannot, so a chunk costs as
    many requests as the most samples on one of its rows."""
    nb, L = c.shape[0], c.shape[1]
    v = c.reshape(-1, 32)
    big = int(v.max()) + 2
    gid = torch.arange(v.shape[0], device=v.device, dtype=torch.int64)[:, None]
    key = (gid * big + v)[v >= 0]
    key, _ = torch.sort(key)
    key, cnt = torch.unique_consecutive(key, return_counts=True)
    chunk = (key // big) * big + (key % big) * F // 16
    chunk, inv = torch.unique_consecutive(chunk, return_inverse=True)
    most = torch.zeros(chunk.numel(), dtype=cnt.dtype, device=cnt.device)
    most.scatter_reduce_(0, inv, cnt, "amax")
    level = (chunk // big) // 8 % L
    out = torch.zeros(L, dtype=torch.int64, device=c.device)
    out.scatter_add_(0, level, most)
    return out.cpu()


def _merge_uniform(c):
    """c with every (block, level, pair) whose 16 samples share one pair of
    slots reduced to its first sample."""
    same = ((c == c[:, :, :, :1, :]) | (c < 0)).all(dim=4).all(dim=3, keepdim=True)
    keep = torch.zeros_like(c, dtype=torch.bool)
    keep[:, :, :, 0, :] = True
    return torch.where(same.unsqueeze(4) & ~keep, torch.full_like(c, -1), c)


def _merge_runs(c):
    """c with every run of neighbouring samples on one slot reduced to its
    last sample (a segmented sum over the block's 16 samples)."""
    tail = torch.ones_like(c, dtype=torch.bool)
    tail[:, :, :, :-1, :] = c[:, :, :, :-1, :] != c[:, :, :, 1:, :]
    return torch.where(tail, c, torch.full_like(c, -1))


def _serve_sub(model, table16, mlp_params, gen, dims, args, n_req):
    """Render p50/p99 of the trained mixed model (FP16 tables, its 16-bit
    decoder) at saturation and three Poisson rates: continuous batching
    (backfill) against one request at a time, same arrivals."""
    import numpy as np

    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import synth
    from paper_2507_03836_amd.serving import (GpuExecutor, Request, ResidentModel, Scheduler,
                                              latency_stats, poisson_arrivals)
    tf = torch.from_numpy(synth.transfer_function()).cuda()
    rm = ResidentModel(index=model.index, mlp=model.mlp, table=table16,
                       params=mlp_params, mask_bits=gen["bits"], dims=dims, tf=tf,
                       keep=(model._dir,), occ=fl.fhash_occupancy_grid(gen["bits"], dims))
    C = 1 << 22
    rng = np.random.default_rng(5004)
    spec = []
    for i in range(n_req):
        S = int(rng.choice([256, 512, 1024]))
        spec.append((S, synth.orbit_view(dims, float(rng.uniform(0, 2 * np.pi)),
                                         float(rng.uniform(-np.pi / 3, np.pi / 3)), S, S),
                     float(rng.uniform(0, dims[3] - 1))))

    def reqs(arr):
        return [Request(model="m", kind="render", view=v, t=t, W=S, H=S, arrival=float(a))
                for (S, v, t), a in zip(spec, arr)]

    def serve(arr, realtime, **kw):
        ex = GpuExecutor(sample_budget=C)
        ex.add_model("m", rm)
        free, _ = torch.cuda.mem_get_info()
        sch = Scheduler(ex, sample_budget=C, mem_budget=int(free * 0.8), **kw)
        torch.cuda.synchronize()
        return latency_stats(sch.run(reqs(arr), realtime=realtime))

    serve([0.0] * 2, realtime=False)
    sat = serve([0.0] * n_req, realtime=False)
    sat_one = serve([0.0] * n_req, realtime=False, max_active=1)
    rates = []
    for frac in (0.25, 0.5, 0.9):
        rate = frac * sat["requests_per_s"]
        arr = poisson_arrivals(rate, n_req, seed=5004)
        row = {"rate_frac": frac, "rate_per_s": rate,
               "continuous_backfill": serve(arr, realtime=True),
               "one_at_a_time": serve(arr, realtime=True, max_active=1)}
        log(f"[headline] render {rate:.1f}/s: batched p50 "
            f"{row['continuous_backfill']['p50_ms']:.1f} p99 "
            f"{row['continuous_backfill']['p99_ms']:.1f} ms; one at a time p50 "
            f"{row['one_at_a_time']['p50_ms']:.1f} p99 {row['one_at_a_time']['p99_ms']:.1f} ms")
        rates.append(row)
    return {"workload": "render requests of side 256/512/1024 (uniform), t ~ U[0, 59], orbit "
                        "cameras, ds = 1/2 voxel, ARM max 64, alpha stop 0.99, FP16 tables, "
                        f"{model.decoder} decoder", "requests_per_rate": n_req,
            "sample_budget": C, "saturation": sat, "one_at_a_time_saturation": sat_one,
            "rates": rates}


def copy_calibration():
    """A plain streaming copy kernel of known size (4 GiB read + 4 GiB
    written): an elementwise x*1, so that it runs as a kernel rather than a DMA
    transfer.  Its FETCH_SIZE / WRITE_SIZE readings give the counters' scale."""
    src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def headline_bench(args):
    import numpy as np

    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import volume
    from paper_2507_03836_amd.model import FHashConfig, FHashModel, geometric_resolutions

    fl.lib()
    torch.cuda.set_device(0)
    dims = HEADLINE_DIMS
    B = 1 << 20
    t0 = time.time()
    gen = volume.production_volume(dims, seed=1003)
    log(f"[headline] volume {dims} in {time.time() - t0:.1f} s; coreset {gen['M']} of "
        f"{gen['N']} voxels")
    res = geometric_resolutions(16, 16, 512, 4, dims[3], dims)
    cfg = FHashConfig(res=res, n_features=2, hidden=64, n_hidden=3,
                      layout=LAYOUTS[args.layout])
    P = 1 << 22
    ppos = torch.empty(P, 4, device="cuda")
    ptgt = torch.empty(P, device="cuda")
    fl.fhash_sample(4003, 1, P, gen["coreset"], gen["M"], dims, gen["field"], ppos, ptgt)
    pos = torch.empty(B, 4, device="cuda")
    tgt = torch.empty(B, device="cuda")
    # load every kernel of both paths once (code-object loading and first-launch
    # costs stay out of both paths' timings)
    for prec in ("fp32", "mixed"):
        small = FHashModel(FHashConfig(res=[[4, 4, 4, 2]] * 16, n_features=2, hidden=64,
                                       n_hidden=3), None, dims, precision=prec, lazy=True,
                           **_layout_kw(args), max_steps=4, **_reads_kw(args, prec))
        fl.fhash_sample(1, 1, 4096, gen["coreset"], gen["M"], dims, gen["field"], pos, tgt)
        if args.sort:
            fl.fhash_sort_samples(pos, tgt, 4096)
        small.prepare(pos[:4096])
        small.fwd_bwd(pos[:4096], tgt[:4096], prepared=True)
        small.optimizer_step()
        small.flush()
        small.forward(pos[:4096])
        del small
    torch.cuda.synchronize()
    if args.calibrate_copy:
        copy_calibration()
    paths, keep, cpu = {}, None, None
    for prec in args.paths.split(","):
        model = FHashModel(cfg, gen["bits"], dims, init_seed=3003, precision=prec, lazy=True,
                           **_layout_kw(args), **_reads_kw(args, prec),
                           max_steps=args.max_steps + args.warmup + args.steps + 8)
        model.coarse_lds = args.coarse_lds
        r, step, t_first = _train_timed(model, gen, dims, B, args.steps, args.warmup, 2003, pos,
                                        tgt, sort=args.sort, sort_reduce=args.sort_reduce)
        log(f"[headline] {prec}: {r['ms_per_step']:.2f} ms/step ({r['samples_per_s'] / 1e6:.1f}"
            f" M samples/s): {r['breakdown_ms']}")
        r["time_to_psnr"] = _to_psnr(model, step, args.warmup + args.steps, t_first, ppos, ptgt,
                                     args.psnr_target or 40.0, args.eval_every, args.max_steps)
        # the timed batch's compulsory lines (the batch of the last timed step, in
        # the order it was trained in; drawn again, after the clock of the PSNR run)
        fl.fhash_sample(2003, args.warmup + args.steps, B, gen["coreset"], gen["M"], dims,
                        gen["field"], pos, tgt)
        if args.sort:
            fl.fhash_sort_samples(pos, tgt, B)
        r["compulsory"] = compulsory_lines(model, pos)
        r["params"] = model.n_params
        r["decoder"] = model.decoder
        r["table_reads"] = "f16" if model.shadow is not None else "f32"
        if prec == "mixed":
            r["loss_scale"] = model.loss_scale
            r["skipped_steps"] = model.skipped
        paths[prec] = r
        model.flush()
        if prec == "mixed":
            # what serving keeps of the trained mixed model: its FP16 table (the
            # flushed master rounded to FP16) and decoder; the rest is freed
            if model.shadow is not None:
                table16 = model.shadow[: model.n_table]
            else:
                table16 = torch.empty(model.n_table, dtype=torch.float16, device="cuda")
                fl.fhash_cast(model.table, table16)
            keep = (model, table16, model.mlp_params.clone())
        elif not args.no_cpu_baseline:
            try:
                cpu = cpu_baseline_all_cores(model, gen, dims, B, args.cpu_samples, 2003)
            except Exception as e:  # reported, never hidden
                cpu = {"error": repr(e)}
        model.params = model.grads = model.m = model.v = None
        model.mv = model.pm = model.gv = model.lazy = None
        model.mlp_p = model.mlp_g = model.mlp_m = model.mlp_v = None
        del model
        # the freed blocks stay in torch's cache, and the next path's state
        # arrays of the same sizes reuse them: state allocated afresh after
        # returning them to the driver made the catch-up's scattered segment
        # transactions about 0.5 ms slower per step (4.66 against 5.19 ms)

    serve = _serve_sub(*keep, gen, dims, args, args.serve_requests)
    mx, fp = paths["mixed"], paths["fp32"]
    fused_ms = mx["breakdown_ms"]["fused_fwd_bwd"]
    reads16 = mx["table_reads"] == "f16"
    # FP16 (FP32) gather 1024 (2048) + FP32 scatter read-modify-write 2048 + 20 B I/O
    alg = (3092 if reads16 else 4116) * B
    comp = mx["compulsory"]["bytes"]
    # with FHASH_COARSE_LDS the fused kernel issues the requests of the levels
    # with more than one cell per sample only; the coarse levels' requests are
    # replaced by one per touched vertex row segment of a chunk's LDS box
    # (the library takes the LDS path on row-ordered indexes only)
    lc = coarse_levels(cfg.res, B) if args.coarse_lds and args.layout == "rows" else 0
    areq = int(sum(mx["compulsory"]["atomic_requests_per_level"][lc:]))
    same = (FUSED_TRAFFIC["source_md5"] == _fused_src_md5() and
            args.coarse_lds == FUSED_TRAFFIC["coarse_lds"] and
            mx["table_reads"] == FUSED_TRAFFIC["table_reads"] and
            mx["decoder"] == FUSED_TRAFFIC["decoder"] and
            args.moments == FUSED_TRAFFIC["moments"] and args.sort == FUSED_TRAFFIC["sorted"])
    roof = {"kernel": "fused_kernel<TRAIN, F=2, " + ("FP16" if reads16 else "FP32")
                      + " table, 32-64-64-64-1, " + mx["decoder"].upper() + " decoder>"
                      + (f" + coarse_scatter_kernel (levels 0-{lc - 1})" if lc else ""),
            "bound": "hbm", "achieved": alg / (fused_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": alg / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": FUSED_TRAFFIC["bytes"] if same else None,
            "algorithmic_bytes": alg, "kernel_ms": fused_ms,
            "compulsory_bytes": comp,
            "compulsory_GB_s": comp / (fused_ms * 1e-3) / 1e9,
            "compulsory_frac": comp / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "compulsory_detail": mx["compulsory"],
            # what bounds the kernel: the scatter's memory-side atomic requests
            "coarse_lds_levels": lc,
            "atomic_requests": areq, "atomic_G_per_s": areq / (fused_ms * 1e-3) / 1e9,
            "atomic_ceiling_G_per_s": ATOMIC_CEILING_GPS,
            "atomic_frac": areq / (fused_ms * 1e-3) / 1e9 / ATOMIC_CEILING_GPS}
    ttp_m, ttp_f = mx["time_to_psnr"], fp["time_to_psnr"]
    out = {
        "metric": "train samples/s fwd+bwd (FP32 vs FP16/BF16) at equal PSNR; render p50/p99 ms",
        "value": mx["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mx["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": mx["decoder"] + " decoder MFMA, " + mx["table_reads"]
                 + " table reads, f32 master/Adam/accumulation",
        "data": "synthetic",
        "config": {"workload": "F-Hash differentiated mixed-precision training, 432x432x432x60 "
                               "synthetic volume, 16 levels x 2 features, MLP 32-64-64-64-1, "
                               "batch 2^20 coreset draws, Adam with deferred large-level "
                               "updates (equal to the dense update bit for bit)",
                   "shape": dims, "levels": 16, "batch": B, "params": mx["params"],
                   "coreset": gen["M"], "slot_order": args.layout},
        "paths": {"mixed": mx, "fp32": fp},
        "mixed_over_fp32_samples_per_s": mx["samples_per_s"] / fp["samples_per_s"],
        "equal_psnr": {"target_db": ttp_m["target_db"],
                       "mixed_s": ttp_m["seconds"], "fp32_s": ttp_f["seconds"],
                       "mixed_steps": ttp_m["steps"], "fp32_steps": ttp_f["steps"]},
        "render": serve,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: multi-GPU runs are not supported (the path "
                          "would shard by slabs of the fine levels)"}))
        sys.exit(2)
    global torch
    import numpy as np
    import torch

    if args.serve_multi:
        return serve_multi_bench(args)
    if args.fold_sweep:
        return fold_sweep_bench(args)
    if (args.workload == "headline" and args.key_frames <= 1 and not args.serve and
            not args.coreset):
        return headline_bench(args)
    if args.key_frames > 1:
        return key_frame_bench(args)
    if args.serve:
        return serve_bench(args)
    if args.coreset:
        return coreset_bench(args)

    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import synth, volume
    from paper_2507_03836_amd.model import FHashConfig, FHashModel, geometric_resolutions

    fl.lib()
    torch.cuda.set_device(0)
    dims = [int(x) for x in args.shape.split(",")]
    t0 = time.time()
    gen = volume.production_volume(dims, seed=args.field_seed)
    log(f"[bench] volume {dims} generated in {time.time() - t0:.1f} s; coreset {gen['M']} "
        f"of {gen['N']} voxels ({gen['M'] / gen['N']:.3f}), threshold {gen['threshold']:.4g}")
    res = geometric_resolutions(args.levels, 16, 512, 4, dims[3], dims)
    cfg = FHashConfig(res=res, n_features=2, hidden=64, n_hidden=args.hidden_layers,
                      layout=LAYOUTS[args.layout])
    t0 = time.time()
    model = FHashModel(cfg, None if args.dense_index else gen["bits"], dims,
                       hash_bits=args.hash_bits, init_seed=3000 + args.field_seed - 1000,
                       precision=args.precision, track_touched=args.optimizer == "tracked",
                       **_reads_kw(args, args.precision),
                       lazy=args.optimizer == "lazy",
                       **_layout_kw(args, args.optimizer == "lazy"),
                       max_steps=max(args.max_steps, args.warmup + args.steps) + 64)
    model.coarse_lds = args.coarse_lds
    torch.cuda.synchronize()
    dense = sum(int(np.prod(r)) for r in res)
    log(f"[bench] index built in {time.time() - t0:.1f} s: {model.rows} active vertices of "
        f"{dense} ({model.rows / dense:.3f}); params {model.n_params}")
    if args.calibrate_copy:
        copy_calibration()
    B = args.batch
    pos = torch.empty(B, 4, device="cuda")
    tgt = torch.empty(B, device="cuda")
    coreset, M, field = gen["coreset"], gen["M"], gen["field"]
    stream = torch.cuda.current_stream()

    sort_ws = [None]

    def step(k, ev=None):
        fl.fhash_sample(args.sampler_seed, k, B, coreset, M, dims, field, pos, tgt)
        if args.sort:
            sort_ws[0] = fl.fhash_sort_samples(pos, tgt, B, sort_ws[0])
        if ev is not None:
            ev[0].record(stream)
        model.prepare(pos, fl.LAZY_MARK)
        if ev is not None:
            ev[1].record(stream)
        model.prepare(pos, fl.LAZY_CATCH_UP)
        if ev is not None:
            ev[2].record(stream)
        model.fwd_bwd(pos, tgt, sorted_batch=args.sort and args.sort_reduce, prepared=True)
        if ev is not None:
            ev[3].record(stream)
        model.optimizer_step()
        if ev is not None:
            ev[4].record(stream)

    t_train0 = time.perf_counter()
    for k in range(args.warmup):
        step(k + 1)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    fev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    lazy = model.lazy is not None
    st0 = fl.fhash_lazy_stats(model.lazy) if lazy else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k + 1, evs[k])
    # deferred Adam: the timed work ends with every parameter up to date
    st1 = fl.fhash_lazy_stats(model.lazy) if lazy else None  # the steps' catch-ups only
    fev[0].record(stream)
    model.flush()
    fev[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mark_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    catch_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    prep_ms = mark_ms + catch_ms
    fb_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    adam_ms = float(np.mean([e[3].elapsed_time(e[4]) for e in evs]))
    flush_ms = fev[0].elapsed_time(fev[1])
    loss = model.loss_sum.item() / (B * (args.warmup + args.steps))
    ms = wall * 1e3 / args.steps
    mixed = args.precision == "mixed"
    shadow = model.shadow is not None
    P = model.n_params
    k_done = args.warmup + args.steps
    per = ADAM_RW_BYTES_PER_PARAM + (2 if shadow else 0)
    flagged = None
    if model.touch is None:
        adam_bytes = (per + 4) * P
    else:
        # one more step outside the timed region, to count the flagged segments
        k_done += 1
        fl.fhash_sample(args.sampler_seed, k_done, B, coreset, M, dims, field, pos, tgt)
        if args.sort:
            sort_ws[0] = fl.fhash_sort_samples(pos, tgt, B, sort_ws[0])
        model.fwd_bwd(pos, tgt, sorted_batch=args.sort and args.sort_reduce)
        flagged = int((model._touch_flags != 0).sum().item())
        model.optimizer_step()
        T = model.touch.end - model.touch.begin
        adam_bytes = per * P + 4 * (P - T) + 4 * fl.TOUCH_FLOATS * flagged + T // fl.TOUCH_FLOATS
    achieved = adam_bytes / (adam_ms * 1e-3) / 1e9
    roof_kernel, roof_ms, roof_bytes, extra = "adam_kernel", adam_ms, adam_bytes, {}
    if lazy:
        # dominant kernel: the catch-up of the deferred update (one launch per step)
        d = {k: (st1[k] - st0[k]) / args.steps for k in st1}
        nseg = (model.lazy.desc.end - model.lazy.desc.begin + 15) // 16
        roof_bytes = (nseg + LAZY_ENTRY_BYTES * d["segments"]
                      + LAZY_LOADED_BYTES * d["loaded"] + LAZY_PENDING_BYTES * d["pending"]
                      + (LAZY_SHADOW_BYTES * d["loaded"] if shadow else 0))
        roof_kernel, roof_ms = "lazy_catchup_kernel", catch_ms
        achieved = roof_bytes / (roof_ms * 1e-3) / 1e9
        extra = {"segments_per_launch": d["segments"], "loaded_per_launch": d["loaded"],
                 "pending_per_launch": d["pending"],
                 "replayed_param_steps_per_launch": 16 * d["segment_steps"]}
        flagged = None
    import hashlib
    src = os.path.join(ROOT, "paper_2507_03836_amd", "csrc", "optim.hip")
    same_src = hashlib.md5(open(src, "rb").read()).hexdigest() == ADAM_TRAFFIC["source_md5"]
    # (the order of the samples within a batch changes neither the parameters nor the
    # segments the update touches)
    traffic = ADAM_TRAFFIC["bytes"] if (same_src and not mixed and model.touch is not None and
                                        args.moments == ADAM_TRAFFIC["moments"] and
                                        model.n_params == ADAM_TRAFFIC["params"]) else None
    if lazy:
        srcs = [os.path.join(ROOT, "paper_2507_03836_amd", "csrc", f)
                for f in ("lazy.hip", "adam_dev.h")]
        md5 = hashlib.md5(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()
        same = (md5 == CATCHUP_TRAFFIC["source_md5"] and not mixed and
                args.moments == CATCHUP_TRAFFIC["moments"] and
                model.n_params == CATCHUP_TRAFFIC["params"] and
                args.steps == CATCHUP_TRAFFIC["steps"] and B == CATCHUP_TRAFFIC["batch"])
        traffic = CATCHUP_TRAFFIC["bytes"] if same else None
    log(f"[bench] step {ms:.3f} ms: mark {mark_ms:.3f} ms, catch-up {catch_ms:.3f} ms, "
        f"fused fwd+bwd {fb_ms:.3f} ms, "
        f"adam {adam_ms:.3f} ms, final flush {flush_ms:.3f} ms; mean loss {loss:.4g}")
    out = {
        "metric": ("train samples/s fwd+bwd (" + (("FP16" if shadow else "FP32")
                                                  + " table reads, " + model.decoder.upper()
                                                  + " decoder, FP32 master"
                                                  if mixed else "FP32 path")
                   + "), whole training step incl. Adam over every parameter"),
        "value": B / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": (("f16" if shadow else "f32") + " table reads, " + model.decoder
                  + " decoder MFMA, f32 master" if mixed else "f32"),
        "data": "synthetic",
        "config": {"workload": (f"F-Hash training, {'x'.join(map(str, dims))} synthetic volume, "
                                f"{args.levels} levels x 2 features, MLP "
                                + "-".join(map(str, cfg.width))
                                + f", batch 2^{int(np.log2(B))} coreset draws"
                                + (", Morton-sorted batches" if args.sort else "")
                                + (" with equal slots merged before the atomics" if args.sort and
                                   args.sort_reduce else "")
                                + (", dense index (every box vertex)" if args.dense_index
                                   else "")
                                + (f", spatial-hash index (2^{args.hash_bits} rows per large "
                                   "level)" if args.hash_bits else "")),
                   "shape": dims, "levels": args.levels, "batch": B,
                   "active_vertices": model.rows, "params": model.n_params,
                   "coreset": M, "slot_order": args.layout},
        "breakdown_ms": {"lazy_mark": mark_ms, "lazy_catch_up": catch_ms,
                         "fused_fwd_bwd": fb_ms, "adam": adam_ms,
                         "final_flush_per_step": flush_ms / args.steps,
                         ("sampler_sort_and_other" if args.sort else "sampler_and_other"):
                         ms - fb_ms - adam_ms - prep_ms - flush_ms / args.steps},
        "optimizer": args.optimizer,
        # deferred Adam: catch-up and mark time of single timed steps, by step number
        "lazy_by_step": [{"step": args.warmup + k + 1,
                          "catch_up_ms": evs[k][1].elapsed_time(evs[k][2]),
                          "mark_ms": evs[k][0].elapsed_time(evs[k][1]),
                          "fused_ms": evs[k][2].elapsed_time(evs[k][3])}
                         for k in sorted({0, 1, 4, 9, 19, 49, 99, 199, 499, 999, 1499, 1999,
                                          args.steps - 1}) if 0 <= k < args.steps]
        if lazy else None,
        "flush_ms": flush_ms,
        "roofline": {"kernel": roof_kernel, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes": roof_bytes,
                     "kernel_ms": roof_ms, "flagged_segments": flagged, **extra},
    }
    if mixed:
        out["loss_scale"] = model.loss_scale
        out["skipped_steps"] = model.skipped
    if args.psnr_target > 0:
        out["time_to_psnr"] = time_to_psnr(args, model, step, gen, dims, t_train0, k_done)
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(model, gen, dims, B, args.cpu_samples, 2002)
        except Exception as e:  # reported, never hidden
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
