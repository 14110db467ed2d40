#!/usr/bin/env python3
"""Training-throughput benchmark of the F-Hash hot path on one MI355X.

Workload (the production-shape training configuration): a seeded synthetic
480 x 720 x 120 x 100 float32 volume (64 advected Gaussian blobs + 3-octave
value-noise turbulence, min-max normalised), feature mask |grad| > 80th
percentile dilated by 2, coreset = masked voxels; 16 levels (spatial 16..512,
temporal 4..100, geometric, clamped to the volume), 2 features per level,
decoder 32 -> 64 -> 64 -> 1, batch 2^18 coreset draws per step.

One step = sampler (Philox draw from the coreset, positions, labels) ->
fused encoding + decoder forward, MSE, backward (scatter-add into the tables,
decoder gradients) -> dense Adam over every parameter.  Inputs are resident in
HBM before timing starts.  Prints ONE JSON line on stdout.
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
ADAM_BYTES_PER_PARAM = 28  # read p, g, m, v; write p, m, v (gradient reset not counted)
# HBM bytes of one adam_kernel launch at the default workload, from rocprofv3 FETCH_SIZE
# (x2.000) and WRITE_SIZE (x1.000) passes, scaled by a plain streaming copy of known size;
# valid only for the parameter count and the optimizer source they were taken on.
ADAM_TRAFFIC = {"bytes": 179.33e9, "params": 6390343593,
                "source_md5": "24b6c98a519b406c345b253a42521331"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1 << 18)
    ap.add_argument("--shape", type=str, default="480,720,120,100")
    ap.add_argument("--levels", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1 << 12)
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part "
                          "of it (see DESIGN.md for how the path would shard)"}))
        sys.exit(2)
    global torch
    import numpy as np
    import torch

    from paper_2507_03836_amd import _lib as fl
    from paper_2507_03836_amd import synth
    from paper_2507_03836_amd.model import FHashConfig, FHashModel, geometric_resolutions

    fl.lib()
    torch.cuda.set_device(0)
    dims = [int(x) for x in args.shape.split(",")]
    t0 = time.time()
    gen = synth.production_volume_gpu(dims, seed=1002)
    log(f"[bench] volume {dims} generated in {time.time() - t0:.1f} s; coreset {gen['M']} "
        f"of {gen['N']} voxels ({gen['M'] / gen['N']:.3f}), threshold {gen['threshold']:.4g}")
    res = geometric_resolutions(args.levels, 16, 512, 4, 100, dims)
    cfg = FHashConfig(res=res, n_features=2, hidden=64, n_hidden=2)
    t0 = time.time()
    model = FHashModel(cfg, gen["bits"], dims)
    torch.cuda.synchronize()
    dense = sum(int(np.prod(r)) for r in res)
    log(f"[bench] index built in {time.time() - t0:.1f} s: {model.rows} active vertices of "
        f"{dense} ({model.rows / dense:.3f}); params {model.n_params}")
    if args.calibrate_copy:
        # a plain streaming copy kernel of known size (4 GiB read + 4 GiB written);
        # an elementwise x*1 so that it runs as a kernel rather than a DMA transfer
        src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    B = args.batch
    pos = torch.empty(B, 4, device="cuda")
    tgt = torch.empty(B, device="cuda")
    coreset, M, field = gen["coreset"], gen["M"], gen["field"]
    stream = torch.cuda.current_stream()

    def step(k, ev=None):
        fl.fhash_sample(2002, k, B, coreset, M, dims, field, pos, tgt)
        if ev is not None:
            ev[0].record(stream)
        model.fwd_bwd(pos, tgt)
        if ev is not None:
            ev[1].record(stream)
        model.optimizer_step()
        if ev is not None:
            ev[2].record(stream)

    for k in range(args.warmup):
        step(k + 1)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k + 1, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fb_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    adam_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    loss = model.loss_sum.item() / (B * (args.warmup + args.steps))
    ms = wall * 1e3 / args.steps
    adam_bytes = ADAM_BYTES_PER_PARAM * model.n_params
    achieved = adam_bytes / (adam_ms * 1e-3) / 1e9
    import hashlib
    src = os.path.join(ROOT, "paper_2507_03836_amd", "csrc", "optim.hip")
    same_src = hashlib.md5(open(src, "rb").read()).hexdigest() == ADAM_TRAFFIC["source_md5"]
    traffic = ADAM_TRAFFIC["bytes"] if same_src and model.n_params == ADAM_TRAFFIC["params"] \
        else None
    log(f"[bench] step {ms:.3f} ms: fused fwd+bwd {fb_ms:.3f} ms, adam {adam_ms:.3f} ms; "
        f"mean loss {loss:.4g}")
    out = {
        "metric": "train samples/s fwd+bwd (FP32 path), whole training step incl. dense Adam",
        "value": B / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "F-Hash training, 480x720x120x100 synthetic volume, 16 levels "
                   "x 2 features, MLP 32-64-64-1, batch 2^18 coreset draws",
                   "shape": dims, "levels": args.levels, "batch": B,
                   "active_vertices": model.rows, "params": model.n_params,
                   "coreset": M},
        "breakdown_ms": {"fused_fwd_bwd": fb_ms, "adam": adam_ms,
                         "sampler_and_other": ms - fb_ms - adam_ms},
        "roofline": {"kernel": "adam_kernel", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes": adam_bytes},
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(model, gen, dims, B, args.cpu_samples, 2002)
        except Exception as e:  # reported, never hidden
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
