"""Benchmark: adaptive black-hole image rendering on one MI355X.

One step = one full adaptive render (Sec. 3.2) of the thermal-plasma workload:
Kerr a = 0.94, inclination 163 deg, polarised I,Q,U,V transfer at 230 GHz,
base 129^2 vertices refined 3 levels to 1025^2 with R_rel = 0.01 and
R_abs = 1e-3 x (max of the level-0 image).  Every step runs the whole hot path:
base-grid tracing, the level-0 reduction, and per level the estimator /
interpolation / ballot compaction kernel and the persistent tracing kernel.
Inputs (camera, plasma parameters) are resident before the timed region.

value = traced rays per second of wall time; effective pixels/s = 1025^2 /
render time.  The image is checked against the uniform (every-pixel) render:
normalised MSE <= 1e-3 (Sec. 4.1, Eq. 9).  The roofline entry reports the
tracing kernel's algorithmic FP64 throughput (hand-counted FLOPs per geodesic
step and per emitting step) against the FP64 vector peak; the CPU baseline is
the FP64 oracle timed on a random sample of the rays the render traced.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s and effective pixels/s at image MSE ≤0.1%; learned+batched vs plain"

# Algorithmic FLOPs (+, -, *, /, sqrt and each transcendental = 1), counted
# from the method's expressions:
FLOP_GEO_STEP = 381          # 4 right-hand sides, RK4 combination, step rule, midpoint
FLOP_PLASMA_THERMAL = 390    # flow, field, frame, Walker-Penrose angle, coefficients
FLOP_TRANSFER_IQUV = 790     # two closed-form Lorentz exponentials, O update, emission
FLOP_TRANSFER_I = 10
FLOP_PLASMA_TOY = 96
PEAK_FP64_VECTOR = 78.6e12   # MI355X published FP64 vector peak
PEAK_FP32_VECTOR = 157.3e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops(stats, cfg):
    emit = FLOP_PLASMA_THERMAL if cfg["model"] == "thermal" else FLOP_PLASMA_TOY
    emit += FLOP_TRANSFER_IQUV if cfg.get("nstokes", 1) == 4 else FLOP_TRANSFER_I
    return stats["steps"] * FLOP_GEO_STEP + stats["steps_emit"] * emit


def cpu_baseline(cfg, budget_s):
    """The oracle's complete adaptive render of the same workload (its ray
    tracer over every base and refined point, its numpy refinement), repeated
    until the time budget is spent; rays/s and effective pixels/s."""
    from oracle import ray as oray
    from oracle import refine as oref
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    fn = lambda x, y: oray.trace(cfg, x, y, nthreads=cores)[0]
    oray.trace(cfg, np.array([0.0]), np.array([0.0]), nthreads=1)   # build / load
    rays, px, n, t0 = 0, 0, 0, time.perf_counter()
    while n == 0 or time.perf_counter() - t0 < budget_s:
        o = oref.refine(fn, cfg["fov"], cfg["nx0"], cfg["ny0"], cfg["levels"], cfg["r_rel"],
                        cfg["r_abs"], cfg["abs_norm"], cfg["nstokes"])
        rays += o["rays"]
        px += o["nx"] * o["ny"]
        n += 1
    dt = time.perf_counter() - t0
    return dict(value=rays / dt, unit="rays/s", cores=cores, kind="oracle",
                effective_px_per_s=px / dt,
                sample="%d complete oracle adaptive renders of the same workload (%d rays each, "
                       "FP64 scalar C ray tracer on %d threads + numpy refinement), %.1f s"
                       % (n, rays // n, cores, dt))


def batched(art, torch, art_inputs, args):
    """64 images (spin x inclination x frequency, 1-4 levels each) in one batch:
    one work queue per level, the level loop captured once in a hipGraph and
    replayed; launch shape from the autotuner."""
    from paper_2103_07417_amd import autotune
    cfgs = art_inputs.batch_workload(precision="mixed")
    B = art.Batch(cfgs)
    npix = sum(im.shape[1] * im.shape[2] for im in B.images)
    s = torch.cuda.Stream()
    tune = None
    if not args.no_autotune:
        tune = autotune.autotune(B, s, reps=1, use_cache=False, log=log)
        log("autotune: %s" % {k: tune[k] for k in ("trace_blocks", "trace_threads", "refill", "ms")})
    B.render(s)
    s.synchronize()
    eager = B.stats()
    B.capture(s)
    B.launch(s)
    s.synchronize()
    st = B.stats()
    assert st["rays"] == eager["rays"]
    reps = max(2, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        B.launch(s)
    s.synchronize()
    dt = (time.perf_counter() - t0) / reps
    # accuracy: one image per refinement depth against its uniform render
    mses = {}
    for k in (20, 21, 22, 23):      # a=0.5, i=60 deg, all four frequencies, 1..4 levels
        truth, _, _ = art.render_uniform(cfgs[k])
        fe, mse = art.metrics(truth[0], B.images[k][0])
        mses[cfgs[k]["name"]] = dict(levels=cfgs[k]["levels"], mse=mse, flux_error=fe,
                                     npix=B.images[k].shape[1] * B.images[k].shape[2])
    B.close()
    log("batched: %.1f ms per 64-image batch, %d rays, %d px" % (dt * 1e3, st["rays"], npix))
    return {
        "workload": "64 thermal-plasma images: a in {0,0.5,0.94,-0.94} x i in {17,60,90,163} deg x "
                    "nu in {86,230,345,690} GHz, base 129^2, 1+(k mod 4) levels (257^2..2049^2), "
                    "IQUV, FP64 geodesic / FP32 transfer, one hipGraph replay per batch",
        "ms_per_batch": dt * 1e3, "rays": st["rays"], "effective_px": npix,
        "rays_per_s": st["rays"] / dt, "effective_px_per_s": npix / dt,
        "interp_frac": st["interp_frac"], "mse_check": mses,
        "mse_ok": all(v["mse"] <= 1e-3 for v in mses.values()),
        "launch": tune and {k: tune[k] for k in ("trace_blocks", "trace_threads", "refill", "ms",
                                                   "default", "default_ms")},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import art_inputs
    from paper_2103_07417_amd import art

    cfg = dict(art_inputs.workload("thermal_1025"), precision=args.precision)
    nx, ny = art.image_size(cfg)
    log("workload thermal_1025: %dx%d, precision %s" % (nx, ny, args.precision))

    # truth image (untimed): one ray per pixel
    truth, _, ust = art.render_uniform(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    truth, _, ust = art.render_uniform(cfg)
    torch.cuda.synchronize()
    t_uniform = time.perf_counter() - t0
    log("uniform render: %d rays in %.1f ms" % (ust["rays"], t_uniform * 1e3))

    bufs = art.alloc(cfg)
    for _ in range(args.warmup):
        art.render(cfg, out=bufs)
    torch.cuda.synchronize()
    log("warmup done")
    tr_ms, launches, fl, rays = 0.0, 0, 0, 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        img, lev, _, st = art.render(cfg, out=bufs)
        tr_ms += st["t_trace_ms"]
        launches += st["trace_launches"]
        fl += flops(st, cfg)
        rays += st["rays"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("timed %d renders in %.1f ms" % (args.steps, dt * 1e3))
    ms = dt / args.steps * 1e3
    fe, mse = art.metrics(truth[0], img[0])
    rays_per_render = rays // args.steps
    value = rays_per_render / (ms * 1e-3)
    px_s = nx * ny / (ms * 1e-3)
    achieved = (fl / launches) / (tr_ms / launches * 1e-3)
    peak = PEAK_FP64_VECTOR
    roof = dict(bound="alu", achieved=achieved / 1e12, peak=peak / 1e12, unit="TFLOP/s",
                frac=achieved / peak, traffic=None,
                kernel="k_trace (FP64 geodesic + %s transfer)" % args.precision,
                avg_launch_ms=tr_ms / launches, flops_per_render=fl // args.steps,
                trace_share_of_render=tr_ms / (dt * 1e3))
    out = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64-geodesic/f32-transfer",
        "data": "synthetic",
        "config": {"workload": "thermal_1025: Kerr a=0.94, i=163 deg, IQUV at 230 GHz, "
                               "power-law thermal plasma, base 129^2 -> 3 levels -> 1025^2, "
                               "R_rel=0.01, R_abs=1e-3 max I0",
                   "base": 129, "final": nx, "levels": 3, "precision": args.precision},
        "effective_px_per_s": px_s,
        "rays_per_render": rays_per_render,
        "interp_frac": st["interp_frac"],
        "image_mse_vs_uniform": mse, "flux_error_vs_uniform": fe, "mse_ok": mse <= 1e-3,
        "uniform": {"ms": t_uniform * 1e3, "rays": ust["rays"],
                    "rays_per_s": ust["rays"] / t_uniform,
                    "speedup_adaptive_vs_uniform": t_uniform * 1e3 / ms},
        "roofline": roof,
    }
    if not args.no_batch:
        out["batched"] = batched(art, torch, art_inputs, args)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
