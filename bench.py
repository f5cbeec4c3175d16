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


def cpu_baseline(cfg, level_map, budget_s):
    """Oracle rays/s on a random sample of the pixels the render traced."""
    from oracle import ray as oray
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    ny, nx = level_map.shape
    jj, ii = np.nonzero(level_map >= 0)
    rng = np.random.default_rng(0)
    order = rng.permutation(ii.size)
    oray.trace(cfg, np.array([0.0]), np.array([0.0]), nthreads=1)   # build / load
    done, t0, k = 0, time.perf_counter(), 0
    chunk = 2048
    while time.perf_counter() - t0 < budget_s and k < order.size:
        sel = order[k:k + chunk]
        x, y = oray.screen_coords(cfg["fov"], nx, ny, ii[sel], jj[sel])
        oray.trace(cfg, x, y, nthreads=cores)
        done += sel.size
        k += chunk
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="rays/s", cores=cores, kind="oracle",
                sample="%d rays drawn uniformly from the %d pixels the adaptive render traced "
                       "(same camera, plasma and step rule), FP64 scalar C, %.1f s"
                       % (done, ii.size, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
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
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cfg, lev.cpu().numpy(), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
