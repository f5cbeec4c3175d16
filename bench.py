"""Benchmark: adaptive black-hole image rendering on one MI355X.

Headline workload (the batched configuration): 64 images of a power-law
thermal plasma, spins a in {0, 0.5, 0.94, -0.94} x inclinations {17, 60, 90,
163} deg x frequencies {86, 230, 345, 690} GHz, polarised I, Q, U, V, base
129^2 vertices with image k refined 1 + (k mod 4) levels (257^2 ... 2049^2,
89.3 M effective pixels), R_abs = 1e-3 x (max of the level-0 image), FP32
plasma and transfer with the FP64 geodesic (the selective-FP64 policy, FP32
right-hand sides away from the photon shell, the horizon and the theta
turning points, and the all-FP64 path are timed beside it: on this chip an
FP64 FMA issues at the unpacked FP32 rate, so the selective policy saves no
time).  One step = one render of the batch,
the whole level loop one hipGraph replay; steps are timed with several
batches in flight (depth and persistent-grid shape autotuned per form).

Forms compared at the 0.1 % MSE bar (normalised MSE of Stokes I against the
uniform render of the same view, Sec. 4.1 Eq. 9):
  - learned + batched: the proposal network (trained first, untimed, on
    plain renders of 16 other images of the batch's structure) looks two
    levels ahead, the criterion of Sec. 3.2 judges and traces what it missed
    (or only counts it: judge-only forms); the network runs at every level it
    can look ahead from, or (forms *_l0) at level 0 only, the deeper levels
    taking the criterion alone;
  - plain batched: the criterion alone.
Each form's tolerance is chosen on a held-out batch of the same structure
(other spins, inclinations and field phases): the loosest R_rel of a fixed
grid at which all 64 held-out images pass the bar, then applied unchanged to
the timed batch; among the learned forms the one fastest on the held-out
batch at its operating point is timed.  A form with no passing R_rel on the held-out batch is timed
at the grid's tightest R_rel and reported as such; the plain criterion is
also timed at the loosest R_rel that passes on the timed batch itself (a
choice made on the measured images, favourable to it).  Timings are repeated
and interleaved between forms; the median and the range are reported.

value = traced rays per second of the learned + batched form (median step);
effective pixels/s = 89.3 M / time per batch.  Q, U and V errors are reported
per plane beside the bar (the bar itself is on Stokes I).  The roofline entry
reports the tracing kernel's algorithmic FLOP rate (per geodesic step and per
emitting step, counted by the oracle's instrumented build) against the
vector ALU peak; the CPU baseline is the FP64 oracle's complete adaptive
render of a sample of the headline images.

Further sections (each with its own timing): the plain method one image at a
time on the thermal view (the paper's method), the uniform render, the
gridded snapshot at 4097^2, the snapshot at 16385^2 with subrings n = 0..3
and the visibility domain of its learned render (Sec. 4.3), adaptive sampling
along frequency and time, and the refinement variants.
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

# Algorithmic operations (+, -, *, /, sqrt and each transcendental call = 1)
# of the method as the FP64 oracle evaluates it, counted by its instrumented
# build (oracle/opcount.cpp) and averaged over rays of the thermal view
# (tests/test_oracle_opcount.py pins these against the counter):
FLOP_GEO_STEP = 414          # 4 right-hand sides, RK4 combination, step rule, midpoint, features
FLOP_PLASMA_THERMAL = 429    # flow, field, frame, Walker-Penrose angle, coefficients (emitting step)
FLOP_PLASMA_NOEMIT = 77      # plasma point of a step outside the emitting region
FLOP_TRANSFER_IQUV = 1266    # two Lorentz exponentials, mean depth, emission, O <- O M
FLOP_TRANSFER_I = 16
FLOP_PLASMA_TOY = 176
# The same steps in the tracer's own structured forms (sin/cos of theta
# rotated instead of recomputed, the propagator's block structure): what the
# GPU actually executes, reported beside the algorithmic figure.
FLOP_STRUCTURED = dict(geo=381, plasma=390, transfer_iquv=639)
PEAK_VECTOR = 78.6e12        # MI355X FP64 vector peak = its unpacked FP32 rate (no packed FP32 here)
PEAK_FP64_MATRIX = 78.6e12   # MI355X FP64 matrix (MFMA) peak: the visibility stages
COPY_BYTES = 256 << 20       # read and written once by the calibration copy
ROOF_RENDERS = 2             # eager renders of the headline form timed for the roofline
# Algorithmic HBM bytes per traced ray of the thermal model: the list item
# (8 B) read, I,Q,U,V (32 B), the features (16 B) and the step count (2 B)
# written.
BYTES_PER_RAY = 58

# HBM traffic of the tracing kernel from FETCH_SIZE / WRITE_SIZE counter runs
# of this benchmark, per render of the headline form; valid only for the
# kernel sources it was measured on (hash below), else reported as null.
TRAFFIC = dict(bytes_per_render=313801608, kernel_hash="d340999eb37e1e55", form="judge_z2_l0",
               precision="mixed",
               source="profiles/k_trace_learned_batched_uneven_64.md: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 "
                      "(scales from a 256 MiB device copy), k_trace launches of the two roofline renders, "
                      "counter runs at 256 x 256 threads, 224 refinement blocks, refill 4, long-ray "
                      "threshold 700")
# the tracer and the kernels that build its queues (the queue order sets which
# rays finish together, and so how many of their scattered result stores share
# a sector)
TRAFFIC_SOURCES = ("paper_2103_07417_amd/csrc/art_trace.hip", "paper_2103_07417_amd/csrc/art_device.hpp",
                   "paper_2103_07417_amd/csrc/art_kernels.hip", "paper_2103_07417_amd/csrc/art_cnn.hip")

# proposal thresholds of the judge-only render at 16385^2, chosen on a held-out
# snapshot (other turbulence seed, same view)
DEPLOY_Z = (0.0, 1.0, 2.0, 3.0, 4.0, 6.0)
DEPLOY_HELDOUT_SEED = 5

# operating-point grid (R_rel) and the look-ahead proposal thresholds tried
OP_RREL = (0.001, 0.002, 0.003, 0.005, 0.0075, 0.01, 0.0125, 0.015)
OP_Z = (0.0, 2.0, 4.0)
OP_Z_JUDGE = (0.0, 2.0)      # judge-only forms (no fallback pass)
OP_Z_JUDGE_L0 = (0.0, 2.0, 4.0, 6.0)    # judge-only forms with the network at level 0 only
HELDOUT_LAUNCH = dict(trace_blocks=256, trace_threads=256, refill=1, groups=1)
TRAIN_RREL = 0.005           # tolerance of the plain renders the network learns from
PRECISION_NAMES = dict(fp64="FP64 throughout", mixed="FP64 geodesic, FP32 plasma and transfer",
                       mixed_geo="FP64 geodesic with FP32 right-hand sides outside the sensitive zones, "
                                 "FP32 plasma and transfer")
# depths searched for the batches in flight (the box gives a process four
# hardware queues)
IN_FLIGHT_DEPTHS = (2, 3, 4)
TIMING_ROUNDS = 5            # interleaved timing rounds per form


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(launches, form, precision):
    """HBM bytes per tracing launch of the roofline renders (per-render counter
    total over this run's launches per render), or None for other kernels,
    another headline form or another precision policy (another kernel
    instantiation)."""
    if not TRAFFIC or TRAFFIC["kernel_hash"] != kernel_hash() or TRAFFIC["form"] != form or \
            TRAFFIC["precision"] != precision or launches <= 0:
        return None
    return dict(bytes_per_launch=TRAFFIC["bytes_per_render"] * ROOF_RENDERS / launches,
                source=TRAFFIC["source"])


def finite(x):
    """The report with infinite option values (a disabled threshold) written
    as strings, so that the line is strict JSON."""
    if isinstance(x, dict):
        return {k: finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite(v) for v in x]
    if isinstance(x, float) and (x != x or x in (float("inf"), float("-inf"))):
        return repr(x)
    return x


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops(stats, cfg, counts=None):
    """Algorithmic operations of a render from its step counts."""
    c = counts or dict(geo=FLOP_GEO_STEP, plasma=FLOP_PLASMA_THERMAL, noemit=FLOP_PLASMA_NOEMIT,
                       transfer_iquv=FLOP_TRANSFER_IQUV)
    steps, emit = stats["steps"], stats["steps_emit"]
    if cfg["model"] == "thermal":
        emitf = c["plasma"] + (c["transfer_iquv"] if cfg.get("nstokes", 1) == 4 else FLOP_TRANSFER_I)
        return steps * c["geo"] + emit * emitf + (steps - emit) * c.get("noemit", 0)
    emitf = FLOP_PLASMA_TOY + (FLOP_TRANSFER_IQUV if cfg.get("nstokes", 1) == 4 else FLOP_TRANSFER_I)
    return steps * c["geo"] + emit * emitf


def cpu_cores():
    """Threads the oracle baseline uses: the process's CPUs, at most 16 (the
    CPU share of one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n)), n


def cpu_baseline(cfgs, budget_s, budget_1core_s):
    """The oracle's complete adaptive renders (its ray tracer over every base
    and refined point, its numpy refinement) of headline images in a fixed
    shuffled order until the time budget is spent, on all threads of the CPU
    share and on one thread; rays/s and effective pixels/s of the sample."""
    from oracle import ray as oray
    from oracle import refine as oref
    cores, visible = cpu_cores()
    order = list(np.random.default_rng(7).permutation(len(cfgs)))
    oray.trace(cfgs[0], np.array([0.0]), np.array([0.0]), nthreads=1)   # build / load

    def run(nthreads, budget, order):
        rays, px, names, t0 = 0, 0, [], time.perf_counter()
        for k in order:
            c = cfgs[k]
            fn = lambda x, y, c=c: oray.trace(c, x, y, nthreads=nthreads)[0]
            o = oref.refine(fn, c["fov"], c["nx0"], c["ny0"], c["levels"], c["r_rel"], c["r_abs"],
                            c["abs_norm"], c["nstokes"])
            rays += o["rays"]
            px += o["nx"] * o["ny"]
            names.append(c["name"])
            if time.perf_counter() - t0 >= budget:
                break
        dt = time.perf_counter() - t0
        return dict(rays_per_s=rays / dt, effective_px_per_s=px / dt, seconds=dt, rays=rays, images=names)
    full = run(cores, budget_s, order)
    # one thread: the one-level images only (each a few seconds)
    one = run(1, budget_1core_s, [k for k in order if cfgs[k]["levels"] == 1])
    return dict(value=full["rays_per_s"], unit="rays/s", cores=cores, kind="oracle",
                effective_px_per_s=full["effective_px_per_s"], cpus_visible=visible,
                one_core=dict(rays_per_s=one["rays_per_s"], effective_px_per_s=one["effective_px_per_s"],
                              images=len(one["images"]), seconds=one["seconds"]),
                sample="complete oracle adaptive renders (FP64 scalar C ray tracer + numpy refinement) of "
                       "%d headline images in a fixed shuffled order (%s; %d rays) on %d threads in %.1f s; "
                       "one thread: %d one-level images in %.1f s; rays/s and px/s of the sample stand in for "
                       "the 64-image batch (extrapolated)"
                       % (len(full["images"]), ",".join(full["images"]), full["rays"], cores, full["seconds"],
                          len(one["images"]), one["seconds"]))


def mse_check(art, cfgs, images, truths, planes=1):
    """Normalised MSE (Eq. 9) and flux error of every image against its
    uniform render, per plane for the first `planes` planes; the bar is on
    plane 0 (Stokes I)."""
    out = []
    for k, c in enumerate(cfgs):
        m = []
        for q in range(planes):
            # a truth given as one 2D plane is Stokes I
            t = truths[k] if truths[k].dim() == 2 else truths[k][q]
            fe, mse = art.metrics(t, images[k][q])
            m.append(mse)
            if q == 0:
                fe0 = fe
        out.append(dict(name=c["name"], mse=m[0], mse_planes=m, flux_error=fe0))
    res = dict(mse_max=max(o["mse"] for o in out), mse_mean=sum(o["mse"] for o in out) / len(out),
               flux_error_max=max(o["flux_error"] for o in out), mse_ok=all(o["mse"] <= 1e-3 for o in out),
               n_over_bar=sum(1 for o in out if o["mse"] > 1e-3),
               worst=max(out, key=lambda o: o["mse"])["name"])
    if planes > 1:
        res["mse_max_planes"] = [max(o["mse_planes"][q] for o in out) for q in range(planes)]
    return res


def time_graph(B, torch, s, reps):
    B.capture(s)
    B.launch(s)
    s.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        B.launch(s)
    s.synchronize()
    return (time.perf_counter() - t0) / reps


def time_pipelined(Bs, torch, streams, reps):
    """Time per batch with len(Bs) batches in flight: batch k % n is replayed
    on its own stream, so one batch's latency-bound refinement passes overlap
    the next batch's throughput-bound base pass.  Every step renders a whole
    batch; the clock stops when every stream has finished."""
    from paper_2103_07417_amd import autotune
    return autotune.time_in_flight(Bs, torch, streams, reps) * 1e-3


def operating_points(search, op_forms):
    """Per form, the search row with the loosest R_rel at which every image
    passed the bar (forms that never pass are left out)."""
    op = {}
    for name, opts in op_forms:
        passing = [r for r in search if r["form"] == name and r["ok"]]
        if passing:
            op[name] = dict(max(passing, key=lambda r: r["r_rel"]), options=opts)
    return op


def parse_launch(text):
    """BLOCKSxTHREADS[:REFINE_BLOCKS] -> launch dict (refine_blocks 0: the
    refinement passes use BLOCKS)."""
    shape, _, rb = text.lower().partition(":")
    tb, tt = (int(v) for v in shape.split("x"))
    return dict(trace_blocks=tb, trace_threads=tt, refill=1, groups=1, refine_blocks=int(rb) if rb else 0)


def choose_forms(op_heldout, op_timed, grid, heldout_ms=None):
    """The forms timed on the headline batch, as (name, form, R_rel, how):
    the learned form fastest on the held-out batch at its held-out operating
    point (heldout_ms: form -> ms per batch; without it the one with the
    fewest held-out rays); the plain criterion at its held-out operating
    point, or at the grid's tightest R_rel if it has none; and the plain
    criterion at the loosest R_rel passing on the timed batch itself, if that
    differs."""
    out = []
    lop = {k: v for k, v in op_heldout.items() if k != "plain"}
    if lop:
        if heldout_ms:
            k = min((n for n in lop if n in heldout_ms), key=lambda n: heldout_ms[n])
            how = "held-out operating point, fastest learned form on the held-out batch"
        else:
            k = min(lop, key=lambda n: lop[n]["rays"])
            how = "held-out operating point"
        out.append(("learned_batched", k, lop[k]["r_rel"], how))
    if "plain" in op_heldout:
        out.append(("plain_batched", "plain", op_heldout["plain"]["r_rel"], "held-out operating point"))
    else:
        out.append(("plain_batched", "plain", min(grid), "tightest tolerance of the grid (no held-out "
                                                         "operating point)"))
    if "plain" in op_timed and op_timed["plain"]["r_rel"] != out[-1][2]:
        out.append(("plain_batched_own_op", "plain", op_timed["plain"]["r_rel"],
                    "loosest tolerance passing on the timed batch itself"))
    return out


def search_batch(art, torch, cfgs, truths, net, op_forms, s, feat_planes=1):
    """Eager renders of a batch at every R_rel of the grid and every form:
    rays, steps and the MSE check of each."""
    rows = []
    for rr in OP_RREL:
        X = art.Batch([dict(c, r_rel=rr) for c in cfgs], feat=True)
        for name, opts in op_forms:
            X.set_learned(None) if opts is None else X.set_learned(net, **opts)
            X.render(s)
            st = X.stats(stream=s)
            chk = mse_check(art, cfgs, X.images, truths, feat_planes)
            rows.append(dict(form=name, r_rel=rr, rays=st["rays"], steps=st["steps"], mse_max=chk["mse_max"],
                             n_over_bar=chk["n_over_bar"], worst=chk["worst"], ok=chk["mse_ok"],
                             mse_max_planes=chk.get("mse_max_planes")))
        X.close()
    return rows


def c4_forms(art, torch, art_inputs, args):
    """The headline: learned + batched against plain batched on the uneven
    64-image batch, each at its operating point chosen on the held-out batch;
    batches in flight, interleaved timing rounds; the roofline renders."""
    from paper_2103_07417_amd import autotune, learn
    nmax = args.in_flight or max(IN_FLIGHT_DEPTHS)
    Ss = [art.Stream() for _ in range(nmax)]
    ss = [S.torch for S in Ss]
    s = ss[0]
    t0 = time.perf_counter()
    net, tinfo = learn.train(art_inputs.training_workload_batch(precision="mixed", r_rel=TRAIN_RREL),
                             steps=args.train_steps, lr=3e-3, seed=4, stream=s)
    s.synchronize()
    t_train = time.perf_counter() - t0
    log("trained proposal network in %.1f s: loss %s -> %s" % (t_train, tinfo["loss_first"], tinfo["loss_last"]))
    inf = float("inf")
    op_forms = [("plain", None)] + [("lookahead_z%g" % z, dict(z_propose=z, z_suppress=-inf, fallback=True))
                                    for z in OP_Z] + \
        [("judge_z%g" % z, dict(z_propose=z, z_suppress=-inf, fallback=False)) for z in OP_Z_JUDGE] + \
        [("lookahead_z4_l0", dict(z_propose=4.0, z_suppress=-inf, fallback=True, level_cap=1))] + \
        [("judge_z%g_l0" % z, dict(z_propose=z, z_suppress=-inf, fallback=False, level_cap=1))
         for z in OP_Z_JUDGE_L0]
    opts_of = dict(op_forms)

    def truths_of(cfgs):
        out = []
        for c in cfgs:
            t, _, _ = art.render_uniform(c, stream=s)
            out.append(t.clone())
            del t
        s.synchronize()
        return out
    held = art_inputs.batch_workload_heldout(precision=args.precision)
    truths_h = truths_of(held)
    search_h = search_batch(art, torch, held, truths_h, net, op_forms, s)
    del truths_h
    op_h = operating_points(search_h, op_forms)
    log("held-out operating points: %s" % {k: (v["r_rel"], v["rays"], "%.2e" % v["mse_max"])
                                           for k, v in op_h.items()})
    # the learned forms timed on the held-out batch at their operating points
    # (a fixed launch shape, three batches in flight): the fastest is timed
    # on the headline batch
    ms_h = {}
    dh = min(3, nmax)
    if args.learned_form and args.learned_form not in op_h:
        raise SystemExit("--learned-form %s: no held-out operating point for that form (have %s)"
                         % (args.learned_form, sorted(op_h)))
    for name, row in op_h.items():
        if name == "plain" or (args.learned_form and name != args.learned_form):
            continue
        bs = [art.Batch([dict(c, r_rel=row["r_rel"]) for c in held], feat=True) for _ in range(dh)]
        for X in bs:
            X.set_learned(net, **opts_of[name])
            X.set_launch(**HELDOUT_LAUNCH)
        ms_h[name] = min(time_pipelined(bs, torch, ss[:dh], args.steps) for _ in range(2)) * 1e3
        for X in bs:
            X.close()
    log("learned forms on the held-out batch (ms per batch): %s" % {k: round(v, 2) for k, v in ms_h.items()})
    cfgs = art_inputs.batch_workload(precision=args.precision)
    truths = truths_of(cfgs)
    search_c = search_batch(art, torch, cfgs, truths, net, op_forms, s, 4)
    op_c = operating_points(search_c, op_forms)
    log("operating points on the timed batch itself: %s" % {k: (v["r_rel"], v["rays"], "%.2e" % v["mse_max"])
                                                            for k, v in op_c.items()})
    chosen = choose_forms(op_h, op_c, OP_RREL, ms_h)
    npix = sum(c_img.shape[1] * c_img.shape[2] for c_img in truths)
    forms, sets = {}, {}
    for name, form, rr, how in chosen:
        c_rr = [dict(c, r_rel=rr) for c in cfgs]
        opts = opts_of[form]
        bset = [art.Batch(c_rr, feat=opts is not None) for _ in range(nmax)]
        for X in bset:
            X.set_learned(None) if opts is None else X.set_learned(net, **opts)
        depth, tune = nmax, None
        launch = dict(trace_blocks=512, trace_threads=256, refill=1, groups=1, refine_blocks=0, long_steps=0)
        if args.launch:
            # a fixed shape (counter runs serialise dispatches, which would
            # steer the in-flight search to other shapes than the timed run's)
            launch = dict(parse_launch(args.launch), refill=args.refill, long_steps=args.long_steps)
            depth = args.in_flight or 3
        elif not args.no_autotune:
            depths = (args.in_flight,) if args.in_flight else IN_FLIGHT_DEPTHS
            tune = autotune.autotune_in_flight(bset, ss, depths=depths, log=None)
            depth = tune["in_flight"]
            launch = {k: tune[k] for k in ("trace_blocks", "trace_threads", "refill", "groups", "refine_blocks",
                                           "long_steps")}
        for X in bset:
            X.set_launch(**launch)
        for X in bset[depth:]:
            X.close()
        bset = bset[:depth]
        # latency of one batch alone: the in-flight shape with the base grid's
        # size for every pass (a smaller refinement grid only pays when other
        # batches take the freed slots) and with twice that grid (alone, a
        # batch has every wave slot of the chip), each with one and with two
        # image groups (one group's pass tail overlaps the other's work); the
        # fastest is reported
        B0 = bset[0]
        lat, lat_launch = None, None
        for groups in (1, 2):
            for mult in (1, 2):
                shape = dict(launch, trace_blocks=launch["trace_blocks"] * mult, refine_blocks=0, groups=groups)
                B0.set_launch(**shape)
                t = time_graph(B0, torch, s, max(3, args.steps // 3))
                if lat is None or t < lat:
                    lat, lat_launch = t, shape
        B0.set_launch(**launch)
        for X in bset:
            X.set_launch(**launch)
        for _ in range(args.warmup):
            for X, sx in zip(bset, ss):
                X.render(sx)
        torch.cuda.synchronize()
        B0.render(s)
        st = B0.stats(stream=s)
        chk = mse_check(art, c_rr, B0.images, truths, 4)
        f = dict(form=form, r_rel=rr, chosen_by=how, options=opts, in_flight=depth, launch=launch,
                 latency_ms=lat * 1e3, latency_launch=lat_launch, rays=st["rays"], steps=st["steps"],
                 steps_emit=st["steps_emit"],
                 passes=st["trace_launches"], interp_frac=st["interp_frac"], check=chk, rounds_ms=[])
        if opts is not None:
            f["judge"] = st["learned"]
        forms[name] = f
        sets[name] = bset
        log("%s: %s at R_rel %g (%s), %d rays, %.4g steps, %d passes, mse max I %.2e (%d over), planes %s" % (
            name, form, rr, how, st["rays"], st["steps"], st["trace_launches"], chk["mse_max"], chk["n_over_bar"],
            ["%.1e" % x for x in chk["mse_max_planes"]]))
    # interleaved timing rounds: every form K steps in flight per round
    for r in range(TIMING_ROUNDS):
        for name, bset in sets.items():
            dt = time_pipelined(bset, torch, ss[:len(bset)], args.steps)
            forms[name]["rounds_ms"].append(dt * 1e3)
    for name, f in forms.items():
        ms = sorted(f["rounds_ms"])
        f["ms_per_batch"] = ms[len(ms) // 2]
        f["ms_range"] = [ms[0], ms[-1]]
        f["rays_per_s"] = f["rays"] / (f["ms_per_batch"] * 1e-3)
        f["effective_px_per_s"] = npix / (f["ms_per_batch"] * 1e-3)
        log("%s: %.2f ms/batch median of %d rounds [%.2f, %.2f], %d in flight; alone %.1f ms" % (
            name, f["ms_per_batch"], len(ms), ms[0], ms[-1], f["in_flight"], f["latency_ms"]))
    # the other precision policies: the same forms, tolerances, depth and
    # launch shape, timed the same way (two rounds), with the MSE check
    policies = {}
    for prec in ("mixed", "mixed_geo", "fp64"):
        if prec == args.precision:
            continue
        for name in ("learned_batched", "plain_batched"):
            if name not in forms:
                continue
            f = forms[name]
            opts = opts_of[f["form"]]
            c_rr = [dict(c, r_rel=f["r_rel"], precision=prec) for c in cfgs]
            bs = [art.Batch(c_rr, feat=opts is not None) for _ in range(f["in_flight"])]
            for X in bs:
                X.set_learned(None) if opts is None else X.set_learned(net, **opts)
                X.set_launch(**f["launch"])
            ms = sorted(time_pipelined(bs, torch, ss[:len(bs)], args.steps) * 1e3 for _ in range(2))
            bs[0].render(s)
            st = bs[0].stats(stream=s)
            chk = mse_check(art, c_rr, bs[0].images, truths, 1)
            policies.setdefault(prec, {})[name] = dict(
                ms_per_batch=ms[0], ms_range=[ms[0], ms[-1]], rays=st["rays"], steps=st["steps"],
                rays_per_s=st["rays"] / (ms[0] * 1e-3), effective_px_per_s=npix / (ms[0] * 1e-3),
                mse_max=chk["mse_max"], mse_ok=chk["mse_ok"])
            log("%s in %s: %.2f ms/batch, %d rays, mse max %.2e" % (name, prec, ms[0], st["rays"], chk["mse_max"]))
            for X in bs:
                X.close()
    # eager renders of the headline form with HIP events around each tracing
    # launch (on the group stream): the roofline figures
    head = "learned_batched" if "learned_batched" in forms else "plain_batched"
    Bh = sets[head][0]
    Bh.set_launch(**forms[head]["launch"])
    tr_ms, launches, fl, fls, render_ms, rays = 0.0, 0, 0, 0, 0.0, 0
    hcfg = cfgs[0]
    for _ in range(ROOF_RENDERS):
        Bh.render(s)
        st = Bh.stats(stream=s)
        tr_ms += st["t_trace_ms"]
        launches += st["trace_launches"]
        fl += flops(st, hcfg)
        fls += flops(st, hcfg, dict(FLOP_STRUCTURED, noemit=0))
        render_ms += st["t_render_ms"]
        rays += st["rays"]
    training = dict(seconds=t_train, steps=args.train_steps, images=16, pos_weight=tinfo["pos_weight"],
                    loss_first={str(k): v for k, v in tinfo["loss_first"].items()},
                    loss_last={str(k): v for k, v in tinfo["loss_last"].items()})
    for bset in sets.values():
        for X in bset:
            X.close()
    net.close()
    for S in Ss:
        S.close()
    del truths
    torch.cuda.empty_cache()
    roof_src = dict(tr_ms=tr_ms, launches=launches, flops=fl, flops_structured=fls, render_ms=render_ms,
                    rays=rays)
    search = dict(heldout=search_h, timed=search_c, operating_points_heldout=op_h,
                  operating_points_timed=op_c, learned_heldout_ms=ms_h)
    return forms, head, training, npix, roof_src, search, policies


def grid_forms(art, torch, art_inputs, args):
    """The gridded snapshot at 4097^2 (base 257^2, 4 levels, the paper's GRMHD
    tolerances): plain adaptive render in FP64 and mixed precision against
    the uniform (16.8 M-ray) render."""
    from art_inputs import mks
    t0 = time.perf_counter()
    grid, _ = mks.mks_snapshot(seed=2)
    g = torch.from_numpy(grid).cuda()
    t_gen = time.perf_counter() - t0
    out = dict(snapshot_seconds=t_gen, snapshot_bytes=int(grid.nbytes))
    truth = None
    for prec in ("mixed", "fp64"):
        cfg = dict(art_inputs.workload("grid_4097"), grid_dev=g, precision=prec)
        nx, ny = art.image_size(cfg)
        if truth is None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t, _, ust = art.render_uniform(cfg)
            torch.cuda.synchronize()
            t_uni = time.perf_counter() - t0
            truth = t[0].clone()
            del t
            out["uniform"] = dict(ms=t_uni * 1e3, rays=ust["rays"], rays_per_s=ust["rays"] / t_uni,
                                  precision=prec)
        bufs = art.alloc(cfg)
        art.render(cfg, out=bufs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            img, lev, _, st = art.render(cfg, out=bufs)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        fe, mse = art.metrics(truth, img[0])
        out[prec] = dict(ms_per_image=dt * 1e3, rays=st["rays"], passes=st["trace_launches"],
                         rays_per_s=st["rays"] / dt, effective_px_per_s=nx * ny / dt,
                         interp_frac=st["interp_frac"], mse_vs_uniform_mixed=mse, flux_error=fe)
        log("grid_4097 %s: %.1f ms, %d rays, IF %.4f, mse %.2e" % (prec, dt * 1e3, st["rays"],
                                                                  st["interp_frac"], mse))
        del bufs, img, lev
    del g
    torch.cuda.empty_cache()
    return out


def deploy_threshold(search, bar=1e-3):
    """Proposal threshold of the 16385^2 judge-only render from the held-out
    search rows (z_propose, mse): the largest z whose render kept Stokes I
    within the bar, else the smallest z tried."""
    passing = [r["z_propose"] for r in search if r["mse"] <= bar]
    return max(passing) if passing else min(r["z_propose"] for r in search)


def deploy_16385(art, torch, art_inputs, args):
    """Learned proposal deployed on the snapshot at 16385^2 (base 257^2, 6
    levels, Stokes I): plain and learned adaptive renders against the uniform
    render (268 M rays).  The network is trained on plain renders of the
    snapshot seen from other views (4097^2) and of the thermal images."""
    from art_inputs import mks
    from paper_2103_07417_amd import learn
    grid, _ = mks.mks_snapshot(seed=2)
    g = torch.from_numpy(grid).cuda()
    # the subring planes run with the FP32-transfer policy (the selective-FP64
    # geodesic policy has no subring variant)
    prec = "mixed" if args.precision == "mixed_geo" else args.precision
    cfg = dict(art_inputs.workload("grid_16385"), grid_dev=g, precision=prec)
    nx, ny = art.image_size(cfg)
    out = {"workload": "gridded snapshot a=0.94 i=163 deg, 230 GHz, Stokes I split into subrings n=0..3, "
                       "base 257^2 -> 6 levels -> %dx%d, R_rel=1e-3, R_abs=0.025 Ibar_int" % (nx, ny)}
    t0 = time.perf_counter()
    train_cfgs = art_inputs.grid_training_workload(g, precision=prec) + \
        art_inputs.training_workload(precision=prec)
    net, tinfo = learn.train(train_cfgs, steps=args.train_steps, lr=3e-3, seed=4)
    torch.cuda.synchronize()
    out["training"] = dict(seconds=time.perf_counter() - t0, images=len(train_cfgs),
                           loss_first={str(k): v for k, v in tinfo["loss_first"].items()},
                           loss_last={str(k): v for k, v in tinfo["loss_last"].items()})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    truth, _, ust = art.render_uniform(cfg)
    torch.cuda.synchronize()
    t_uni = time.perf_counter() - t0
    nsub = cfg["subrings"]

    def sub_flux(img):
        f = [float(img[1 + n].sum()) for n in range(nsub)]
        return dict(flux=f, ratio=[f[n + 1] / f[n] if f[n] else None for n in range(nsub - 1)])

    out["uniform"] = dict(ms=t_uni * 1e3, rays=ust["rays"], rays_per_s=ust["rays"] / t_uni,
                          subrings=sub_flux(truth))

    def sub_mse(img):
        return [art.metrics(truth[1 + n], img[1 + n])[1] for n in range(nsub)]
    log("16385^2 uniform: %d rays in %.0f ms" % (ust["rays"], t_uni * 1e3))
    bufs = art.alloc(cfg, feat=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    (img, lev, ft, st), dt = timed(lambda: art.render(cfg, out=bufs))
    fe, mse = art.metrics(truth[0], img[0])
    out["plain"] = dict(ms=dt * 1e3, rays=st["rays"], passes=st["trace_launches"], mse=mse, flux_error=fe,
                        effective_px_per_s=nx * ny / dt, rays_per_s=st["rays"] / dt,
                        subrings=sub_flux(img), subring_mse=sub_mse(img))
    log("16385^2 plain: %.0f ms, %d rays, mse %.2e" % (dt * 1e3, st["rays"], mse))
    # the criterion on every plane (I and the four subring planes)
    cfg_all = dict(cfg, all_planes=True)
    (img, lev, ft, st), dt = timed(lambda: art.render(cfg_all, out=bufs))
    fe, mse = art.metrics(truth[0], img[0])
    out["plain_all_planes"] = dict(ms=dt * 1e3, rays=st["rays"], passes=st["trace_launches"], mse=mse,
                                   flux_error=fe, effective_px_per_s=nx * ny / dt, rays_per_s=st["rays"] / dt,
                                   subrings=sub_flux(img), subring_mse=sub_mse(img))
    log("16385^2 plain, criterion on every plane: %.0f ms, %d rays, mse %.2e, subring mse %s" % (
        dt * 1e3, st["rays"], mse, ["%.2e" % x for x in out["plain_all_planes"]["subring_mse"]]))
    # ... with every plane against its own normalisation (the faint subrings
    # refined on their own structure)
    cfg_own = dict(cfg, all_planes="own")
    (img, lev, ft, st), dt = timed(lambda: art.render(cfg_own, out=bufs))
    fe, mse = art.metrics(truth[0], img[0])
    out["plain_own_norm"] = dict(ms=dt * 1e3, rays=st["rays"], passes=st["trace_launches"], mse=mse,
                                 flux_error=fe, effective_px_per_s=nx * ny / dt, rays_per_s=st["rays"] / dt,
                                 subrings=sub_flux(img), subring_mse=sub_mse(img))
    log("16385^2 plain, every plane against its own normalisation: %.0f ms, %d rays, mse %.2e, subring mse %s" % (
        dt * 1e3, st["rays"], mse, ["%.2e" % x for x in out["plain_own_norm"]["subring_mse"]]))
    for name, opts in (("learned_judge", dict(z_propose=args.z_propose, fallback=False)),
                       ("learned_fallback", dict(z_propose=args.z_propose, fallback=True))):
        (img, lev, ft, st), dt = timed(lambda: art.render_learned(cfg, net, out=bufs, **opts))
        fe, mse = art.metrics(truth[0], img[0])
        out[name] = dict(ms=dt * 1e3, rays=st["rays"], passes=st["trace_launches"], mse=mse, flux_error=fe,
                         effective_px_per_s=nx * ny / dt, rays_per_s=st["rays"] / dt, judge=st["learned"],
                         options=opts, subrings=sub_flux(img), subring_mse=sub_mse(img))
        log("16385^2 %s: %.0f ms, %d rays, %d passes, mse %.2e, judge %s" % (
            name, dt * 1e3, st["rays"], st["trace_launches"], mse, st["learned"]))
    # the judge-only form at the proposal threshold chosen on a held-out
    # snapshot (turbulence of another seed, the same view): the largest z of
    # the grid whose render of it keeps Stokes I within the bar
    img_keep = img.clone()
    held, _ = mks.mks_snapshot(seed=DEPLOY_HELDOUT_SEED)
    gh = torch.from_numpy(held).cuda()
    del held
    cfg_h = dict(cfg, grid_dev=gh)
    truth_h, _, _ = art.render_uniform(cfg_h)
    search = []
    for z in DEPLOY_Z:
        img_h, _, _, st_h = art.render_learned(cfg_h, net, out=bufs, z_propose=z, fallback=False)
        search.append(dict(z_propose=z, mse=art.metrics(truth_h[0], img_h[0])[1], rays=st_h["rays"]))
    del truth_h, gh, cfg_h
    torch.cuda.empty_cache()
    z_h = deploy_threshold(search)
    opts = dict(z_propose=z_h, fallback=False)
    (img, lev, ft, st), dt = timed(lambda: art.render_learned(cfg, net, out=bufs, **opts))
    fe, mse = art.metrics(truth[0], img[0])
    out["learned_judge_heldout_z"] = dict(
        ms=dt * 1e3, rays=st["rays"], passes=st["trace_launches"], mse=mse, flux_error=fe,
        effective_px_per_s=nx * ny / dt, rays_per_s=st["rays"] / dt, judge=st["learned"], options=opts,
        subrings=sub_flux(img), subring_mse=sub_mse(img), heldout_seed=DEPLOY_HELDOUT_SEED, heldout_search=search,
        vs_plain=dict(ms=dt * 1e3 / out["plain"]["ms"], rays=st["rays"] / out["plain"]["rays"]))
    log("16385^2 learned_judge at z = %g (held-out snapshot %s): %.0f ms, %d rays, %d passes, mse %.2e, "
        "subring mse %s" % (z_h, ["%g: %.2e" % (r["z_propose"], r["mse"]) for r in search], dt * 1e3,
                            st["rays"], st["trace_launches"], mse,
                            ["%.2e" % x for x in out["learned_judge_heldout_z"]["subring_mse"]]))
    img = img_keep
    net.close()
    out["visibility"] = deploy_visibility(art, torch, art_inputs, cfg, img, truth)
    del bufs, truth, img, lev, ft, g
    torch.cuda.empty_cache()
    return out


def deploy_visibility(art, torch, art_inputs, cfg, img, truth):
    """Visibility domain of the learned 16385^2 render (Sec. 4.3): the 2D
    window |u|, |v| <= 1000 G-lambda (Sgr A* mass and distance) on the
    1/FOV grid, u >= 0 half plane, taper FWHM = FOV/4, for Stokes I and the
    four subring planes, and for the residual image (learned - uniform)."""
    fov = float(cfg["fov"])
    ny, nx = img.shape[1], img.shape[2]
    dx = fov / (nx - 1)
    per_gl = art_inputs.glambda_to_inv_m(1.0)            # cycles per M per G-lambda
    du = 1.0 / fov
    k = int(np.floor(art_inputs.glambda_to_inv_m(1000.0) / du + 1e-9))
    u = torch.arange(0, k + 1, dtype=torch.float64, device="cuda") * du
    v = torch.arange(-k, k + 1, dtype=torch.float64, device="cuda") * du
    P = img.shape[0]
    art.visibility(img, dx, u, v, fwhm=fov / 4)          # warm (workspace in the caching allocator)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    V = art.visibility(img, dx, u, v, fwhm=fov / 4)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nu, nv = u.numel(), v.numel()
    flops = 2.0 * P * (ny * nx * 2.0 * nu + 2.0 * nu * ny * 2.0 * nv)
    resid = (img[0] - truth[0]).unsqueeze(0).contiguous()
    Vr = art.visibility(resid, dx, u, v, fwhm=fov / 4)[0]
    Vt = art.visibility(truth[0:1].contiguous(), dx, u, v, fwhm=fov / 4)[0]
    torch.cuda.synchronize()
    A = V.abs()
    ratio = (Vr.abs() / Vt.abs().clamp_min(1e-300)).flatten()
    q = torch.quantile(ratio[torch.randperm(ratio.numel(), device="cuda")[:1 << 20]],
                       torch.tensor([0.5, 0.99], dtype=torch.float64, device="cuda")).cpu().tolist()
    uaxis = A[:, k, :].cpu().numpy()                     # |V(u, 0)| per plane
    vaxis = A[:, :, 0].cpu().numpy()[:, k:]              # |V(0, v)|, v >= 0
    ug = u.cpu().numpy() / per_gl

    def envelope(a, w=9):
        pad = np.pad(a, w // 2, mode="edge")
        return np.lib.stride_tricks.sliding_window_view(pad, w).max(-1)

    def crossings(ax):
        # first baseline where the envelope of subring s+1 exceeds that of subring s
        out = []
        for s_ in range(P - 2):
            idx = np.nonzero(envelope(ax[2 + s_]) > envelope(ax[1 + s_]))[0]
            out.append(float(ug[idx[0]]) if idx.size else None)
        return out

    # ring period (Sec. 4.3.1): |V(u, 0)| of a ring of diameter d oscillates
    # with period 1/d (two limbs: |V|^2 = A1^2 + A2^2 + 2 A1 A2 cos(2 pi u d));
    # d is read off as the dominant oscillation of |V(u, 0)|^2 over
    # 50-800 G-lambda for subrings n = 2 and 3 of the adaptive and the uniform
    # render, and compared with the image-domain diameter (peak separation of
    # their projections onto the u direction)
    uf = torch.linspace(50.0 * per_gl, 800.0 * per_gl, 8001, dtype=torch.float64, device="cuda")
    dfu = float(uf[1] - uf[0])

    def ring_d(plane_img):
        a = art.visibility(plane_img.unsqueeze(0).contiguous(), dx, uf, [0.0], fwhm=fov / 4)[0, 0]
        p2 = (a.abs() ** 2).cpu().numpy()
        sig = (p2 - p2.mean()) * np.hanning(p2.size)
        spec = np.abs(np.fft.rfft(sig, 8 * sig.size))
        xs = np.fft.rfftfreq(8 * sig.size, dfu)
        ok = xs > 2.0
        return float(xs[ok][np.argmax(spec[ok])])
    d_vis = {"adaptive_n2": ring_d(img[3]), "adaptive_n3": ring_d(img[4]),
             "uniform_n2": ring_d(truth[3]), "uniform_n3": ring_d(truth[4])}
    xg = (np.arange(nx) - 0.5 * (nx - 1)) * dx
    d_img = []
    for pl in (3, 4):
        pr = img[pl].sum(dim=0).cpu().numpy()
        d_img.append(float(xg[np.argmax(np.where(xg > 0, pr, -1.0))] - xg[np.argmax(np.where(xg < 0, pr, -1.0))]))
    res = dict(window_glambda=1000.0, nu=nu, nv=nv, planes=P, taper_fwhm=fov / 4, ms=ms,
               tflops=flops / ms / 1e9, frac_fp64_peak=flops / ms / 1e9 / (PEAK_FP64_MATRIX / 1e12),
               residual_ratio_median=q[0], residual_ratio_p99=q[1],
               residual_ratio_u_axis_max=float((Vr.abs()[k] / Vt.abs()[k]).max()),
               u_axis_samples_glambda=[0, 100, 250, 500, 1000],
               u_axis_amplitude=[[float(uaxis[p][int(round(g * per_gl / du))]) for g in (0, 100, 250, 500, 1000)]
                                 for p in range(P)],
               subring_dominance_u_glambda=crossings(uaxis), subring_dominance_v_glambda=crossings(vaxis),
               ring_diameter_from_visibility_m=d_vis, ring_diameter_from_image_m=d_img)
    log("16385^2 visibilities: %d planes x %d x %d baselines in %.1f ms (%.1f TFLOP/s), residual/|V| "
        "median %.2e p99 %.2e, ring diameter %s M (image: %s), subring dominance along u at %s G-lambda" % (
            P, nv, nu, ms, res["tflops"], q[0], q[1], {k: round(v, 2) for k, v in d_vis.items()},
            ["%.2f" % x for x in d_img],
            ["%.0f" % x if x is not None else None for x in res["subring_dominance_u_glambda"]]))
    del V, Vr, Vt, resid
    return res


def in_flight_ms(art, torch, make, steps, depth=3):
    """Time per batch (ms) with `depth` batches from make() in flight on
    library streams, one image group each at the 256 x 256 persistent grid,
    every batch a captured graph."""
    Ss = [art.Stream() for _ in range(depth)]
    Bs = [make() for _ in range(depth)]
    for X in Bs:
        X.set_launch(256, 256, 1, 1)
    dt = time_pipelined(Bs, torch, [S.torch for S in Ss], steps)
    for X in Bs:
        X.close()
    for S in Ss:
        S.close()
    return dt * 1e3


def spectral_1025(art, torch, art_inputs, args):
    """Adaptive sampling along frequency (the Sec. 6 extension): the
    thermal_1025 view as a 17-frequency cube from 86 to 690 GHz (3 base
    frequencies, 3 spectral levels), against plain adaptive renders of the
    same 17 frequencies (one batch, hipGraph replay) and uniform truths."""
    from paper_2103_07417_amd import art as A
    cfg = dict(art_inputs.workload("thermal_1025"), precision=args.precision)
    n0, L = 3, 3
    lo, hi = 86e9, 690e9
    n = A.cube_size(n0, L)
    nus = [lo * (hi / lo) ** (i / (n - 1.0)) for i in range(n)]
    truths = []
    for nu in nus:
        t, _, _ = art.render_uniform(dict(cfg, freq_hz=nu))
        truths.append(t[0].clone())
    art.render_spectral(cfg, lo, hi, n0, L)              # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    imgs, levs, _, sts = art.render_spectral(cfg, lo, hi, n0, L)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rays = sum(st["rays"] for st in sts)
    spec = sum(st["spectral"] for st in sts)
    mses = [art.metrics(truths[i], imgs[i][0])[1] for i in range(n)]
    cube = dict(ms=sts[0]["t_render_ms"], wall_ms=wall * 1e3, rays=rays, spectral_values=spec,
                passes=sts[0]["trace_launches"], mse_max=max(mses), mse_mean=sum(mses) / n,
                mse_ok=max(mses) <= 1e-3)
    del imgs, levs
    cfgs = [dict(cfg, name="nu_%02d" % i, freq_hz=nu) for i, nu in enumerate(nus)]
    B = art.Batch(cfgs)
    s = torch.cuda.Stream()
    B.render(s)
    s.synchronize()
    dt = time_graph(B, torch, s, 3)
    st = B.stats(stream=s)
    chk = mse_check(art, cfgs, B.images, truths)
    plain = dict(ms=dt * 1e3, rays=st["rays"], passes=st["trace_launches"], mse_max=chk["mse_max"],
                 mse_mean=chk["mse_mean"], mse_ok=chk["mse_ok"])
    B.close()
    # throughput: three cubes / three plain batches in flight
    cube["ms_in_flight"] = in_flight_ms(art, torch, lambda: art.Batch(cfgs, cube=(n0, L, cfg["r_rel"],
                                                                                    cfg["r_abs"])), args.steps)
    plain["ms_in_flight"] = in_flight_ms(art, torch, lambda: art.Batch(cfgs), args.steps)
    log("spectral cube in flight: %.1f ms per cube, plain %.1f ms per batch (3 in flight)" % (
        cube["ms_in_flight"], plain["ms_in_flight"]))
    out = dict(workload="thermal_1025 view (a=0.94, i=163 deg, IQUV) at %d frequencies 86-690 GHz equally "
                        "spaced in ln nu (3 base + 3 spectral levels), 1025^2, R_rel=0.01, R_abs=1e-3 max I0 "
                        "on both axes" % n,
               cube=cube, plain_batched=plain, rays_ratio=rays / max(plain["rays"], 1))
    log("spectral cube %d x 1025^2: %.1f ms (wall %.1f), %d rays (+%d spectral values), mse max %.2e; "
        "plain batch %.1f ms, %d rays, mse max %.2e" % (n, cube["ms"], cube["wall_ms"], rays, spec,
                                                       cube["mse_max"], plain["ms"], plain["rays"],
                                                       plain["mse_max"]))
    return out


MOVIE_RABS = (1.0, 0.5, 0.25)   # R_abs of both axes as fractions of the paper's 0.025 Ibar_int


def movie_1025(art, torch, art_inputs, args):
    """Adaptive sampling in time (the Sec. 6 extension): 9 snapshots of the
    evolving synthetic flow at the paper's 5 M cadence (t = 0..40 M), gridded
    model, 1025^2 (base 129^2, 3 levels), Stokes I, as a cube along t (3 base
    frames, 2 levels) against plain adaptive renders of the 9 frames (one
    batch, hipGraph replay) and uniform truths.  R_abs (both axes) is chosen
    on a held-out movie (the turbulence of another seed) as the loosest of
    MOVIE_RABS x 0.025 Ibar_int at which its 9 cube frames pass the bar, then
    applied unchanged to the cube and the plain renders of the timed movie."""
    from art_inputs import mks
    times = [5.0 * k for k in range(9)]
    base0 = dict(art_inputs.workload("grid_4097"), nx0=129, ny0=129, levels=3, nstokes=1,
                 precision=args.precision)

    def movie(seed, base):
        grids, _ = mks.mks_movie(times, seed=seed)
        gd = [torch.from_numpy(g).cuda() for g in grids]
        del grids
        cf = [dict(base, name="t%03d" % int(t), grid_dev=g) for t, g in zip(times, gd)]
        tr = []
        for c in cf:
            t, _, _ = art.render_uniform(c)
            tr.append(t[0].clone())
        return gd, cf, tr
    gh, cfh, trh = movie(5, base0)
    held = []
    ra = base0["r_abs"] * MOVIE_RABS[-1]
    for f in MOVIE_RABS:
        ra_f = base0["r_abs"] * f
        cf = [dict(c, r_abs=ra_f) for c in cfh]
        im, _, _, sth = art.render_cube(cf, 3, 2)
        m = max(art.metrics(trh[i], im[i][0])[1] for i in range(len(cf)))
        held.append(dict(r_abs=ra_f, mse_max=m, rays=sum(x["rays"] for x in sth)))
        del im
        if m <= 1e-3:
            ra = ra_f
            break
    del gh, cfh, trh
    log("movie: R_abs chosen on the held-out movie: %g (%s)" % (ra, ["%.2e" % h["mse_max"] for h in held]))
    base = dict(base0, r_abs=ra)
    gdev, cfgs, truths = movie(2, base)
    art.render_cube(cfgs, 3, 2)                          # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    imgs, levs, _, sts = art.render_cube(cfgs, 3, 2)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rays = sum(st["rays"] for st in sts)
    spec = sum(st["spectral"] for st in sts)
    mses = [art.metrics(truths[i], imgs[i][0])[1] for i in range(len(cfgs))]
    cube = dict(ms=sts[0]["t_render_ms"], wall_ms=wall * 1e3, rays=rays, axis_values=spec,
                passes=sts[0]["trace_launches"], mse_max=max(mses), mse_mean=sum(mses) / len(mses),
                mse_ok=max(mses) <= 1e-3)
    del imgs, levs
    B = art.Batch(cfgs)
    s = torch.cuda.Stream()
    B.render(s)
    s.synchronize()
    dt = time_graph(B, torch, s, 3)
    st = B.stats(stream=s)
    chk = mse_check(art, cfgs, B.images, truths)
    plain = dict(ms=dt * 1e3, rays=st["rays"], passes=st["trace_launches"], mse_max=chk["mse_max"],
                 mse_mean=chk["mse_mean"], mse_ok=chk["mse_ok"])
    B.close()
    cube["ms_in_flight"] = in_flight_ms(art, torch, lambda: art.Batch(cfgs, cube=(3, 2, base["r_rel"], ra)),
                                        args.steps)
    plain["ms_in_flight"] = in_flight_ms(art, torch, lambda: art.Batch(cfgs), args.steps)
    log("movie cube in flight: %.1f ms per cube, plain %.1f ms per batch (3 in flight)" % (
        cube["ms_in_flight"], plain["ms_in_flight"]))
    log("movie cube 9 x 1025^2: %.1f ms, %d rays (+%d values from neighbouring frames), mse max %.2e; "
        "plain batch %.1f ms, %d rays, mse max %.2e" % (cube["ms"], rays, spec, cube["mse_max"], plain["ms"],
                                                       plain["rays"], plain["mse_max"]))
    del gdev, truths
    torch.cuda.empty_cache()
    return dict(workload="gridded snapshot movie a=0.94 i=163 deg 230 GHz, 9 frames at 5 M cadence "
                         "(Keplerian-sheared turbulence renewed over 200 M), 1025^2, Stokes I, R_rel=1e-3, "
                         "R_abs=%g Ibar_int on both axes (chosen on a held-out movie), 3 base frames + 2 levels "
                         "in time" % ra,
                cube=cube, plain_batched=plain, rays_ratio=rays / max(plain["rays"], 1), r_abs_heldout=held)


def refine_variants(art, torch, cfg, args):
    """The refinement variants on the thermal_1025 view, one image at a time:
    the linear branch of Eqs. 5-6 (the paper's method), the nearest-neighbour
    branch, and the linear branch with the criterion on every Stokes plane;
    time, rays and the MSE of every plane against the uniform render."""
    truth, _, _ = art.render_uniform(cfg)
    truth = truth.clone()
    torch.cuda.synchronize()
    out = {}
    for name, kw in (("linear", {}), ("nearest", dict(interp="nearest")), ("linear_all_planes", dict(all_planes=True))):
        c = dict(cfg, **kw)
        bufs = art.alloc(c)
        art.render(c, out=bufs)
        torch.cuda.synchronize()
        reps = max(3, args.steps // 3)
        t0 = time.perf_counter()
        for _ in range(reps):
            img, lev, _, st = art.render(c, out=bufs)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        mses = [art.metrics(truth[q], img[q])[1] for q in range(c["nstokes"])]
        out[name] = dict(ms=dt * 1e3, rays=st["rays"], interp_frac=st["interp_frac"], mse_iquv=mses)
        log("refinement %s: %.1f ms, %d rays, IF %.4f, mse I,Q,U,V %s" % (
            name, dt * 1e3, st["rays"], st["interp_frac"], ["%.2e" % m for m in mses]))
        del bufs, img, lev
    return out


def plain_single(art, torch, cfg, args):
    """The paper's method, one image at a time, and the uniform render."""
    truth, _, ust = art.render_uniform(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    truth, _, ust = art.render_uniform(cfg)
    torch.cuda.synchronize()
    t_uniform = time.perf_counter() - t0
    bufs = art.alloc(cfg)
    for _ in range(args.warmup):
        art.render(cfg, out=bufs)
    torch.cuda.synchronize()
    rays = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        img, lev, _, st = art.render(cfg, out=bufs)
        rays += st["rays"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    fe, mse = art.metrics(truth[0], img[0])
    nx, ny = img.shape[2], img.shape[1]
    plain = dict(ms_per_image=dt * 1e3, rays=rays // args.steps, passes=st["trace_launches"],
                 rays_per_s=rays / args.steps / dt, effective_px_per_s=nx * ny / dt,
                 interp_frac=st["interp_frac"], mse=mse, flux_error=fe)
    uniform = dict(ms=t_uniform * 1e3, rays=ust["rays"], steps=ust["steps"], steps_emit=ust["steps_emit"],
                   rays_per_s=ust["rays"] / t_uniform, effective_px_per_s=nx * ny / t_uniform)
    return plain, uniform


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "mixed_geo"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-1core-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--in-flight", type=int, default=0, choices=[0, 1, 2, 3, 4],
                    help="batches in flight in the timed step (0: autotuned over 2-4)")
    ap.add_argument("--launch", default="",
                    help="persistent-tracer shape BLOCKSxTHREADS[:REFINE_BLOCKS] of the timed forms instead of the "
                         "in-flight autotuner (with --in-flight, else three batches in flight)")
    ap.add_argument("--refill", type=int, default=1,
                    help="refill threshold of the timed forms with --launch (lanes idle before a wave claims rays)")
    ap.add_argument("--long-steps", type=int, default=0,
                    help="long-ray threshold of the refinement queues of the timed forms with --launch (0: 800)")
    ap.add_argument("--learned-form", default="",
                    help="learned form timed on the headline batch instead of the fastest on the held-out "
                         "batch (for counter runs, whose serialised dispatches change the held-out timings)")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--no-deploy", action="store_true")
    ap.add_argument("--no-spectral", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--z-propose", type=float, default=0.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import art_inputs
    from paper_2103_07417_amd import art

    cfg = dict(art_inputs.workload("thermal_1025"), precision=args.precision)
    nx, ny = art.image_size(cfg)
    plain, uniform = plain_single(art, torch, cfg, args)
    log("thermal view, plain one image at a time: %.1f ms/image, %d rays, mse %.2e; uniform %.1f ms" % (
        plain["ms_per_image"], plain["rays"], plain["mse"], uniform["ms"]))
    forms, head, training, npix, rs, search, policies = c4_forms(art, torch, art_inputs, args)
    L = forms[head]
    P = forms["plain_batched"]
    achieved = (rs["flops"] / rs["launches"]) / (rs["tr_ms"] / rs["launches"] * 1e-3)
    traffic = measured_traffic(rs["launches"], L["form"], args.precision)
    roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_VECTOR / 1e12, unit="TFLOP/s",
                frac=achieved / PEAK_VECTOR, traffic=traffic and traffic["bytes_per_launch"],
                kernel="k_trace (%s), %s render" % (PRECISION_NAMES[args.precision], head),
                launches=rs["launches"], renders=ROOF_RENDERS,
                avg_launch_ms=rs["tr_ms"] / rs["launches"],
                flops_per_launch=rs["flops"] / rs["launches"],
                algorithmic_bytes_per_launch=rs["rays"] * BYTES_PER_RAY / rs["launches"],
                achieved_structured=(rs["flops_structured"] / rs["launches"]) /
                                    (rs["tr_ms"] / rs["launches"] * 1e-3) / 1e12,
                achieved_whole_render=rs["flops"] / (rs["render_ms"] * 1e-3) / 1e12,
                achieved_pipelined=rs["flops"] / ROOF_RENDERS / (L["ms_per_batch"] * 1e-3) / 1e12,
                frac_pipelined=rs["flops"] / ROOF_RENDERS / (L["ms_per_batch"] * 1e-3) / PEAK_VECTOR,
                traffic_source=traffic and traffic["source"],
                note="achieved = operations counted by the oracle's instrumented build (per geodesic step, "
                     "emitting and non-emitting step) x this render's step counts / mean tracing-launch "
                     "duration (HIP events around each launch of two eager renders, one image group); "
                     "achieved_structured counts the tracer's own structured forms instead; "
                     "achieved_pipelined = the same operations per batch / the timed step with %d batches in "
                     "flight (the chip-level rate).  peak: FP64 vector rate, which is also the rate of "
                     "unpacked FP32 (this code is built without packed FP32)" % L["in_flight"])
    out = {
        "metric": METRIC, "value": L["rays_per_s"], "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": L["ms_per_batch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f64-geodesic/f32-transfer",
                  "mixed_geo": "f64/f32-geodesic/f32-transfer"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "batched uneven refinement: 64 thermal images (a in {0,0.5,0.94,-0.94} x "
                               "i in {17,60,90,163} deg x nu in {86,230,345,690} GHz), IQUV, base 129^2, "
                               "image k refined 1 + (k mod 4) levels (257^2..2049^2, %d effective px), "
                               "R_abs=1e-3 max I0, R_rel chosen on a held-out batch, one hipGraph replay "
                               "per batch, %d batches in flight" % (npix, L["in_flight"]),
                   "images": 64, "base": 129, "levels": "1-4", "precision": args.precision,
                   "form": head, "r_rel": L["r_rel"], "options": L.get("options")},
        "effective_px_per_s": L["effective_px_per_s"],
        "image_mse_vs_uniform_max": L["check"]["mse_max"], "mse_ok": L["check"]["mse_ok"],
        "mse_max_planes_iquv": L["check"].get("mse_max_planes"),
        "ms_per_step_range": L["ms_range"],
        "learned_batched_vs_plain_batched": {
            "plain_form": "plain_batched", "plain_r_rel": P["r_rel"], "plain_chosen_by": P["chosen_by"],
            "effective_px_per_s": L["effective_px_per_s"] / P["effective_px_per_s"],
            "rays": L["rays"] / P["rays"], "steps": L["steps"] / P["steps"],
            "plain_mse_ok": P["check"]["mse_ok"], "learned_mse_ok": L["check"]["mse_ok"]},
        "learned_batched_vs_plain_single": {
            "effective_px_per_s": L["effective_px_per_s"] / plain["effective_px_per_s"]},
        "forms": forms,
        "operating_point_search": search,
        "plain": plain,
        "uniform": uniform,
        "training": training,
        "roofline": roof,
        "precision_policies": policies,
    }
    if "plain_batched_own_op" in forms:
        O = forms["plain_batched_own_op"]
        out["learned_batched_vs_plain_own_op"] = {
            "plain_r_rel": O["r_rel"], "effective_px_per_s": L["effective_px_per_s"] / O["effective_px_per_s"],
            "rays": L["rays"] / O["rays"], "steps": L["steps"] / O["steps"]}
    if not args.no_grid:
        out["grid_4097"] = grid_forms(art, torch, art_inputs, args)
    if not args.no_deploy:
        out["deploy_16385"] = deploy_16385(art, torch, art_inputs, args)
    if not args.no_spectral:
        out["spectral_1025"] = spectral_1025(art, torch, art_inputs, args)
        out["movie_1025"] = movie_1025(art, torch, art_inputs, args)
    if not args.no_variants:
        out["refinement_variants"] = refine_variants(art, torch, cfg, args)
    # a plain device copy of known size: reference reading for the HBM byte
    # counters (FETCH_SIZE / WRITE_SIZE) of a profiled run
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_calibration_bytes"] = COPY_BYTES
    out["kernel_hash"] = kernel_hash()
    del src, dst
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline([dict(c, r_rel=L["r_rel"]) for c in
                                            art_inputs.batch_workload(precision="fp64")],
                                           args.cpu_seconds, args.cpu_1core_seconds)
    print(json.dumps(finite(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
