"""Launch-shape autotuner for the persistent tracer.

Times a batch's adaptive render (HIP events on the render stream) over a small
grid of launch shapes -- image groups rendered concurrently, blocks per CU
multiple, threads per block, refill threshold -- keeps the fastest, and caches
the choice per (device, batch signature) in a JSON file.
"""
import hashlib
import json
import os
import time

from . import art

CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                     "art", "autotune.json")


def signature(cfgs):
    keys = ("model", "nstokes", "precision", "nx0", "ny0", "levels", "a", "inc_deg", "freq_hz",
            "r_rel", "r_abs", "eps")
    blob = json.dumps([[c.get(k) for k in keys] for c in cfgs], sort_keys=True)
    return hashlib.sha1(blob.encode()).hexdigest()[:16]


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def time_render(batch, torch, stream, reps):
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        with torch.cuda.stream(stream):
            start.record(stream)
            batch.render(stream)
            stop.record(stream)
        stop.synchronize()
        best = min(best, start.elapsed_time(stop))
    return best


def autotune(batch, stream=None, reps=2, use_cache=True, log=None):
    """Pick and apply the fastest launch shape for `batch`.  Returns a dict
    with the chosen shape, its time and the full search table."""
    import torch
    stream = stream or torch.cuda.current_stream()
    dev = torch.cuda.get_device_name(0)
    key = dev + "/" + signature(batch.cfgs)
    cache = _load() if use_cache else {}
    if key in cache and "groups" in cache[key]:
        c = cache[key]
        batch.set_launch(c["trace_blocks"], c["trace_threads"], c["refill"], c["groups"])
        return dict(c, cached=True)
    default = batch.get_launch()
    threads0 = default["trace_threads"]
    per_cu = max(1, default["trace_blocks"] // max(1, torch.cuda.get_device_properties(0).multi_processor_count))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    table = []
    t0 = time.perf_counter()
    batch.render(stream)            # warm-up (code objects, caches)
    stream.synchronize()
    n = len(batch.cfgs)
    group_choices = sorted({g for g in (1, 2, 4, 8) if g <= n})
    for groups in group_choices:
        for threads in (128, 256):
            blocks_per_cu = max(1, per_cu * threads0 // threads)
            for mult in (0.25, 0.5, 1, 2):
                blocks = max(1, int(round(cus * blocks_per_cu * mult)))
                for refill in (1, 16):
                    batch.set_launch(blocks, threads, refill, groups)
                    ms = time_render(batch, torch, stream, reps)
                    table.append(dict(trace_blocks=blocks, trace_threads=threads, refill=refill,
                                      groups=groups, ms=ms))
                    if log:
                        log("autotune groups=%d blocks=%d threads=%d refill=%d: %.2f ms"
                            % (groups, blocks, threads, refill, ms))
    best = min(table, key=lambda r: r["ms"])
    batch.set_launch(best["trace_blocks"], best["trace_threads"], best["refill"], best["groups"])
    out = dict(trace_blocks=best["trace_blocks"], trace_threads=best["trace_threads"],
               refill=best["refill"], groups=best["groups"], ms=best["ms"], default=default,
               default_ms=next((r["ms"] for r in table if r["trace_threads"] == threads0
                                and r["trace_blocks"] == default["trace_blocks"]
                                and r["refill"] == default["refill"]
                                and r["groups"] == default["groups"]), None),
               search_s=time.perf_counter() - t0)
    if use_cache:
        cache = _load()
        cache[key] = {k: out[k] for k in ("trace_blocks", "trace_threads", "refill", "groups", "ms")}
        _store(cache)
    out["table"] = table
    out["cached"] = False
    return out


def time_in_flight(batches, torch, streams, reps):
    """Time per batch with the batches replayed round robin, each on its own
    stream (graphs captured first); the clock stops when every stream is done."""
    for b, s in zip(batches, streams):
        b.capture(s)
    for b, s in zip(batches, streams):
        b.launch(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(reps):
        batches[k % len(batches)].launch(streams[k % len(batches)])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def median_in_flight(batches, torch, streams, reps, k=3):
    """Median of k in-flight timings: a shape whose time scatters between
    replays is judged by its typical time, not its best."""
    return sorted(time_in_flight(batches, torch, streams, reps) for _ in range(k))[k // 2]


def autotune_in_flight(batches, streams, depths=None, reps=None, log=None):
    """Launch shape and depth for batches in flight (one image group each, the
    streams take the groups' role): with d batches in flight each batch's
    persistent grid should fill only its share of the chip so the batches
    co-reside.  For every depth d in `depths` (default: all the batches)
    the first d batches are replayed round robin on the first d streams,
    searching blocks per CU (256-thread blocks; every candidate timed as the
    median of three replays of the batches); then, at the fastest
    (depth, shape), smaller grids for the refinement passes (7/8 and 3/4 of
    the base grid: fewer waves left with idle lanes once a pass's queue has
    drained, while the other batches take the freed slots) crossed with
    refill thresholds 1, 2, 4, 8 (a wave that waits for a few idle lanes
    starts their rays with one pass through the ray set-up instead of one
    per termination); then, at that choice, the long-ray threshold of the
    refinement queues (600, 700, 900 besides the default 800: the points
    queued at the front should be about as many as the lanes that start
    them); last, a larger grid for the base pass alone (5/4, 3/2, 2 of it,
    the refinement grid kept).  The fastest choice is applied to every batch.
    Returns the choice and the table."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    depths = tuple(depths or (len(batches),))
    if max(depths) > len(batches) or max(depths) > len(streams) or min(depths) < 1:
        raise ValueError("depths %s need as many batches and streams" % (depths,))
    table = []
    t0 = time.perf_counter()
    for d in depths:
        n = reps or max(4, 2 * d)
        # 256-thread blocks only: with batches in flight, 128-thread shapes
        # timed well here and then ran 10-15 % slower and unevenly in the
        # longer timed replays
        for threads in (256,):
            for waves_per_cu in (4, 8, 12, 16):
                blocks = max(1, cus * waves_per_cu * 64 // threads)
                for b in batches[:d]:
                    b.set_launch(blocks, threads, 1, 1)
                ms = median_in_flight(batches[:d], torch, streams[:d], n)
                table.append(dict(in_flight=d, trace_blocks=blocks, trace_threads=threads, refill=1, groups=1,
                                  ms=ms))
                if log:
                    log("autotune in flight depth=%d blocks=%d threads=%d: %.2f ms/batch"
                        % (d, blocks, threads, ms))
    best = dict(min(table, key=lambda r: r["ms"]), refine_blocks=0)
    d = best["in_flight"]
    # the later stages' differences are a few percent: longer timings, and
    # the first stage's row timed again the same way
    n = reps or max(12, 4 * d)
    for b in batches[:d]:
        b.set_launch(best["trace_blocks"], best["trace_threads"], 1, 1)
    best = dict(best, ms=median_in_flight(batches[:d], torch, streams[:d], n))
    table.append(best)
    for frac in (1.0, 0.875, 0.75):
        rb = max(1, int(round(best["trace_blocks"] * frac)))
        for refill in (1, 2, 4, 8):
            if frac == 1.0 and refill == 1:
                continue                      # the first stage's row
            for b in batches[:d]:
                b.set_launch(best["trace_blocks"], best["trace_threads"], refill, 1, refine_blocks=rb)
            ms = median_in_flight(batches[:d], torch, streams[:d], n)
            table.append(dict(best, refine_blocks=rb, refill=refill, ms=ms))
            if log:
                log("autotune in flight depth=%d blocks=%d threads=%d refine_blocks=%d refill=%d: %.2f ms/batch"
                    % (d, best["trace_blocks"], best["trace_threads"], rb, refill, ms))
    best = min(table[-12:], key=lambda r: r["ms"])
    best = dict(best, refine_blocks=best.get("refine_blocks", 0), long_steps=0)
    for ls in (600, 700, 900):
        for b in batches[:d]:
            b.set_launch(best["trace_blocks"], best["trace_threads"], best["refill"], 1,
                         refine_blocks=best["refine_blocks"], long_steps=ls)
        ms = median_in_flight(batches[:d], torch, streams[:d], n)
        table.append(dict(best, long_steps=ls, ms=ms))
        if log:
            log("autotune in flight depth=%d blocks=%d threads=%d refine_blocks=%d refill=%d long_steps=%d: "
                "%.2f ms/batch" % (d, best["trace_blocks"], best["trace_threads"], best["refine_blocks"],
                                   best["refill"], ls, ms))
    best = min([best] + table[-3:], key=lambda r: r["ms"])
    rb = best["refine_blocks"] or best["trace_blocks"]
    for mult in (1.25, 1.5, 2.0):
        tb = int(round(best["trace_blocks"] * mult))
        for b in batches[:d]:
            b.set_launch(tb, best["trace_threads"], best["refill"], 1, refine_blocks=rb,
                         long_steps=best["long_steps"])
        ms = median_in_flight(batches[:d], torch, streams[:d], n)
        table.append(dict(best, trace_blocks=tb, refine_blocks=rb, ms=ms))
        if log:
            log("autotune in flight depth=%d base blocks=%d threads=%d refine_blocks=%d refill=%d "
                "long_steps=%d: %.2f ms/batch" % (d, tb, best["trace_threads"], rb, best["refill"],
                                                  best["long_steps"], ms))
    best = min([best] + table[-3:], key=lambda r: r["ms"])
    for b in batches:
        b.set_launch(best["trace_blocks"], best["trace_threads"], best["refill"], 1,
                     refine_blocks=best["refine_blocks"], long_steps=best["long_steps"])
    return dict(best, search_s=time.perf_counter() - t0, table=table)
