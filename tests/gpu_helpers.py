"""Shared helpers of the GPU parity tests (HIP path vs CPU oracle).

Decision protocol (Sec. 3.2 decision rule): the oracle is replayed with the
GPU's level map, computing every ray itself, and at every candidate point it
also evaluates its own rule on its own values (given the same history).
Wherever the GPU's decision differs from that, the oracle's tie margin --
the smallest relative perturbation of the values the rule reads that could
change the decision -- must lie below eta: 1e-9 for the FP64 path (per-ray
values agree to ~1e-13 there), larger for reduced precision.  The image is
then compared with the replay.
"""
import numpy as np

from oracle import ray as oray
from oracle import refine as oref

ETA_FP64 = 1e-9
# reduced precision: FP32 transfer moves per-ray values by ~1e-7..1e-6
# relative (FP32 rounding accumulated over 10^2..10^3 emitting steps; the
# largest margin among differing decisions measured at full size is 1.8e-6);
# a decision a 1e-4 relative change of its inputs can flip counts as a tie
ETA_MIXED = 1e-4


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return np.sqrt(np.sum((a - b) ** 2)) / (den if den > 0 else 1.0)


def nmse(a, b):
    """Normalised MSE (Eq. 9) of a against the reference b."""
    return rel_l2(a, b) ** 2


def oracle_adaptive(cfg, forced=None, grid=None):
    fn = lambda x, y: oray.trace(cfg, x, y, grid=grid)[0]
    planes = cfg["nstokes"] + cfg.get("subrings", 0)
    return oref.refine(fn, cfg["fov"], cfg["nx0"], cfg["ny0"], cfg["levels"], cfg["r_rel"],
                       cfg["r_abs"], cfg["abs_norm"], planes, forced_level=forced,
                       interp=cfg.get("interp", "linear"), all_planes=cfg.get("all_planes", False))


def check_ties(res, level_map, eta, tau_z=None, state_of=None, label=""):
    """Every decision of level_map that differs from the oracle's own rule in
    the forced replay `res` must sit at a tie: criterion margin < eta, or,
    for a learned render, the logit within tau_z of a proposal threshold.
    Returns the number of differing decisions."""
    n, bad, worst = 0, [], 0.0
    for a in res["audit"]:
        given = level_map[a["j"], a["i"]]
        if state_of is not None:
            given = state_of(given)
        d = np.nonzero(given != a["own"])[0]
        n += d.size
        m = a["margin"][d]
        ok = m < eta
        if tau_z is not None and "zmargin" in a:
            ok |= a["zmargin"][d] < tau_z
        worst = max(worst, float(m.max()) if d.size else 0.0)
        for k in d[~ok]:
            bad.append((int(a["i"][k]), int(a["j"][k]), int(a["own"][k]), int(given[k]),
                        float(a["margin"][k]), float(a.get("zmargin", np.full(1, np.inf))[k]
                                                         if "zmargin" in a else np.inf)))
    print("decisions differing from the oracle's own rule%s: %d (largest margin %.3g)"
          % (label, n, worst), flush=True)
    assert not bad, ("decisions off a tie (i, j, own, gpu, margin, logit gap)", bad[:10])
    return n


def check_adaptive(art, cfg, img_tol, grid=None, eta=ETA_FP64, render=None):
    """Adaptive GPU render vs the oracle: every decision the oracle's own rule
    would take differently sits at a tie (margin < eta), and the image agrees
    with the oracle's replay of the GPU's level map to relative L2 img_tol
    per plane.  Returns (gpu image, level map, stats, replay)."""
    img, lev, _, st = render() if render is not None else art.render(cfg)
    g = img.cpu().numpy()
    gl = lev.cpu().numpy()
    o = oracle_adaptive(cfg, forced=gl, grid=grid)
    check_ties(o, gl, eta)
    for s in range(cfg["nstokes"] + cfg.get("subrings", 0)):
        assert rel_l2(g[s], o["img"][s]) <= img_tol, (s, rel_l2(g[s], o["img"][s]))
    assert st["rays"] == int((gl >= 0).sum())
    assert abs(st["interp_frac"] - float((gl < 0).mean())) <= 1e-15
    return g, gl, st, o
