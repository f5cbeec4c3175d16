"""Shared helpers of the GPU parity tests (HIP path vs CPU oracle)."""
import numpy as np

from oracle import ray as oray
from oracle import refine as oref


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return np.sqrt(np.sum((a - b) ** 2)) / (den if den > 0 else 1.0)


def oracle_adaptive(cfg, forced=None, grid=None):
    fn = lambda x, y: oray.trace(cfg, x, y, grid=grid)[0]
    planes = cfg["nstokes"] + cfg.get("subrings", 0)
    return oref.refine(fn, cfg["fov"], cfg["nx0"], cfg["ny0"], cfg["levels"], cfg["r_rel"],
                       cfg["r_abs"], cfg["abs_norm"], planes, forced_level=forced,
                       interp=cfg.get("interp", "linear"), all_planes=cfg.get("all_planes", False))


def check_adaptive(art, cfg, img_tol, grid=None):
    """Adaptive GPU render vs the oracle.  Decisions may differ only at
    floating-point ties (<= 1 per 10^4 points); the oracle is then replayed
    with the GPU's decisions and the images must agree to img_tol."""
    img, lev, _, st = art.render(cfg)
    g = img.cpu().numpy()
    gl = lev.cpu().numpy()
    o = oracle_adaptive(cfg, grid=grid)
    flips = int((gl != o["level"]).sum())
    if flips:
        assert flips <= max(2, gl.size // 10000), flips
        o = oracle_adaptive(cfg, forced=gl, grid=grid)
    for s in range(cfg["nstokes"] + cfg.get("subrings", 0)):
        assert rel_l2(g[s], o["img"][s]) <= img_tol, (s, rel_l2(g[s], o["img"][s]))
    assert st["rays"] == int((gl >= 0).sum())
    assert abs(st["interp_frac"] - o["interp_frac"]) <= flips / gl.size + 1e-15
    return g, gl, st, o
