"""Pins of the tie margins the oracle attaches to its refinement decisions.

A GPU level map may differ from the oracle's own decisions only at ties: at
points where a relative perturbation of the values the criterion reads, of
the size of the two implementations' rounding differences, could change the
decision.  The oracle reports, per decision, the smallest such perturbation
(the margin).  These tests check that the margin is a sound bound and that
the audit is consistent:

- an unforced render's audit equals its own level map at every point
  (linear and nearest branches, per-plane criterion, axis-sampled cubes,
  learned look-ahead);
- perturbing every ray value by a relative delta and replaying with the
  unperturbed level map, every decision that changes has margin <= delta,
  and with a delta large enough some decisions do change;
- a planted flip in a forced map is found with its margin.
"""
import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import learned as olearned
from oracle import refine
from oracle import spectral as osp


def field(x, y, seed=0):
    """Ring + blobs + a little structure: many decisions near the thresholds."""
    rng = np.random.default_rng(seed)
    rho = np.hypot(x, y)
    I = np.exp(-0.5 * ((rho - 6.0) / 0.8) ** 2) + 0.3 * np.exp(-rho ** 2 / 60.0)
    for _ in range(3):
        cx, cy = rng.uniform(-12, 12, 2)
        I += 0.2 * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / 4.0)
    return I


def ray_fn_for(seed=0, delta=0.0, nplanes=1):
    def fn(x, y):
        I = field(x, y, seed)
        if delta:
            # deterministic per-point relative perturbation in [-delta, delta]
            h = np.sin(12.9898 * x + 78.233 * y) * 43758.5453
            I = I * (1.0 + delta * (2.0 * (h - np.floor(h)) - 1.0))
        planes = [I, 0.3 * I * np.cos(0.2 * x), 0.2 * I * np.sin(0.3 * y), 0.05 * I][:nplanes]
        return np.stack(planes, -1)
    return fn


KW = dict(fov=40.0, nx0=9, ny0=9, levels=3, r_rel=0.02, r_abs=0.01)


def run(fn, nplanes=1, **kw):
    a = dict(KW, **kw)
    return refine.refine(fn, a["fov"], a["nx0"], a["ny0"], a["levels"], a["r_rel"], a["r_abs"],
                         "mean", nplanes, forced_level=kw.get("forced_level"),
                         interp=kw.get("interp", "linear"), all_planes=kw.get("all_planes", False))


@pytest.mark.parametrize("opts", [dict(), dict(interp="nearest"), dict(all_planes=True), dict(all_planes="own")])
def test_unforced_audit_equals_own_map(opts):
    nplanes = 4 if opts.get("all_planes") else 1
    out = run(ray_fn_for(1, nplanes=nplanes), nplanes, **opts)
    n, worst, _ = refine.disagreements(out, out["level"])
    assert n == 0
    m = np.concatenate([a["margin"] for a in out["audit"]])
    assert np.all(m >= 0) and np.isfinite(m).sum() > 100


@pytest.mark.parametrize("opts", [dict(), dict(interp="nearest"), dict(all_planes=True), dict(all_planes="own")])
@pytest.mark.parametrize("delta", [1e-9, 1e-6, 1e-3])
def test_decisions_changed_by_a_perturbation_have_smaller_margins(opts, delta):
    nplanes = 4 if opts.get("all_planes") else 1
    base = run(ray_fn_for(2, nplanes=nplanes), nplanes, **opts)
    pert = run(ray_fn_for(2, delta, nplanes), nplanes, forced_level=base["level"], **opts)
    n, worst, rows = refine.disagreements(pert, base["level"])
    assert worst <= delta * (1 + 1e-6), rows[:5]
    if delta >= 1e-3:
        assert n > 0          # the bound is not vacuous: large perturbations do flip


def test_planted_flip_is_found_with_its_margin():
    base = run(ray_fn_for(3))
    lev = base["level"].copy()
    a = base["audit"][2]
    k = int(np.argmax(np.where(np.isfinite(a["margin"]), a["margin"], -1)))
    i, j = a["i"][k], a["j"][k]
    lev[j, i] = -1 if lev[j, i] >= 0 else 2
    forced = run(ray_fn_for(3), forced_level=lev)
    n, worst, rows = refine.disagreements(forced, lev)
    assert n >= 1 and (int(i), int(j)) in [(r[0], r[1]) for r in rows]
    assert worst >= a["margin"][k] * 0.999


def test_spectral_cube_audit_and_perturbation():
    fn_nu = lambda d: (lambda nu: (lambda x, y: ray_fn_for(4, d)(x, y) * (nu / 230e9) ** -0.7
                                   * (1 + 0.05 * np.log(nu / 230e9) ** 2)))
    args = (40.0, 9, 9, 2, 0.02, 0.01, 86e9, 690e9, 3, 2, 0.002, 1e-4)
    res, _ = osp.render_spectral(fn_nu(0.0), *args)
    for r in res:
        assert refine.disagreements(r, r["level"])[0] == 0
    nspec = sum(int((r["level"] == refine.SPECTRAL).sum()) for r in res)
    assert nspec > 0
    delta = 1e-6
    pert, _ = osp.render_spectral(fn_nu(delta), *args, forced_levels=[r["level"] for r in res])
    for r, p in zip(res, pert):
        n, worst, rows = refine.disagreements(p, r["level"])
        assert worst <= delta * (1 + 1e-6), rows[:5]


def test_learned_audit_consistent_and_forced_replay():
    params = ocnn.init_params(5)

    def ray3(x, y):
        S = ray_fn_for(6)(x, y)
        return S, np.full(S.shape[0], 5.0, dtype=np.float32), np.zeros(S.shape[0], dtype=np.int32)
    logits = lambda x: ocnn.forward(params, x)[0]
    kw = dict(fov=40.0, nx0=9, ny0=9, levels=3, r_rel=0.02, r_abs=0.01, abs_norm="mean", nstokes=1,
              logits_fn=logits, z_hi=0.2, z_lo=-0.2, fallback=True)
    out = olearned.refine_learned(ray3, **kw)
    assert refine.disagreements(out, out["level"])[0] == 0
    rep = olearned.refine_learned(ray3, forced_level=out["level"], **kw)
    assert refine.disagreements(rep, out["level"])[0] == 0
    assert np.array_equal(rep["img"], out["img"], equal_nan=True)
    assert np.array_equal(rep["level"], out["level"])
