"""Pins of the oracle's instrumented operation counter and of the benchmark's
algorithmic FLOP figures.

- The counting build computes what the plain build computes: the same step
  counts and bitwise the same Stokes values on every sampled ray.
- The counter counts each arithmetic operation once: a 4x4 matrix product is
  4 x 4 x (4 multiplications + 4 additions) = 128 operations, the horizon
  radius 1 + sqrt(1 - a a) four.
- The benchmark's per-step figures (geodesic step, emitting plasma point,
  non-emitting plasma point, IQUV and I transfer updates, toy-disk plasma
  point) equal the counter's averages over a seeded sample of rays of the
  thermal view and the toy disk within 1 % (they vary a little with the step
  rule's and the series' branches).
"""
import numpy as np
import pytest

import art_inputs
import bench
from oracle import ray as oray


def sample(n=160, seed=3):
    rng = np.random.default_rng(seed)
    return rng.uniform(-18, 18, n), rng.uniform(-18, 18, n)


def test_counting_build_computes_the_same_rays():
    cfg = art_inputs.workload("thermal_1025")
    al, be = sample(40)
    c = oray.count_ops(cfg, al, be)
    S, f = oray.trace(cfg, al, be, nthreads=1)
    assert np.array_equal(c["steps"], f["steps"])
    assert np.array_equal(c["S"], S[:, :4])


def test_counter_counts_each_operation_once():
    assert oray.count_probe(0) == 128
    assert oray.count_probe(1) == 4


@pytest.fixture(scope="module")
def thermal_counts():
    al, be = sample()
    return oray.count_ops(art_inputs.workload("thermal_1025"), al, be)


def close(a, b):
    return abs(a / b - 1.0) < 0.01


def test_geodesic_and_plasma_figures(thermal_counts):
    c = thermal_counts
    emit = c["emit"].sum()
    assert close(c["geo"].sum() / c["steps"].sum(), bench.FLOP_GEO_STEP)
    assert close((c["plasma"] - c["plasma_noemit"]).sum() / emit, bench.FLOP_PLASMA_THERMAL)
    assert close(c["plasma_noemit"].sum() / (c["steps"] - c["emit"]).sum(), bench.FLOP_PLASMA_NOEMIT)


def test_transfer_figures(thermal_counts):
    c = thermal_counts
    assert close(c["transfer"].sum() / c["emit"].sum(), bench.FLOP_TRANSFER_IQUV)
    al, be = sample(60)
    c1 = oray.count_ops(dict(art_inputs.workload("thermal_1025"), nstokes=1), al, be)
    assert close(c1["transfer"].sum() / c1["emit"].sum(), bench.FLOP_TRANSFER_I)


def test_toy_disk_figures():
    al, be = sample(60)
    c = oray.count_ops(art_inputs.workload("toy_disk_64"), al, be)
    assert close((c["plasma"] - c["plasma_noemit"]).sum() / c["emit"].sum(), bench.FLOP_PLASMA_TOY)
    assert close(c["geo"].sum() / c["steps"].sum(), bench.FLOP_GEO_STEP)


def test_structured_forms_do_no_more_than_the_plain_definition(thermal_counts):
    """The tracer's own structured forms need at most the operations the
    plain definition counts (what the roofline's side figure relies on)."""
    s = bench.FLOP_STRUCTURED
    assert s["geo"] <= bench.FLOP_GEO_STEP and s["plasma"] <= bench.FLOP_PLASMA_THERMAL
    assert s["transfer_iquv"] <= bench.FLOP_TRANSFER_IQUV
