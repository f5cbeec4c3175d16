"""Host logic of the benchmark script (no GPU): the report is strict JSON,
the measured HBM traffic is reported only for the kernel sources and the
headline form it was counted on, the operation count of a render adds up,
and the operating points and timed forms follow the held-out protocol."""
import json
import math

import bench


def test_report_is_strict_json():
    rep = {"a": [1.0, float("inf"), {"b": -float("inf")}], "c": float("nan"), "d": "x", "e": 3}
    line = json.dumps(bench.finite(rep), allow_nan=False)
    back = json.loads(line)
    assert back == {"a": [1.0, "inf", {"b": "-inf"}], "c": "nan", "d": "x", "e": 3}


def test_traffic_only_for_profiled_sources_and_form():
    t = bench.TRAFFIC
    if t is None:
        assert bench.measured_traffic(8, "judge_z2", "mixed") is None
        return
    launches = 8
    got = bench.measured_traffic(launches, t["form"], t["precision"])
    if t["kernel_hash"] == bench.kernel_hash():
        assert got is not None
        assert math.isclose(got["bytes_per_launch"], t["bytes_per_render"] * bench.ROOF_RENDERS / launches)
    else:
        assert got is None
    assert bench.measured_traffic(launches, "some_other_form", t["precision"]) is None
    other = next(p for p in ("mixed", "mixed_geo", "fp64") if p != t["precision"])
    assert bench.measured_traffic(launches, t["form"], other) is None
    assert bench.measured_traffic(0, t["form"], t["precision"]) is None


def test_flop_count_of_a_render():
    cfg = {"model": "thermal", "nstokes": 4}
    st = {"steps": 10, "steps_emit": 4}
    want = 10 * bench.FLOP_GEO_STEP + 4 * (bench.FLOP_PLASMA_THERMAL + bench.FLOP_TRANSFER_IQUV) + \
        6 * bench.FLOP_PLASMA_NOEMIT
    assert bench.flops(st, cfg) == want
    s = bench.FLOP_STRUCTURED
    assert bench.flops(st, cfg, dict(s, noemit=0)) == 10 * s["geo"] + 4 * (s["plasma"] + s["transfer_iquv"])
    assert bench.flops(st, {"model": "toy_disk", "nstokes": 1}) == 10 * bench.FLOP_GEO_STEP + 4 * (
        bench.FLOP_PLASMA_TOY + bench.FLOP_TRANSFER_I)


def test_search_grids():
    assert list(bench.OP_RREL) == sorted(bench.OP_RREL) and bench.OP_RREL[0] == 0.001
    assert all(1 <= d <= 4 for d in bench.IN_FLIGHT_DEPTHS)


def test_operating_points_pick_the_loosest_passing_tolerance():
    forms = [("plain", None), ("lookahead_z4", {"z_propose": 4.0})]
    search = [
        dict(form="plain", r_rel=0.01, rays=100, ok=True),
        dict(form="lookahead_z4", r_rel=0.01, rays=104, ok=True),
        dict(form="plain", r_rel=0.015, rays=95, ok=False),
        dict(form="lookahead_z4", r_rel=0.015, rays=97, ok=True),
        dict(form="lookahead_z4", r_rel=0.02, rays=93, ok=False),
    ]
    op = bench.operating_points(search, forms)
    assert op["plain"]["r_rel"] == 0.01 and op["lookahead_z4"]["r_rel"] == 0.015
    assert op["lookahead_z4"]["options"] == {"z_propose": 4.0}
    # a form that never passes has no operating point
    assert "x" not in bench.operating_points([dict(form="x", r_rel=0.01, rays=1, ok=False)], [("x", None)])


def test_forms_timed_follow_the_held_out_choice():
    grid = (0.001, 0.005, 0.01)
    op_h = {"lookahead_z0": dict(r_rel=0.005, rays=120), "lookahead_z4": dict(r_rel=0.005, rays=100),
            "plain": dict(r_rel=0.001, rays=130)}
    op_t = {"plain": dict(r_rel=0.01, rays=90)}
    got = bench.choose_forms(op_h, op_t, grid)
    assert [(n, f, r) for n, f, r, _ in got] == [("learned_batched", "lookahead_z4", 0.005),
                                                 ("plain_batched", "plain", 0.001),
                                                 ("plain_batched_own_op", "plain", 0.01)]
    # no held-out operating point for plain: its tightest grid tolerance
    got = bench.choose_forms({"lookahead_z4": dict(r_rel=0.005, rays=100)}, {"plain": dict(r_rel=0.001)}, grid)
    assert [(n, r) for n, _, r, _ in got] == [("learned_batched", 0.005), ("plain_batched", 0.001)]
    assert "tightest" in got[1][3]
    # with held-out timings the fastest learned form is taken, not the one with the fewest rays
    op_h["judge_z2"] = dict(r_rel=0.005, rays=110)
    got = bench.choose_forms(op_h, op_t, grid, {"lookahead_z0": 40.0, "lookahead_z4": 38.0, "judge_z2": 36.5})
    assert got[0][:3] == ("learned_batched", "judge_z2", 0.005) and "fastest" in got[0][3]


def test_training_heldout_and_timed_batches_are_disjoint():
    """The network's training images, the held-out batch (operating points)
    and the timed batch share no spin, no inclination and no field phase;
    the training set has the batch's frequencies and both network levels."""
    import art_inputs
    tr = art_inputs.training_workload_batch()
    ho = art_inputs.batch_workload_heldout()
    tb = art_inputs.batch_workload()
    key = lambda cs, f: {c[f] for c in cs}
    for f in ("a", "inc_deg"):
        assert not (key(tr, f) & key(ho, f)) and not (key(tr, f) & key(tb, f)) and not (key(ho, f) & key(tb, f))
    phase = lambda cs: {tuple(c["mp"]) for c in cs}
    assert not (phase(tr) & phase(ho)) and not (phase(tr) & phase(tb)) and not (phase(ho) & phase(tb))
    assert key(tr, "freq_hz") == key(tb, "freq_hz") and {c["levels"] for c in tr} == {4}
    assert all(c["nx0"] == tb[0]["nx0"] for c in tr)


def test_one_gpu_only(monkeypatch, capsys):
    import sys
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_mse_check_reads_whole_planes():
    """A truth given as one 2D plane is Stokes I; a 3D truth is compared plane
    by plane (a 2D truth must not be indexed by row)."""
    import torch

    class FakeArt:
        @staticmethod
        def metrics(t, a):
            t, a = t.double(), a.double()
            return float(abs(t.sum() - a.sum()) / t.sum()), float(((t - a) ** 2).sum() / (t * t).sum())
    truth = torch.ones(4, 3, 5, dtype=torch.float64)
    img = truth.clone()
    img[0, 2, 4] = 1.5                       # one pixel of plane 0, last row
    img[1] *= 2.0
    cfgs = [{"name": "a"}]
    whole = bench.mse_check(FakeArt, cfgs, [img], [truth[0]])
    assert math.isclose(whole["mse_max"], 0.25 / 15)
    per = bench.mse_check(FakeArt, cfgs, [img], [truth], planes=2)
    assert math.isclose(per["mse_max_planes"][0], 0.25 / 15) and math.isclose(per["mse_max_planes"][1], 1.0)
    assert per["mse_ok"] is False and per["n_over_bar"] == 1


def test_parse_launch():
    assert bench.parse_launch("256x256") == dict(trace_blocks=256, trace_threads=256, refill=1, groups=1,
                                                  refine_blocks=0)
    assert bench.parse_launch("256X128:192")["refine_blocks"] == 192
    assert bench.parse_launch("256X128:192")["trace_threads"] == 128


def test_deploy_threshold():
    rows = [dict(z_propose=z, mse=m) for z, m in ((0.0, 6e-5), (2.0, 2e-4), (4.0, 5e-4), (6.0, 1.2e-3))]
    assert bench.deploy_threshold(rows) == 4.0
    assert bench.deploy_threshold([dict(r, mse=2e-3) for r in rows]) == 0.0
    assert bench.deploy_threshold([dict(r, mse=1e-4) for r in rows]) == 6.0
