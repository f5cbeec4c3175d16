"""Host logic of the benchmark script (no GPU): the report is strict JSON,
the measured HBM traffic is reported only for the kernel sources and the
headline form it was counted on, and the FLOP count of one step adds up."""
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
    launches = 8
    got = bench.measured_traffic(launches, t["form"])
    if t["kernel_hash"] == bench.kernel_hash():
        assert got is not None
        assert math.isclose(got["bytes_per_launch"], t["bytes_per_render"] * bench.ROOF_RENDERS / launches)
    else:
        assert got is None
    assert bench.measured_traffic(launches, "some_other_form") is None
    assert bench.measured_traffic(0, t["form"]) is None


def test_flop_count_of_a_step():
    cfg = {"model": "thermal", "nstokes": 4}
    st = {"steps": 10, "steps_emit": 4}
    want = 10 * bench.FLOP_GEO_STEP + 4 * (bench.FLOP_PLASMA_THERMAL + bench.FLOP_TRANSFER_IQUV)
    assert bench.flops(st, cfg) == want
    assert bench.flops(st, {"model": "toy_disk", "nstokes": 1}) == 10 * bench.FLOP_GEO_STEP + 4 * (
        bench.FLOP_PLASMA_TOY + bench.FLOP_TRANSFER_I)


def test_search_grids():
    assert list(bench.OP_RREL) == sorted(bench.OP_RREL) and bench.OP_RREL[0] == 0.01
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
    extra = bench.forms_to_time(op, 0.01)
    assert [n for n, _ in extra] == ["learned_batched_op"] and extra[0][1]["rays"] == 97
    # a plain operating point looser than the workload's tolerance is timed too
    op2 = bench.operating_points(search + [dict(form="plain", r_rel=0.0125, rays=98, ok=True)], forms)
    assert [n for n, _ in bench.forms_to_time(op2, 0.01)] == ["plain_batched_op", "learned_batched_op"]
    # a form that never passes has no operating point
    assert "x" not in bench.operating_points([dict(form="x", r_rel=0.01, rays=1, ok=False)], [("x", None)])
