"""Selection logic of the in-flight autotuner with a synthetic cost model
(no device: the timer and the device query are replaced)."""
import types

import torch

from paper_2103_07417_amd import autotune


class FakeBatch:
    def __init__(self):
        self.launch = None

    def set_launch(self, blocks, threads, refill, groups, refine_blocks=0, long_steps=0):
        self.launch = dict(trace_blocks=blocks, trace_threads=threads, refill=refill, groups=groups,
                           refine_blocks=refine_blocks, long_steps=long_steps)


def cost(launch, d):
    # fastest at 256 x 256 with 3 in flight, then refill 4, a 224-block refinement grid, threshold 700
    # and a 320-block base grid once the refinement grid is set apart
    rb = launch["refine_blocks"] or launch["trace_blocks"]
    base = launch["trace_blocks"]
    ms = 30.0 + (0 if launch["trace_threads"] == 256 else 1)
    ms += abs(base - 256) / 64 if rb == base else {256: 0.0, 320: -0.2, 384: 0.1, 448: 0.5}.get(base, 3.0)
    ms += {1: 0.0, 2: -0.3, 4: -0.6, 8: -0.2}[launch["refill"]]
    ms += {256: 0.0, 224: -0.4, 192: -0.1}.get(rb, 5.0)
    ms += {0: 0.0, 600: -0.1, 700: -0.3, 900: 0.4}[launch["long_steps"]]
    return ms + (0 if d == 3 else 2)


def test_in_flight_autotuner_picks_the_cheapest_second_stage(monkeypatch):
    monkeypatch.setattr(torch.cuda, "get_device_properties",
                        lambda i: types.SimpleNamespace(multi_processor_count=256))
    monkeypatch.setattr(autotune, "time_in_flight",
                        lambda bs, t, ss, n: cost(bs[0].launch, len(bs)))
    bs = [FakeBatch() for _ in range(3)]
    out = autotune.autotune_in_flight(bs, [None] * 3, depths=(2, 3))
    assert (out["in_flight"], out["trace_blocks"], out["trace_threads"]) == (3, 320, 256)
    assert (out["refill"], out["refine_blocks"], out["long_steps"]) == (4, 224, 700)
    assert out["ms"] == min(r["ms"] for r in out["table"])
    for b in bs:
        assert b.launch == dict(trace_blocks=320, trace_threads=256, refill=4, groups=1, refine_blocks=224,
                                long_steps=700)
    # first stage: 2 depths x 4 grid sizes; second: the best row again + 11 candidates;
    # third: 3 thresholds; fourth: 3 base grids
    assert len(out["table"]) == 8 + 12 + 3 + 3
