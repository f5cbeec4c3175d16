"""Pins of the network oracle (oracle/cnn.py) against what the definitions fix:
central finite differences of the loss, a one-hot kernel that shifts its
input, the bfloat16 rounding rule, and the ownership of new points."""
import numpy as np
import pytest

from oracle import cnn


def _loss(params, xs, ys, vs, w):
    return cnn.loss_and_grads_batch(params, xs, ys, vs, w)[0]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(11)
    W, b = cnn.init_params(seed=3)
    b = [rng.normal(0.0, 0.1, size=a.shape) for a in b]      # nonzero biases exercise db
    params = (W, b)
    xs = [rng.normal(size=(3, 5, 7)), rng.normal(size=(3, 5, 7))]
    ys = [(rng.random((15, 5, 7)) < 0.3).astype(float) for _ in xs]
    vs = [(rng.random((15, 5, 7)) < 0.8).astype(float) for _ in xs]
    loss, dW, db = cnn.loss_and_grads_batch(params, xs, ys, vs, 3.0)
    h = 1e-6
    picks = []
    for l in range(4):
        for _ in range(6):
            picks.append(("W", l, tuple(rng.integers(0, s) for s in W[l].shape)))
        picks.append(("b", l, (int(rng.integers(0, b[l].shape[0])),)))
    worst = 0.0
    for kind, l, idx in picks:
        arr = W[l] if kind == "W" else b[l]
        g = (dW if kind == "W" else db)[l][idx]
        old = arr[idx]
        arr[idx] = old + h
        lp = _loss(params, xs, ys, vs, 3.0)
        arr[idx] = old - h
        lm = _loss(params, xs, ys, vs, 3.0)
        arr[idx] = old
        fd = (lp - lm) / (2 * h)
        err = abs(fd - g) / max(1e-6, abs(fd) + abs(g))
        worst = max(worst, err)
    assert worst < 1e-5, worst


def test_one_hot_kernel_shifts_the_input():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 6, 8))
    for c, dy, dx in ((0, 0, 0), (1, 1, 1), (2, 2, 0), (0, 0, 2)):
        Wk = np.zeros((1, 3, 3, 3))
        Wk[0, c, dy, dx] = 1.0
        out = cnn.conv3x3(x, Wk, np.zeros(1))[0]
        ref = np.zeros((6, 8))
        sy, sx = dy - 1, dx - 1          # out[y, x] = in[y + sy, x + sx], zero outside
        for y in range(6):
            for xx in range(8):
                yy, xs = y + sy, xx + sx
                if 0 <= yy < 6 and 0 <= xs < 8:
                    ref[y, xx] = x[c, yy, xs]
        assert np.array_equal(out, ref)


def test_bf16_rounding_rule():
    ulp = 2.0 ** -7                       # bfloat16 spacing in [1, 2)
    vals = np.array([1.0, 1.0 + ulp / 2, 1.0 + 1.5 * ulp, 1.0 + 0.75 * ulp, -3.0 - ulp / 4,
                     0.0, 65504.0])
    want = np.array([1.0, 1.0, 1.0 + 2 * ulp, 1.0 + ulp, -3.0, 0.0, 65536.0])
    assert np.array_equal(cnn.bf16_round(vals), want)
    r = np.random.default_rng(0).normal(size=10000) * 100
    q = cnn.bf16_round(r)
    # relative error at most half a bfloat16 ulp (2^-8), and idempotent
    assert np.all(np.abs(q - r) <= np.abs(r) * 2.0 ** -8 + 1e-300)
    assert np.array_equal(cnn.bf16_round(q), q)


def test_bf16_forward_stays_close_to_fp64():
    rng = np.random.default_rng(5)
    params = cnn.init_params(seed=4)
    x = rng.normal(size=(3, 9, 11))
    z64, _ = cnn.forward(params, x)
    z16, _ = cnn.forward(params, x, bf16=True)
    rel = np.linalg.norm(z16 - z64) / np.linalg.norm(z64)
    assert 0.0 < rel < 2e-2, rel


@pytest.mark.parametrize("nx0,ny0,levels,l", [(3, 3, 2, 0), (4, 3, 3, 1), (5, 4, 3, 2), (3, 5, 4, 0)])
def test_every_new_point_has_one_owner(nx0, ny0, levels, l):
    nx, ny = cnn.grid_n(nx0, levels), cnn.grid_n(ny0, levels)
    count = np.zeros((ny, nx), dtype=int)
    for lev, p, q, ok in cnn.owned_points(nx0, ny0, levels, l):
        np.add.at(count, (q[ok], p[ok]), 1)
    # new points of level l+1 and (if it exists) l+2, in final-grid units
    expect = np.zeros((ny, nx), dtype=int)
    for lv in (l + 1, l + 2):
        if lv > levels:
            continue
        s = 1 << (levels - lv)
        for q in range(cnn.grid_n(ny0, lv)):
            for p in range(cnn.grid_n(nx0, lv)):
                if p % 2 or q % 2:
                    expect[q * s, p * s] = 1
    assert np.array_equal(count, expect)


def test_labels_read_the_level_map():
    nx0, ny0, levels, l = 3, 3, 3, 1
    nx = cnn.grid_n(nx0, levels)
    rng = np.random.default_rng(1)
    lm = rng.integers(-1, 4, size=(nx, nx)).astype(np.int8)
    lab, val = cnn.labels(lm, nx0, ny0, levels, l)
    for k, (lev, p, q, ok) in enumerate(cnn.owned_points(nx0, ny0, levels, l)):
        assert np.array_equal(val[k] > 0, ok)
        assert np.array_equal(lab[k] > 0, ok & (lm[q, p] == lev))
