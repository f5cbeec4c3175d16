"""GPU parity of the learned refinement proposal network (BF16 MFMA forward
and backward through the C ABI) against the numpy oracle (oracle/cnn.py).

Tolerances (BF16 inputs, weights and activations, FP32 accumulation):
- forward logits: relative L2 <= 3e-3 against the oracle that rounds at the
  same places (bf16=True), <= 3e-2 against the plain FP64 oracle;
- gradients: relative L2 per layer <= 2e-2 (bf16 oracle), <= 6e-2 (FP64);
- loss: relative 1e-4 (bf16 oracle);
- Adam: the step equals the oracle's Adam update of the reported gradient
  to FP32 rounding;
- features, labels: labels bit-exact, features to 1e-6.
Shapes span several 32-wide tiles with ragged tails and a batch of images.
"""
import numpy as np
import pytest

import art_inputs
from oracle import cnn as ocnn
from oracle import refine as oref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def case(name, **kw):
    print("CASE", name, kw, flush=True)


def random_params(seed):
    rng = np.random.default_rng(seed)
    W, b = ocnn.init_params(seed=seed)
    b = [rng.normal(0.0, 0.1, size=x.shape) for x in b]
    return W, b


def random_inputs(seed, B, H, W):
    rng = np.random.default_rng(seed)
    x = np.empty((B, 3, H, W))
    x[:, 0] = rng.normal(-3.0, 2.0, size=(B, H, W))
    x[:, 1] = rng.uniform(0.1, 2.0, size=(B, H, W))
    x[:, 2] = rng.integers(0, 5, size=(B, H, W)) / 4.0
    y = (rng.random((B, 15, H, W)) < 0.25).astype(np.uint8)
    v = (rng.random((B, 15, H, W)) < 0.9).astype(np.uint8)
    return x, y, v


def net_with(art, params):
    net = art.Cnn(seed=1)
    assert net.n_params == ocnn.n_params() == 23727
    net.set_params(ocnn.flatten(params).astype(np.float32))
    return net


def f32_params(params):
    """The oracle sees the FP32 values the GPU holds."""
    return ocnn.unflatten(ocnn.flatten(params).astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("B,H,W", [(1, 5, 7), (2, 37, 45), (3, 17, 64), (1, 33, 97)])
def test_forward_parity(art, B, H, W):
    case("cnn forward", B=B, H=H, W=W)
    params = f32_params(random_params(7))
    x, _, _ = random_inputs(3, B, H, W)
    x = x.astype(np.float32).astype(np.float64)
    net = net_with(art, params)
    z = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    for bi in range(B):
        z16, _ = ocnn.forward(params, x[bi], bf16=True)
        z64, _ = ocnn.forward(params, x[bi])
        assert rel(z[bi], z16) <= 3e-3, (bi, rel(z[bi], z16))
        assert rel(z[bi], z64) <= 3e-2, (bi, rel(z[bi], z64))
    net.close()


def test_one_hot_network_shifts_the_input(art):
    """A network whose layers pass one channel through (one-hot kernels)
    reproduces a shifted copy of a non-negative input channel exactly."""
    case("cnn one-hot")
    W, b = ocnn.init_params(seed=1)
    W = [np.zeros_like(a) for a in W]
    b = [np.zeros_like(a) for a in b]
    W[0][0, 1, 0, 1] = 1.0          # channel 1 shifted up by one row
    W[1][0, 0, 1, 1] = 1.0          # identity
    W[2][0, 0, 1, 2] = 1.0          # shifted left by one column
    W[3][4, 0, 1, 1] = 1.0          # into output 4
    H, Wd = 9, 40
    rng = np.random.default_rng(0)
    x = np.zeros((1, 3, H, Wd))
    x[0, 1] = ocnn.bf16_round(rng.uniform(0.0, 2.0, size=(H, Wd)))
    net = net_with(art, (W, b))
    z = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()[0]
    ref = np.zeros((H, Wd))
    ref[1:, :-1] = x[0, 1, :-1, 1:]     # out[y, x] = in[y - 1, x + 1]
    assert np.array_equal(z[4], ref)
    assert np.abs(np.delete(z, 4, axis=0)).max() == 0.0
    net.close()


@pytest.mark.parametrize("B,H,W,pw", [(1, 9, 11, 1.0), (2, 37, 45, 4.0)])
def test_gradient_parity(art, B, H, W, pw):
    case("cnn gradients", B=B, H=H, W=W, pos_weight=pw)
    params = f32_params(random_params(9))
    x, y, v = random_inputs(4, B, H, W)
    x = x.astype(np.float32).astype(np.float64)
    net = net_with(art, params)
    loss, g = net.gradients(torch.tensor(x, dtype=torch.float32, device="cuda"),
                            torch.tensor(y, device="cuda"), torch.tensor(v, device="cuda"), pw)
    l16, dW16, db16 = ocnn.loss_and_grads_batch(params, list(x), list(y.astype(float)),
                                                list(v.astype(float)), pw, bf16=True)
    l64, dW64, db64 = ocnn.loss_and_grads_batch(params, list(x), list(y.astype(float)),
                                                list(v.astype(float)), pw)
    assert abs(loss - l16) <= 1e-4 * abs(l16), (loss, l16)
    gW, gb = ocnn.unflatten(g)
    for l in range(4):
        assert rel(gW[l], dW16[l]) <= 2e-2, (l, rel(gW[l], dW16[l]))
        assert rel(gb[l], db16[l]) <= 2e-2, (l, rel(gb[l], db16[l]))
        assert rel(gW[l], dW64[l]) <= 6e-2, (l, rel(gW[l], dW64[l]))
    net.close()


def test_adam_step_matches_oracle_update(art):
    case("cnn adam")
    params = f32_params(random_params(2))
    x, y, v = random_inputs(8, 2, 21, 35)
    net = net_with(art, params)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    yt, vt = torch.tensor(y, device="cuda"), torch.tensor(v, device="cuda")
    p = ocnn.flatten(params)
    opt_m = np.zeros_like(p)
    opt_v = np.zeros_like(p)
    for t in range(1, 4):
        _, g = net.gradients(xt, yt, vt, 2.0)             # deterministic: same as inside the step
        net.train_step(xt, yt, vt, lr=1e-3, pos_weight=2.0)
        g = g.astype(np.float64)
        opt_m = 0.9 * opt_m + 0.1 * g
        opt_v = 0.999 * opt_v + 0.001 * g * g
        p = p - 1e-3 * (opt_m / (1 - 0.9 ** t)) / (np.sqrt(opt_v / (1 - 0.999 ** t)) + 1e-8)
        got = net.get_params().astype(np.float64)
        assert np.abs(got - p).max() <= 1e-6, (t, np.abs(got - p).max())
        p = got
    net.close()


def test_gradients_are_deterministic(art):
    case("cnn determinism")
    params = f32_params(random_params(5))
    x, y, v = random_inputs(6, 2, 29, 70)
    net = net_with(art, params)
    args = (torch.tensor(x, dtype=torch.float32, device="cuda"), torch.tensor(y, device="cuda"),
            torch.tensor(v, device="cuda"), 3.0)
    l1, g1 = net.gradients(*args)
    l2, g2 = net.gradients(*args)
    assert l1 == l2 and np.array_equal(g1, g2)
    net.close()


def test_features_and_labels_match_oracle(art):
    cfg = art_inputs.reduced(art_inputs.workload("thermal_1025"), 9, 3)
    cfg["nstokes"] = 1
    case("cnn features/labels", nx0=9, levels=3)
    img, lev, ft, st = art.render(cfg, feat=True)
    I = img.cpu().numpy()[0]
    L = lev.cpu().numpy()
    f = art.feat_numpy(ft)
    for l in range(3):
        x = art.cnn_features(cfg, img, ft, l, st["n_abs"]).cpu().numpy()[0]
        xo = ocnn.features(I, f["rmin"], f["ncross"], 9, 9, 3, l, st["n_abs"])
        assert np.abs(x - xo).max() <= 1e-5
        lab, val = art.cnn_labels(cfg, lev, l)
        lo, vo = ocnn.labels(L, 9, 9, 3, l)
        assert np.array_equal(lab.cpu().numpy()[0], lo.astype(np.uint8))
        assert np.array_equal(val.cpu().numpy()[0], vo.astype(np.uint8))
    # every interpolated point carries the features of its neighbours
    assert (f["rmin"][L < 0] > 0).all()
