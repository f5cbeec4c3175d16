"""Plain FP64 numpy reference of the learned refinement proposal network.

Test infrastructure only.  Four 3x3 convolutions with zero padding ("same"
size), ReLU after the first three, channels 3 -> 32 -> 32 -> 32 -> K.  Inputs
are per-vertex features of a level-l grid; the K outputs are logits of
"this point will be ray traced" for the points a vertex owns at the next two
levels.  Loss: positive-weighted binary cross-entropy on logits, averaged over
valid points.  Optimiser: Adam.  Every step is written out with numpy loops
over the 9 kernel taps (no library convolution), so it can be read against
the definitions.

Weight layout: W[l] has shape (C_out, C_in, 3, 3), b[l] has shape (C_out,);
out[co, y, x] = b[co] + sum_{ci, dy, dx} W[co, ci, dy, dx] in[ci, y+dy-1, x+dx-1].

With bf16=True the forward and backward round, like a BF16 network with
FP32 accumulation would, the network input, the weights, the activations
after the ReLU, the loss gradient and the back-propagated activation
gradients to bfloat16 (round to nearest even); sums stay in FP64.
"""
import numpy as np

CHANNELS = (3, 32, 32, 32)
N_OUT = 15          # 3 points at level l+1 and 12 at level l+2 per level-l vertex


def init_params(seed=4, n_out=N_OUT):
    """He-normal weights, zero biases; seeded."""
    rng = np.random.default_rng(seed)
    chans = list(CHANNELS) + [n_out]
    W, b = [], []
    for l in range(4):
        ci, co = chans[l], chans[l + 1]
        W.append(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(co, ci, 3, 3)))
        b.append(np.zeros(co))
    return W, b


def bf16_round(a):
    """Round to the nearest bfloat16 (8 significand bits), ties to even."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, W, b):
    """x (C_in, H, W) -> (C_out, H, W), zero padding."""
    ci, H, Wd = x.shape
    xp = np.zeros((ci, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((W.shape[0], H, Wd)) + b[:, None, None]
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, dy:dy + H, dx:dx + Wd]                 # (C_in, H, W)
            out += np.einsum("oc,chw->ohw", W[:, :, dy, dx], patch)
    return out


def conv3x3_backward(x, W, dout):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    ci, H, Wd = x.shape
    xp = np.zeros((ci, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, dy:dy + H, dx:dx + Wd]
            dW[:, :, dy, dx] = np.einsum("ohw,chw->oc", dout, patch)
            dxp[:, dy:dy + H, dx:dx + Wd] += np.einsum("oc,ohw->chw", W[:, :, dy, dx], dout)
    return dxp[:, 1:-1, 1:-1], dW, dout.sum(axis=(1, 2))


def forward(params, x, bf16=False):
    """Returns logits and the per-layer cache (inputs and pre-activations)."""
    W, b = params
    cache = []
    h = bf16_round(x) if bf16 else x
    for l in range(4):
        Wl = bf16_round(W[l]) if bf16 else W[l]
        z = conv3x3(h, Wl, b[l])
        cache.append((h, z))
        if l < 3:
            h = np.maximum(z, 0.0)
            if bf16:
                h = bf16_round(h)
        else:
            h = z
    return h, cache


def bce_loss(logits, labels, valid, pos_weight, n_valid=None):
    """Sum over valid points of  -[w y log s(z) + (1-y) log(1 - s(z))]
    divided by n_valid (default: the number of valid points, at least 1), and
    its gradient w.r.t. the logits."""
    z = logits
    ls = -np.logaddexp(0.0, -z)           # log sigmoid(z)
    l1s = -np.logaddexp(0.0, z)           # log (1 - sigmoid(z))
    per = -(pos_weight * labels * ls + (1.0 - labels) * l1s)
    n = max(1.0, float(valid.sum())) if n_valid is None else float(n_valid)
    loss = float((per * valid).sum() / n)
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (pos_weight * labels * (sig - 1.0) + (1.0 - labels) * sig) * valid / n
    return loss, dz


def backward(params, cache, dlogits, bf16=False):
    W, b = params
    dW = [None] * 4
    db = [None] * 4
    g = bf16_round(dlogits) if bf16 else dlogits
    for l in range(3, -1, -1):
        h, z = cache[l]
        if l < 3:
            g = g * (z > 0.0)          # through the ReLU of layer l
            if bf16:
                g = bf16_round(g)
        Wl = bf16_round(W[l]) if bf16 else W[l]
        dx, dW[l], db[l] = conv3x3_backward(h, Wl, g)
        g = dx
    return dW, db


def loss_and_grads(params, x, labels, valid, pos_weight, bf16=False):
    logits, cache = forward(params, x, bf16)
    loss, dz = bce_loss(logits, labels, valid, pos_weight)
    dW, db = backward(params, cache, dz, bf16)
    return loss, dW, db


def loss_and_grads_batch(params, xs, labels, valids, pos_weight, bf16=False):
    """Loss and gradients over a batch of images (lists of (C, H, W) arrays);
    the mean runs over the valid points of the whole batch."""
    n = max(1.0, float(sum(float(v.sum()) for v in valids)))
    loss = 0.0
    dW = [np.zeros_like(a) for a in params[0]]
    db = [np.zeros_like(a) for a in params[1]]
    for x, y, v in zip(xs, labels, valids):
        logits, cache = forward(params, x, bf16)
        li, dz = bce_loss(logits, y, v, pos_weight, n_valid=n)
        loss += li
        gW, gb = backward(params, cache, dz, bf16)
        for l in range(4):
            dW[l] += gW[l]
            db[l] += gb[l]
    return loss, dW, db


class Adam:
    """Adam (Kingma & Ba) with bias correction."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps, self.t = lr, b1, b2, eps, 0
        self.m = [np.zeros_like(a) for a in params[0] + params[1]]
        self.v = [np.zeros_like(a) for a in params[0] + params[1]]

    def step(self, params, dW, db):
        self.t += 1
        flat = params[0] + params[1]
        grads = dW + db
        for i, (p, g) in enumerate(zip(flat, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            p -= self.lr * mh / (np.sqrt(vh) + self.eps)


def flatten(params):
    """Single FP32 vector: W0, b0, W1, b1, W2, b2, W3, b3 (C order)."""
    W, b = params
    return np.concatenate([np.concatenate([W[l].ravel(), b[l].ravel()]) for l in range(4)])


def unflatten(vec, n_out=N_OUT):
    chans = list(CHANNELS) + [n_out]
    W, b, k = [], [], 0
    for l in range(4):
        ci, co = chans[l], chans[l + 1]
        n = co * ci * 9
        W.append(np.asarray(vec[k:k + n], dtype=np.float64).reshape(co, ci, 3, 3))
        k += n
        b.append(np.asarray(vec[k:k + co], dtype=np.float64))
        k += co
    return W, b


def n_params(n_out=N_OUT):
    chans = list(CHANNELS) + [n_out]
    return sum(chans[l + 1] * chans[l] * 9 + chans[l + 1] for l in range(4))


# ----------------------------------------------------- features and labels
# The 15 points a level-l vertex (i, j) owns: 3 new points of level l+1 at
# (2i + dx, 2j + dy) and 12 new points of level l+2 at (4i + dx, 4j + dy),
# (dx, dy) running row-major over the 2x2 and 4x4 blocks with both offsets
# even excluded.  Every new point of levels l+1 and l+2 has exactly one owner.
OWNED = [(1, dx, dy) for dy in range(2) for dx in range(2) if (dx % 2) or (dy % 2)] + \
        [(2, dx, dy) for dy in range(4) for dx in range(4) if (dx % 2) or (dy % 2)]


def grid_n(n0, l):
    return (1 << l) * (n0 - 1) + 1


def owned_points(nx0, ny0, levels, l):
    """For each output k: (level, final-grid x, final-grid y, exists) arrays
    of shape (H, W) over the level-l vertices."""
    H, W = grid_n(ny0, l), grid_n(nx0, l)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    out = []
    for up, dx, dy in OWNED:
        lev = l + up
        if lev > levels:
            out.append((lev, np.zeros_like(ii), np.zeros_like(jj), np.zeros(ii.shape, dtype=bool)))
            continue
        p = (ii << up) + dx
        q = (jj << up) + dy
        ok = (p < grid_n(nx0, lev)) & (q < grid_n(ny0, lev))
        s = 1 << (levels - lev)
        out.append((lev, np.where(ok, p * s, 0), np.where(ok, q * s, 0), ok))
    return out


def features(I, rmin, ncross, nx0, ny0, levels, l, n_abs):
    """Network input of level l: (3, H, W) from final-grid arrays of Stokes I,
    minimum radius and equatorial crossings."""
    s = 1 << (levels - l)
    Iv = I[::s, ::s]
    c0 = np.log(np.maximum(Iv, 0.0) / n_abs + 1e-4)
    c1 = np.minimum(rmin[::s, ::s].astype(np.float64), 20.0) / 10.0
    c2 = np.minimum(ncross[::s, ::s], 4).astype(np.float64) / 4.0
    return np.stack([c0, c1, c2])


def labels(level_map, nx0, ny0, levels, l):
    """Targets of level l from a plain render's level map: (15, H, W) labels
    (point traced at its own level) and the valid mask (point exists)."""
    pts = owned_points(nx0, ny0, levels, l)
    lab = np.stack([ok & (level_map[q, p] == lev) for lev, p, q, ok in pts]).astype(np.float64)
    val = np.stack([ok for _, _, _, ok in pts]).astype(np.float64)
    return lab, val
