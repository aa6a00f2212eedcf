"""FP64 reference of the warm-start network (test infrastructure).

TEST INFRASTRUCTURE: only the test suite may use this module. It shares no code
with the GPU library.

The network maps input planes describing a cavity problem to the steady fields
(u_x, u_y, T) on a fixed grid. It is a four-level encoder-decoder with skip
connections; every convolution is 3x3 with zero padding and a bias:

  level 1 (H x W):     conv cin->w1, ReLU, conv w1->w1, ReLU          -> s1
  level 2 (H/2):       avg-pool 2, conv w1->w2, ReLU, conv w2->w2, ReLU -> s2
  level 3 (H/4):       avg-pool 2, conv w2->w3, ReLU, conv w3->w3, ReLU -> s3
  level 4 (H/8):       avg-pool 2, conv w3->w4, ReLU, conv w4->w4, ReLU
  up to H/4:           nearest upsample 2, concat [., s3], conv (w4+w3)->w3, ReLU,
                       conv w3->w3, ReLU
  up to H/2:           nearest upsample 2, concat [., s2], conv (w3+w2)->w2, ReLU,
                       conv w2->w2, ReLU
  up to H:             nearest upsample 2, concat [., s1], conv (w2+w1)->w1, ReLU,
                       conv w1->w1, ReLU
  output:              conv w1->cout (no activation)

Parameters are a list of (W [cout][cin][3][3], b [cout]) in the order above (15
convolutions). Activations are [C][H][W] per sample. The loss is the mean squared
error over all output elements of the batch.

With quant=True the same network is evaluated with BF16 storage of the operands: the
input planes, the weights, every stored activation (after bias and ReLU, after pooling),
the output gradient, every activation gradient (input gradients of the convolutions, the
upsampling gradient, the ReLU gradient after the skip and pooled gradients are added)
are rounded to the nearest BF16 value (ties to even); the arithmetic between those
points stays FP64 and the network output stays unrounded. A network stored this way in
BF16 and accumulated in a wider type takes the same rounding decisions, so the two agree
element by element up to the accumulation's own rounding.
"""
import numpy as np


def bf16_round(x):
    """Nearest BF16 value (8 significant bits, ties to even) of x, via its FP32 value."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def _q(quant):
    return bf16_round if quant else (lambda a: a)


def layer_shapes(cin, cout, widths):
    w1, w2, w3, w4 = widths
    return [(w1, cin), (w1, w1), (w2, w1), (w2, w2), (w3, w2), (w3, w3), (w4, w3), (w4, w4),
            (w3, w4 + w3), (w3, w3), (w2, w3 + w2), (w2, w2), (w1, w2 + w1), (w1, w1), (cout, w1)]


def init_params(cin, cout, widths, seed):
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for co, ci in layer_shapes(cin, cout, widths):
        lim = np.sqrt(6.0 / (ci * 9))
        out.append((rng.uniform(-lim, lim, (co, ci, 3, 3)), np.zeros(co)))
    return out


# ---------------------------------------------------------------------------
# Primitives (definitions written out with numpy tensordot over the 9 taps)
# ---------------------------------------------------------------------------

def conv3x3(x, w, b):
    C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    y = np.zeros((w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            y += np.tensordot(w[:, :, ky, kx], xp[:, ky:ky + H, kx:kx + W], axes=([1], [0]))
    return y + b[:, None, None]


def conv3x3_backward(x, w, dy):
    C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.tensordot(dy, xp[:, ky:ky + H, kx:kx + W], axes=([1, 2], [1, 2]))
            dxp[:, ky:ky + H, kx:kx + W] += np.tensordot(w[:, :, ky, kx], dy, axes=([0], [0]))
    return dxp[:, 1:H + 1, 1:W + 1], dw, dy.sum(axis=(1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    C, H, W = x.shape
    return x.reshape(C, H // 2, 2, W // 2, 2).mean(axis=(2, 4))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) * 0.25


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(dy):
    C, H, W = dy.shape
    return dy.reshape(C, H // 2, 2, W // 2, 2).sum(axis=(2, 4))


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

def quantized_params(params):
    """Weights rounded to BF16, biases unchanged."""
    return [(bf16_round(w), b) for w, b in params]


def forward(params, x, keep=False, quant=False):
    """x [cin][H][W] -> y [cout][H][W]; with keep=True also the activations backward needs.
    quant: BF16 storage of the operands (see the module docstring)."""
    q = _q(quant)
    if quant:
        params = quantized_params(params)
        x = q(x)
    acts = {}

    def cr(k, inp, act=True):
        z = conv3x3(inp, *params[k])
        acts[k] = (inp, z)
        return q(relu(z)) if act else z

    h = cr(1, cr(0, x));                 s1 = h
    h = cr(3, cr(2, q(avgpool2(s1))));   s2 = h
    h = cr(5, cr(4, q(avgpool2(s2))));   s3 = h
    h = cr(7, cr(6, q(avgpool2(s3))))
    h = cr(9, cr(8, np.concatenate([upsample2(h), s3])))
    h = cr(11, cr(10, np.concatenate([upsample2(h), s2])))
    h = cr(13, cr(12, np.concatenate([upsample2(h), s1])))
    y = cr(14, h, act=False)
    return (y, acts) if keep else y


def backward(params, acts, dy, quant=False):
    """Gradients of the scalar sum(dy * y) with respect to every (W, b).
    quant: BF16 storage of the operands (see the module docstring)."""
    q = _q(quant)
    if quant:
        params = quantized_params(params)
        dy = q(dy)
    grads = [None] * len(params)

    def bcr(k, dout, act=True):
        inp, z = acts[k]
        dz = q(dout * (z > 0)) if act else dout
        dx, dw, db = conv3x3_backward(inp, params[k][0], dz)
        grads[k] = (dw, db)
        return q(dx)

    w1 = params[1][0].shape[0]
    w2 = params[3][0].shape[0]
    w3 = params[5][0].shape[0]
    d = bcr(14, dy, act=False)
    d = bcr(12, bcr(13, d))                           # concat [up(h), s1]
    ds1 = d[d.shape[0] - w1:]
    d = q(upsample2_backward(d[:d.shape[0] - w1]))
    d = bcr(10, bcr(11, d))                           # concat [up(h), s2]
    ds2 = d[d.shape[0] - w2:]
    d = q(upsample2_backward(d[:d.shape[0] - w2]))
    d = bcr(8, bcr(9, d))                             # concat [up(h), s3]
    ds3 = d[d.shape[0] - w3:]
    d = q(upsample2_backward(d[:d.shape[0] - w3]))
    d = bcr(6, bcr(7, d))
    d = bcr(4, bcr(5, avgpool2_backward(d) + ds3))
    d = bcr(2, bcr(3, avgpool2_backward(d) + ds2))
    bcr(0, bcr(1, avgpool2_backward(d) + ds1))
    return grads


def loss_and_grads(params, xs, ts, quant=False):
    """Mean squared error over a batch (xs [B][cin][H][W], ts [B][cout][H][W])."""
    n = ts.size
    loss = 0.0
    total = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    for x, t in zip(xs, ts):
        y, acts = forward(params, x, keep=True, quant=quant)
        r = y - t
        loss += float(np.sum(r * r)) / n
        g = backward(params, acts, 2.0 * r / n, quant=quant)
        total = [(a + dw, c + db) for (a, c), (dw, db) in zip(total, g)]
    return loss, total
