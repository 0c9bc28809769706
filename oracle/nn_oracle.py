"""FP64 CPU oracle for the learned surrogate of the spectral TV decomposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` (and nothing in the product path)
may import this module.  It shares no code with the HIP library.

The paper replaces the model-driven decomposition by a convolutional network
trained on its output (Sec. 3): 3x3 convolutions with ReLU activations,
biases, and the normalised mean squared error loss of Sec. 3 (the squared
error of each band divided by the band's squared norm, averaged over the
bands), minimised with Adam (Sec. 4.1; Kingma and Ba 2015).  The network
here is the 4-level encoder-decoder variant the paper also evaluates (the
U-Net-type architecture of Sec. 4.5: max-pooling down, upsampling and skip
connections up).  Everything below is written from those definitions:

  conv3x3         y[b,i,j,o] = bias[o] + sum_{dy,dx,c} x[b,i+dy-1,j+dx-1,c] w[o,dy,dx,c],
                  zero outside the image (channels last, "same" padding)
  conv3x3_dgrad   the adjoint of conv3x3 in x (no bias)
  conv3x3_wgrad   the gradient of <dy, conv3x3(x, w)> in w
  maxpool2 / upsample2 (nearest) and their gradients
  nmse_loss       (1/(B J)) sum_b sum_j ||o_bj - t_bj||^2 / ||t_bj||^2, with
                  its gradient in o
  adam_step       Kingma and Ba's update with bias correction
  UNetOracle      the encoder-decoder's forward and backward passes
  surrogate_input / surrogate_output / surrogate_target
                  the surrogate's maps around the encoder-decoder: the image
                  enters as 2 f - 1; output channel c is scale[c] times the
                  last layer's channel, and the residual channels add f (a
                  skip from the input, the residual learning of DnCNN, which
                  the paper's network is based on); the last layer is trained
                  towards the bands and r - f

Each tensor is a numpy array in float64, images channels-last [B, H, W, C].
"""
import numpy as np


def conv3x3(x, w, bias=None):
    """x [B,H,W,C], w [O,3,3,C] -> [B,H,W,O], zero padding."""
    B, H, W, C = x.shape
    O = w.shape[0]
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    y = np.zeros((B, H, W, O))
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, dy, dx, :].T
    if bias is not None:
        y += bias
    return y


def conv3x3_dgrad(dy, w):
    """Adjoint of conv3x3 in x: dy [B,H,W,O], w [O,3,3,C] -> dx [B,H,W,C]."""
    B, H, W, O = dy.shape
    C = w.shape[3]
    dxp = np.zeros((B, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + H, kx:kx + W, :] += dy @ w[:, ky, kx, :]
    return dxp[:, 1:H + 1, 1:W + 1, :]


def conv3x3_wgrad(x, dy):
    """Gradient in w of <dy, conv3x3(x, w)>: x [B,H,W,C], dy [B,H,W,O] -> [O,3,3,C]."""
    B, H, W, C = x.shape
    O = dy.shape[3]
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    dw = np.zeros((O, 3, 3, C))
    d2 = dy.reshape(-1, O)
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = d2.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, C)
    return dw


def bias_grad(dy):
    return dy.reshape(-1, dy.shape[-1]).sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def maxpool2(x):
    """2x2 max pooling, stride 2 (H, W even)."""
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).max(axis=(2, 4))


def maxpool2_grad(x, dy):
    """Gradient of maxpool2: each window's gradient goes to its maximum (the
    first one in row-major window order when several are equal)."""
    B, H, W, C = x.shape
    win = x.reshape(B, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 5, 2, 4).reshape(B, H // 2, W // 2, C, 4)
    arg = win.argmax(axis=-1)
    dx = np.zeros((B, H // 2, W // 2, C, 4))
    np.put_along_axis(dx, arg[..., None], dy[..., None], axis=-1)
    return dx.reshape(B, H // 2, W // 2, C, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(B, H, W, C)


def upsample2(x):
    """Nearest-neighbour upsampling by 2."""
    return x.repeat(2, axis=1).repeat(2, axis=2)


def upsample2_grad(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def nmse_loss(o, t, groups, floor=None):
    """Normalised MSE (Sec. 3): o, t [B,H,W,G*g]; the output channels form
    `groups` bands of equal width.  Returns (loss, d loss / d o).

    floor (optional, [groups]) is added to each band's squared norm in the
    denominator (0 gives the paper's loss)."""
    B = o.shape[0]
    g = o.shape[3] // groups
    loss = 0.0
    grad = np.zeros_like(o)
    for b in range(B):
        for j in range(groups):
            sl = (b, slice(None), slice(None), slice(j * g, (j + 1) * g))
            num = np.sum((o[sl] - t[sl]) ** 2)
            den = np.sum(t[sl] ** 2) + (0.0 if floor is None else floor[j])
            loss += num / den
            grad[sl] = 2.0 * (o[sl] - t[sl]) / den
    return loss / (B * groups), grad / (B * groups)


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015, Algorithm 1) at step t >= 1;
    returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def _same(x):
    return x


class UNetOracle:
    """The encoder-decoder: widths w0..w3 at 1, 1/2, 1/4, 1/8 resolution,
    two 3x3 conv + ReLU per level, 2x2 max-pooling down, nearest upsampling,
    skip connections by channel concatenation (upsampled first), and a final
    3x3 conv to the output channels without activation.

    params: dict name -> (w [O,3,3,C], b [O]) with the layer names below.

    Optional storage hooks (default: none, pure float64) apply a rounding at
    the points where an implementation stores tensors in a narrower type:
    act_store on every ReLU layer output, out_store on the network output,
    grad_store on every stored activation gradient (each layer's input
    gradient, the upsampling gradient, the pooled-plus-skip gradient).
    Pooling, upsampling and concatenation move stored values and round
    nothing."""

    def __init__(self, cin, cout, widths, act_store=None, out_store=None, grad_store=None):
        self.cin, self.cout, self.widths = cin, cout, list(widths)
        self.act_store = act_store or _same
        self.out_store = out_store or _same
        self.grad_store = grad_store or _same
        w0, w1, w2, w3 = self.widths
        self.layers = [("e1a", cin, w0), ("e1b", w0, w0), ("e2a", w0, w1), ("e2b", w1, w1),
                       ("e3a", w1, w2), ("e3b", w2, w2), ("e4a", w2, w3), ("e4b", w3, w3),
                       ("d3a", w3 + w2, w2), ("d3b", w2, w2), ("d2a", w2 + w1, w1), ("d2b", w1, w1),
                       ("d1a", w1 + w0, w0), ("d1b", w0, w0), ("out", w0, cout)]

    def forward(self, p, x):
        c = {}
        a = x
        skips = []
        for lvl, (la, lb) in enumerate((("e1a", "e1b"), ("e2a", "e2b"), ("e3a", "e3b"), ("e4a", "e4b"))):
            c[la + "_in"] = a
            a = self.act_store(relu(conv3x3(a, *p[la])))
            c[la] = a
            c[lb + "_in"] = a
            a = self.act_store(relu(conv3x3(a, *p[lb])))
            c[lb] = a
            if lvl < 3:
                skips.append(a)
                c["pool%d_in" % lvl] = a
                a = maxpool2(a)
        for (la, lb), s in zip((("d3a", "d3b"), ("d2a", "d2b"), ("d1a", "d1b")), reversed(skips)):
            a = np.concatenate([upsample2(a), s], axis=3)
            c[la + "_in"] = a
            a = self.act_store(relu(conv3x3(a, *p[la])))
            c[la] = a
            c[lb + "_in"] = a
            a = self.act_store(relu(conv3x3(a, *p[lb])))
            c[lb] = a
        c["out_in"] = a
        y = self.out_store(conv3x3(a, *p["out"]))
        return y, c

    def backward(self, p, c, dy, scales=None):
        """Gradients of <dy, forward(p, x)> in every parameter.  If `scales`
        is a dict it receives, per layer, the same sums taken over absolute
        values, (wgrad(|x|, |da|), sum |da|): the size of the terms each
        gradient entry adds up, against which its rounding error is judged
        (the sums cancel, so their own size is no scale)."""
        g = {}

        def layer(name, da, act=True):
            if act:
                da = da * (c[name] > 0)
            g[name] = (conv3x3_wgrad(c[name + "_in"], da), bias_grad(da))
            if scales is not None:
                scales[name] = (conv3x3_wgrad(np.abs(c[name + "_in"]), np.abs(da)), bias_grad(np.abs(da)))
            return self.grad_store(conv3x3_dgrad(da, p[name][0]))

        d = layer("out", dy, act=False)
        widths = self.widths
        skip_grads = []
        for (la, lb), wskip in zip((("d1a", "d1b"), ("d2a", "d2b"), ("d3a", "d3b")), (widths[0], widths[1], widths[2])):
            d = layer(lb, d)
            d = layer(la, d)
            nup = d.shape[3] - wskip
            skip_grads.append(d[..., nup:])
            d = self.grad_store(upsample2_grad(d[..., :nup]))
        for lvl, (la, lb) in reversed(list(enumerate((("e1a", "e1b"), ("e2a", "e2b"), ("e3a", "e3b"), ("e4a", "e4b"))))):
            if lvl < 3:
                d = self.grad_store(maxpool2_grad(c["pool%d_in" % lvl], d) + skip_grads[lvl])
            d = layer(lb, d)
            d = layer(la, d)
        return g


def surrogate_input(f):
    """Images f [B, 3, H, W] in [0, 1] -> the network's input 2 f - 1,
    channels last [B, H, W, 3]."""
    return np.transpose(2.0 * np.asarray(f, dtype=np.float64) - 1.0, (0, 2, 3, 1))


def surrogate_output(y, f, scale):
    """Last layer's output y [B, H, W, 15] -> decomposition [B, 15, H, W]:
    channel c is scale[c] y_c; channels 3j + c (j < 4) are band j of colour c,
    and 12 + c is the residual of colour c, f_c + scale y."""
    out = np.transpose(np.asarray(y, dtype=np.float64) * np.asarray(scale, dtype=np.float64), (0, 3, 1, 2)).copy()
    out[:, 12:] += np.asarray(f, dtype=np.float64)
    return out


def surrogate_target(f, bands, res):
    """What the last layer (before the output scale) is trained towards,
    [B, H, W, 15]: the bands [B, 4, 3, H, W] and r - f for the residual."""
    B, nb, C, H, W = bands.shape
    t = np.concatenate([np.asarray(bands, dtype=np.float64).reshape(B, nb * C, H, W),
                        np.asarray(res, dtype=np.float64) - np.asarray(f, dtype=np.float64)], axis=1)
    return np.transpose(t, (0, 2, 3, 1))


def identity_error(f, out):
    """Reconstruction-identity error of decompositions out [B, 15, H, W]
    (Eq. (7): f = sum of bands + residual): per image, the mean over
    channels and pixels of |f - sum_j band_j - residual|."""
    f = np.asarray(f, dtype=np.float64)
    out = np.asarray(out, dtype=np.float64)
    B, C, H, W = f.shape
    d = f - out[:, :12].reshape(B, 4, C, H, W).sum(axis=1) - out[:, 12:]
    return np.abs(d).mean(axis=(1, 2, 3))
