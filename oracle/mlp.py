"""Oracle for the learned troubled-cell / AMR indicator: a 16 -> 64 -> 64 -> 1
ReLU network with BF16 weights, trained with Adam on the mean squared error.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy FP64.

Parameter vector (FP32 master copy, 5313 values):
  W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3[1]
(W[j][k]: output unit j, input k).  The forward pass uses the weights rounded
to BF16 (round to nearest, ties to even, of the FP32 bit pattern); the
gradient is taken at those rounded weights and applied to the FP32 masters.

  h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 . h2 + b3
  loss = (1/B) sum_s (y_s - t_s)^2
Adam (Kingma and Ba 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8:
  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
  w = w - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

The network is not in the paper (the learned indicator is an extension).
Pins: the backward pass against central finite differences, the forward pass
against a hand-set network, the first Adam step against its closed form
(a step of lr sign(g) when |g| >> eps), BF16 rounding against exact cases, the
BF16-operand inference pass against the plain one where every operand is
exactly representable in BF16, and against the rounding it adds elsewhere.
"""
import numpy as np

NIN, NH = 16, 64
SIZES = (("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)),
         ("b3", (1,)))
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def unpack(w):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(w[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def bf16(w):
    """Round FP32 values to BF16 (nearest, ties to even), returned as float64."""
    b = np.asarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)


def init(seed):
    """He-uniform initial weights, zero biases (FP32 values)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES:
        if name.startswith("b"):
            d[name] = np.zeros(shape)
        else:
            fan_in = shape[-1] if len(shape) == 2 else NH
            lim = np.sqrt(6.0 / fan_in)
            d[name] = rng.uniform(-lim, lim, shape)
    return pack(d).astype(np.float32)


def forward(w, x):
    """y[B] and the activations, with BF16-rounded weights, FP64 arithmetic."""
    return forward_params(unpack(bf16(w)), x)


def forward_bf16(w, x):
    """y[B] of the library's inference pass: the operands of both matrix
    products are BF16 (the weights, the inputs and the first hidden layer,
    rounded from its FP32 value), everything else FP64 here (FP32 there)."""
    p = unpack(bf16(w))
    xb = bf16(np.asarray(x, dtype=np.float32))
    z1 = xb @ p["W1"].T + p["b1"]
    h1 = bf16(np.maximum(z1, 0.0).astype(np.float32))
    z2 = h1 @ p["W2"].T + p["b2"]
    return np.maximum(z2, 0.0) @ p["W3"] + p["b3"][0]


def forward_params(p, x):
    """Forward pass with the given (already rounded) FP64 parameters."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2, p)


def loss_and_grad(w, x, t):
    """MSE loss and its gradient with respect to the (rounded) weights."""
    y, (x, z1, h1, z2, h2, p) = forward(w, x)
    B = len(y)
    r = y - np.asarray(t, dtype=np.float64)
    loss = (r * r).sum() / B
    dy = 2.0 * r / B
    g = {"W3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


class Adam:
    def __init__(self, w):
        self.w = np.asarray(w, dtype=np.float32).astype(np.float64)
        self.m = np.zeros_like(self.w)
        self.v = np.zeros_like(self.w)
        self.t = 0

    def step(self, x, target, lr):
        loss, g = loss_and_grad(self.w.astype(np.float32), x, target)
        self.t += 1
        self.m = BETA1 * self.m + (1 - BETA1) * g
        self.v = BETA2 * self.v + (1 - BETA2) * g * g
        mh = self.m / (1 - BETA1 ** self.t)
        vh = self.v / (1 - BETA2 ** self.t)
        # the masters are FP32
        self.w = (self.w - lr * mh / (np.sqrt(vh) + EPS)).astype(np.float32).astype(np.float64)
        return loss
