"""Pins of the learned-indicator network oracle (oracle/mlp.py): BF16
rounding on exact cases, the backward pass against central finite
differences, a hand-set forward pass, and Adam's first step."""
import numpy as np

from oracle import mlp as MLP


def test_bf16_rounding_exact_cases():
    one = 1.0
    cases = {one: one, one + 2 ** -7: one + 2 ** -7,
             one + 2 ** -8: one,                    # tie, to even (mantissa ...0)
             one + 3 * 2 ** -8: one + 2 ** -6,      # tie, to even (mantissa ...10)
             one + 2 ** -8 + 2 ** -12: one + 2 ** -7,
             -(one + 2 ** -8 + 2 ** -12): -(one + 2 ** -7), 0.0: 0.0}
    for x, r in cases.items():
        assert MLP.bf16(np.array([x]))[0] == r, (x, r)


def test_param_count():
    assert MLP.NPARAM == 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1 == 5313


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    w = MLP.init(3)
    x = rng.uniform(0, 1, (7, 16))
    t = rng.uniform(0, 0.5, 7)
    y, (_, z1, _, z2, _, p) = MLP.forward(w, x)
    assert min(np.abs(z1).min(), np.abs(z2).min()) > 1e-4  # no ReLU kink within reach
    loss, g = MLP.loss_and_grad(w, x, t)
    flat = MLP.pack(p)
    h = 1e-7
    idx = np.concatenate([rng.choice(np.arange(o, o + k), min(k, 12), replace=False)
                          for o, k in zip(np.cumsum([0] + [int(np.prod(s)) for _, s in MLP.SIZES])[:-1],
                                          [int(np.prod(s)) for _, s in MLP.SIZES])])
    for i in idx:
        wp, wm = flat.copy(), flat.copy()
        wp[i] += h
        wm[i] -= h
        lp = ((MLP.forward_params(MLP.unpack(wp), x)[0] - t) ** 2).mean()
        lm = ((MLP.forward_params(MLP.unpack(wm), x)[0] - t) ** 2).mean()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(g[i])), (i, fd, g[i])


def test_forward_hand_set():
    d = {"W1": np.vstack([np.eye(16), np.zeros((48, 16))]), "b1": np.zeros(64),
         "W2": np.eye(64), "b2": np.zeros(64), "W3": np.r_[np.ones(16), np.zeros(48)],
         "b3": np.array([0.5])}
    w = MLP.pack(d).astype(np.float32)
    x = np.random.default_rng(1).uniform(-1, 1, (5, 16))
    y = MLP.forward(w, x)[0]
    assert np.abs(y - (np.maximum(x, 0).sum(axis=1) + 0.5)).max() < 1e-14


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(2)
    w0 = MLP.init(5)
    x = rng.uniform(0, 1, (32, 16))
    t = rng.uniform(0, 0.5, 32)
    _, g = MLP.loss_and_grad(w0, x, t)
    opt = MLP.Adam(w0)
    lr = 1e-3
    opt.step(x, t, lr)
    dw = opt.w - w0.astype(np.float64)
    big = np.abs(g) > 1e-3
    # |g| >> eps: the first step is lr sign(g) up to eps/|g| and FP32 rounding of w
    err = np.abs(dw[big] + lr * np.sign(g[big]))
    assert (err <= lr * 1e-5 + 2.0 ** -23 * np.abs(w0[big]) + 1e-12).all()


def test_bf16_inference_equals_plain_forward_on_bf16_exact_operands():
    """Weights, inputs and first-layer activations that are exactly BF16
    (small dyadic values): the BF16-operand pass adds no rounding and equals the
    plain forward pass."""
    rng = np.random.default_rng(4)
    d = {"W1": rng.integers(-4, 5, (64, 16)) / 8.0, "b1": rng.integers(-4, 5, 64) / 8.0,
         "W2": rng.integers(-4, 5, (64, 64)) / 64.0, "b2": rng.integers(-4, 5, 64) / 8.0,
         "W3": rng.integers(-4, 5, 64) / 8.0, "b3": np.array([0.25])}
    w = MLP.pack(d).astype(np.float32)
    x = (rng.integers(0, 8, (50, 16)) / 8.0).astype(np.float32)
    # first-layer values: sums of 16 products of (k/8)(m/8) plus b1, multiples
    # of 1/64 below 2^4 in magnitude: exact in BF16 (8 significant bits) only
    # when small; keep the rows whose activations are exact
    z1 = x.astype(np.float64) @ d["W1"].T + d["b1"]
    h1 = np.maximum(z1, 0.0)
    exact = np.all(MLP.bf16(h1) == h1, axis=1)
    assert exact.sum() >= 10
    y0 = MLP.forward(w, x[exact])[0]
    y1 = MLP.forward_bf16(w, x[exact])
    assert np.array_equal(y0, y1)


def test_bf16_inference_rounds_the_inputs_and_the_first_layer():
    """Generic inputs: the BF16 pass equals the plain pass applied to the
    BF16-rounded inputs with the first layer rounded to BF16, and differs from
    the plain pass by the size of that rounding (relative 2^-9 per operand)."""
    w = MLP.init(3)
    x = np.random.default_rng(5).uniform(0, 1, (200, 16)).astype(np.float32)
    p = MLP.unpack(MLP.bf16(w))
    xb = MLP.bf16(x)
    assert np.all(np.abs(xb - x) <= 2.0 ** -8 * np.abs(x))
    h1 = MLP.bf16(np.maximum(xb @ p["W1"].T + p["b1"], 0.0).astype(np.float32))
    ref = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0) @ p["W3"] + p["b3"][0]
    assert np.allclose(MLP.forward_bf16(w, x), ref, rtol=0, atol=0)
    y = MLP.forward(w, x)[0]
    assert 0 < np.abs(MLP.forward_bf16(w, x) - y).max() < 0.05 * np.abs(y).max()
