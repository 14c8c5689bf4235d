"""Pins of the float64 MLP reference: central finite differences, networks with a
closed-form output, Adam's first step, and bfloat16 rounding of hand-picked values."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_hand_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7,
                  -2.5, 3.0e38, 1.0 + 2.0 ** -8 + 2.0 ** -20], np.float32)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0);
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even gives 1 + 2^-6
    # 3e38 = 1.7632 * 2^127; 7 mantissa bits: 1.7632 * 128 = 225.7 -> 226, i.e. 226 * 2^120
    want = [1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -2.5, 226.0 * 2.0 ** 120, 1.0 + 2.0 ** -7]
    got = mlp.bf16_round(x)
    assert np.allclose(got[:5], want[:5], rtol=0, atol=0)
    assert float(got[5]) == want[5]
    assert got[6] == want[6]
    assert np.array_equal(mlp.from_bf16_bits(mlp.bf16_bits(x)), got)


def test_param_count():
    assert mlp.NPARAM == 8641


def test_identity_network_closed_form():
    # h1 = (relu(x0), relu(-x0), 0..), passed through identities, y = h[0] - h[1] = x0
    d = {name: np.zeros(s) for name, s in mlp.SHAPES}
    d["W1"][0, 0] = 1.0
    d["W1"][1, 0] = -1.0
    d["W2"] = np.eye(64)
    d["W3"] = np.eye(64)
    d["W4"][0, 0] = 1.0
    d["W4"][0, 1] = -1.0
    d["b4"][0] = 0.25
    p = mlp.pack(d)
    X = np.random.default_rng(0).normal(size=(50, 3))
    y, cache = mlp.forward(p, X)
    assert np.allclose(y, X[:, 0] + 0.25, atol=1e-14)
    dy = np.random.default_rng(1).normal(size=50)
    g = mlp.unpack(mlp.backward(p, cache, dy))
    assert np.isclose(g["b4"][0], dy.sum())
    assert np.isclose(g["W4"][0, 0], (dy * np.maximum(X[:, 0], 0)).sum())
    assert np.isclose(g["W4"][0, 1], (dy * np.maximum(-X[:, 0], 0)).sum())
    # y = relu(W1[0,0] x0) - relu(W1[1,0] x0): d/dW1[0,0] = x0 [x0 > 0], d/dW1[1,0] = -x0 [x0 < 0]
    assert np.isclose(g["W1"][0, 0], (dy * X[:, 0] * (X[:, 0] > 0)).sum())
    assert np.isclose(g["W1"][1, 0], (dy * -X[:, 0] * (X[:, 0] < 0)).sum())


def test_finite_differences():
    rng = np.random.default_rng(3)
    p = mlp.init_params(5) + rng.normal(0, 0.05, mlp.NPARAM)
    X = rng.normal(size=(16, 3)) * 2
    t = rng.normal(size=16)
    y, cache = mlp.forward(p, X)
    _, dy = mlp.loss_and_dy(y, t)
    g = mlp.backward(p, cache, dy)
    idx = rng.choice(mlp.NPARAM, 200, replace=False)
    idx = np.concatenate([idx, [0, 191, 192, 8639, 8640]])
    h = 1e-6
    worst = 0.0
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        lp, _ = mlp.loss_and_dy(mlp.forward(p + e, X)[0], t)
        lm, _ = mlp.loss_and_dy(mlp.forward(p - e, X)[0], t)
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(1e-8, abs(g).max()))
    assert worst < 1e-6


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    w0 = np.ones(4)
    w, m, v = mlp.adam_step(w0, g, np.zeros(4), np.zeros(4), lr=0.01, step=1)
    assert np.allclose(w[:3], w0[:3] - 0.01 * np.sign(g[:3]), atol=1e-7)
    assert w[3] == 1.0
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
