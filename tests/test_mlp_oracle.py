"""Pins of the surrogate's float64 reference (oracle/mlp.py)."""

import numpy as np
import pytest

from oracle import mlp


def random_params(rng, scale=0.08):
    p = {}
    for name, shape in mlp.SHAPES:
        p[name] = rng.normal(0.0, scale, size=shape)
    return p


def random_tokens(rng, B, n):
    X = np.zeros((B, n, mlp.D_IN))
    X[:, :, :mlp.N_FEAT] = rng.normal(0.0, 1.0, size=(B, n, mlp.N_FEAT))
    for b in range(B):
        pos = rng.permutation(n)
        X[b, np.arange(n), mlp.N_FEAT + pos] = 1.0
    return X


def test_bf16_rounding_known_values():
    # pi in float32 is 0x40490FDB; the kept half 0x4049 rounds down -> 3.140625
    assert mlp.bf16(np.pi) == 3.140625
    assert mlp.bf16(1.0) == 1.0
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(-2.5) == -2.5
    assert mlp.bf16(0.0) == 0.0
    # every bf16 value is a fixed point
    x = mlp.bf16(np.random.default_rng(0).normal(size=1000))
    assert np.array_equal(mlp.bf16(x), x)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_finite_differences(seed):
    """Central differences of the float64 model pin every backward formula."""
    rng = np.random.default_rng(seed)
    params = random_params(rng)
    X = random_tokens(rng, B=5, n=4)
    t = rng.normal(1.0, 0.3, size=5)
    _, _, grads = mlp.loss_and_grads(params, X, t, bf16_points=False)
    eps = 1e-6
    for name, shape in mlp.SHAPES:
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in shape)
            plus = {k: v.copy() for k, v in params.items()}
            minus = {k: v.copy() for k, v in params.items()}
            plus[name][idx] += eps
            minus[name][idx] -= eps
            lp, _, _ = mlp.loss_and_grads(plus, X, t, bf16_points=False)
            lm, _, _ = mlp.loss_and_grads(minus, X, t, bf16_points=False)
            fd = (lp - lm) / (2 * eps)
            assert grads[name][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, idx)


def test_pooling_is_order_invariant_over_tokens():
    """Sum pooling: permuting the token rows of a sample leaves y unchanged."""
    rng = np.random.default_rng(3)
    params = random_params(rng)
    X = random_tokens(rng, B=3, n=6)
    y, _ = mlp.forward(params, X, bf16_points=False)
    Xp = X[:, rng.permutation(6), :]
    yp, _ = mlp.forward(params, Xp, bf16_points=False)
    assert np.allclose(y, yp, rtol=0, atol=1e-12)


def test_adam_first_step_closed_form():
    """After one step from zero moments the bias-corrected update is
    lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    theta, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), step=1, lr=0.01)
    assert np.allclose(theta, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_flatten_roundtrip():
    rng = np.random.default_rng(4)
    p = random_params(rng)
    v = mlp.flatten(p)
    assert v.size == mlp.n_params()
    q = mlp.unflatten(v)
    assert all(np.array_equal(p[k], q[k]) for k in p)


def _hand_params(spec):
    p = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    for name, entries in spec.items():
        for e in entries:
            p[name][tuple(int(i) for i in e[:-1])] = e[-1]
    return p


def _hand_tokens(positions):
    X = np.zeros((1, 2, mlp.D_IN))
    X[0, 0, 0], X[0, 1, 0] = 1.0, 2.0
    for tok, pos in enumerate(positions):
        X[0, tok, mlp.N_FEAT + pos] = 1.0
    return X


@pytest.mark.parametrize("bf16_points", [True, False])
def test_forward_and_backward_hand_worked(golden, bf16_points):
    """Forward outputs of two launch orders and every gradient element of one,
    worked by hand (tests/golden/mlp_hand.json)."""
    g = golden("mlp_hand.json")
    params = _hand_params(g["params"])
    for case in g["cases"]:
        y, _ = mlp.forward(params, _hand_tokens(case["positions"]), bf16_points)
        assert y[0] == case["y"]
    case = g["cases"][0]
    loss, y, grads = mlp.loss_and_grads(params, _hand_tokens(case["positions"]), [case["target"]],
                                        bf16_points)
    assert loss == case["loss"] and y[0] == case["y"]
    for name, shape in mlp.SHAPES:
        want = _hand_params({name: case["grads"].get(name, [])})[name]
        assert np.array_equal(grads[name].reshape(shape), want), name
