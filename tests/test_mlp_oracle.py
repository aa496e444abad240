"""Pins of the FP64 reference of the learned proposer's network: the analytic
gradient against central finite differences, closed forms at zero parameters,
the bfloat16 rounding rule, and the first Adam step."""
import numpy as np

from oracle import mlp_oracle as M


def _rand_params(rng):
    return rng.normal(0, 0.4, M.N_PARAMS)


def _data(rng, n):
    x = np.concatenate([rng.uniform(-1, 1, (n, 16)), rng.integers(1, 6, (n, 1)) / 8.0], axis=1)
    y = rng.integers(0, 2, n).astype(np.float64)
    return x, y


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = _rand_params(rng)
    x, y = _data(rng, 40)
    L, g = M.loss_grad(p, x, y)
    assert abs(L - M.loss(p, x, y)) < 1e-12
    idx = rng.choice(M.N_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, [M.N_PARAMS - 1, 0, 17 * 64]])   # b3, W1[0][0], b1[0]
    h = 1e-6
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (M.loss(p + e, x, y) - M.loss(p - e, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_zero_parameters_closed_form():
    """All-zero parameters: z = 0, loss = log 2, only b3 has a gradient,
    mean(1/2 - y)."""
    rng = np.random.default_rng(1)
    x, y = _data(rng, 33)
    L, g = M.loss_grad(np.zeros(M.N_PARAMS), x, y)
    assert abs(L - np.log(2.0)) < 1e-15
    assert abs(g[-1] - np.mean(0.5 - y)) < 1e-15
    assert np.all(g[:-1] == 0.0)


def test_bf16_round_to_nearest_even():
    one = 1.0
    vals = np.array([one, one + 2 ** -8, one + 3 * 2 ** -8, one + 2 ** -8 + 2 ** -20, -2.5,
                     3.0e-3], np.float32)
    r = M.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # halfway, ties to even (down)
    assert r[2] == one + 2 ** -6             # halfway, ties to even (up)
    assert r[3] == one + 2 ** -7             # above halfway
    assert r[4] == -2.5                      # exactly representable
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = M.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_forward_close_to_exact():
    rng = np.random.default_rng(3)
    p = _rand_params(rng)
    x, _ = _data(rng, 64)
    z, zb = M.forward(p, x), M.forward_bf16(p, x)
    assert np.max(np.abs(z - zb)) < 0.05 * (1 + np.max(np.abs(z)))
