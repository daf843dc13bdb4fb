"""Pins for the FP64 reference of the chooser network: central finite
differences, closed-form gradients of hand-built networks, and the known
first Adam step."""

import numpy as np

from oracle import mlp as M


def _rand(seed, nb=40):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(M.NPARAM) * 0.3
    x = rng.standard_normal((nb, M.NI))
    t = rng.standard_normal((nb, M.NO))
    mask = rng.random((nb, M.NO)) < 0.7
    return p, x, t, mask


def test_param_count():
    assert M.NPARAM == 5648


def test_gradient_matches_central_differences():
    p, x, t, mask = _rand(1)
    g, _ = M.grad(p, x, t, mask)
    _, (z1, _, z2, _) = M.forward(p, x)
    h = 1e-6
    assert np.abs(z1).min() > 1e-4 and np.abs(z2).min() > 1e-4  # no ReLU kink within h
    rng = np.random.default_rng(2)
    for k in rng.choice(M.NPARAM, 300, replace=False):
        e = np.zeros(M.NPARAM)
        e[k] = h
        fd = (M.loss(p + e, x, t, mask) - M.loss(p - e, x, t, mask)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_closed_form_bias_only_network():
    rng = np.random.default_rng(3)
    nb = 25
    c = rng.standard_normal(M.NO)
    p = M.pack({"W1": np.zeros((6, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)),
                "b2": np.zeros(64), "W3": np.zeros((64, 16)), "b3": c})
    x = rng.standard_normal((nb, 6))
    t = rng.standard_normal((nb, 16))
    mask = rng.random((nb, 16)) < 0.5
    g, L = M.grad(p, x, t, mask)
    count = mask.sum()
    want_b3 = 2.0 * (mask * (c - t)).sum(0) / count
    w = M.unpack(g)
    assert np.allclose(w["b3"], want_b3, rtol=1e-14, atol=1e-15)
    for name in ("W1", "b1", "W2", "b2", "W3"):
        assert np.all(w[name] == 0.0), name
    assert np.isclose(L, ((mask * (c - t)) ** 2).sum() / count, rtol=1e-14)


def test_closed_form_single_path_network():
    # y0 = a * x0 through one unit per layer (x0 > 0 keeps every ReLU open)
    a = 0.7
    d = {"W1": np.zeros((6, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)),
         "b2": np.zeros(64), "W3": np.zeros((64, 16)), "b3": np.zeros(16)}
    d["W1"][0, 0] = 1.0
    d["W2"][0, 0] = 1.0
    d["W3"][0, 0] = a
    p = M.pack(d)
    rng = np.random.default_rng(4)
    x = np.zeros((30, 6))
    x[:, 0] = rng.uniform(0.5, 2.0, 30)
    t = rng.standard_normal((30, 16))
    mask = np.zeros((30, 16), bool)
    mask[:, 0] = True
    g = M.unpack(M.grad(p, x, t, mask)[0])
    r = a * x[:, 0] - t[:, 0]
    assert np.isclose(g["W3"][0, 0], 2 * (r * x[:, 0]).sum() / 30, rtol=1e-13)
    assert np.isclose(g["W2"][0, 0], 2 * (r * a * x[:, 0]).sum() / 30, rtol=1e-13)
    assert np.isclose(g["W1"][0, 0], 2 * (r * a * x[:, 0]).sum() / 30, rtol=1e-13)
    assert np.isclose(g["b3"][0], 2 * r.sum() / 30, rtol=1e-13)


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    p1, m, v = M.adam(p, g, np.zeros(100), np.zeros(100), 1, lr=0.01)
    # bias-corrected moments equal g and g^2 at step 1
    assert np.allclose(p - p1, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss_on_a_learnable_target():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((200, 6))
    t = np.tile((x @ rng.standard_normal((6, 1))), (1, 16)) + 0.1 * rng.standard_normal((200, 16))
    mask = np.ones((200, 16), bool)
    p = rng.standard_normal(M.NPARAM) * 0.1
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = M.loss(p, x, t, mask)
    for step in range(1, 301):
        g, _ = M.grad(p, x, t, mask)
        p, m, v = M.adam(p, g, m, v, step, lr=3e-3)
    assert M.loss(p, x, t, mask) < 0.2 * l0
