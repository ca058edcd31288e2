"""Pins for the CPU reference of the band-proposal network (no GPU)."""
import numpy as np

from oracle import mlp_ref


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 3.140625])
    r = mlp_ref.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # halfway: ties to even
    assert r[2] == 1.0 + 2 ** -7            # above halfway rounds up
    assert r[3] == -2.5 and r[4] == 0.0 and r[5] == 3.140625
    h = mlp_ref.bf16_bits(x)
    assert np.array_equal(mlp_ref.from_bf16_bits(h), r)


def test_softmax_xent_closed_forms():
    z = np.zeros((5, 64))
    loss, g = mlp_ref.softmax_xent(z, np.arange(5))
    assert abs(loss - np.log(64)) < 1e-12
    assert np.allclose(g.sum(axis=1), 0.0, atol=1e-15)
    z = np.full((3, 4), -50.0)
    z[np.arange(3), [1, 2, 3]] = 50.0
    loss, _ = mlp_ref.softmax_xent(z, np.array([1, 2, 3]))
    assert loss < 1e-40


def test_softmax_xent_ignores_rows_without_label():
    rng = np.random.default_rng(2)
    z = rng.normal(size=(6, 64))
    lab = np.array([3, -1, 10, 64, 0, -7])
    loss, g = mlp_ref.softmax_xent(z, lab)
    keep = [0, 2, 4]
    l2, g2 = mlp_ref.softmax_xent(z[keep], lab[keep])
    assert abs(loss - l2 * 3 / 6) < 1e-12            # same sum, divisor 6
    assert np.allclose(g[keep], g2 * 3 / 6, atol=1e-15)
    assert np.all(g[[1, 3, 5]] == 0.0)


def test_gradients_match_finite_differences():
    """Back-propagation against central differences of the loss (FP64)."""
    dims = (7, 6, 5, 4)
    params = mlp_ref.init_params(3, dims)
    rng = np.random.default_rng(4)
    for p in params[1::2]:
        p += rng.normal(0, 0.1, size=p.shape)
    x = rng.normal(size=(9, 7))
    labels = rng.integers(0, 4, size=9)
    logits, cache = mlp_ref.forward(params, x)
    _, dl = mlp_ref.softmax_xent(logits, labels)
    grads = mlp_ref.backward(params, cache, dl)
    h = 1e-6
    for p, g in zip(params, grads):
        for idx in list(np.ndindex(p.shape))[:25]:
            old = p[idx]
            p[idx] = old + h
            lp = mlp_ref.loss(params, x, labels)
            p[idx] = old - h
            lm = mlp_ref.loss(params, x, labels)
            p[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-7 + 1e-6 * abs(fd), (idx, fd, g[idx])


def test_adam_first_step_moves_by_lr():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    q, m, v = mlp_ref.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(q, p - 0.01 * np.sign(g), atol=1e-15)
