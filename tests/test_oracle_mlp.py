"""Pins of the surrogate reference: closed forms, finite differences, Adam's
first step, the counter-based batch sampler."""
import numpy as np

from oracle import mlp
from paper_2305_07238_amd import scenes


def _params(seed=0):
    return [p.astype(np.float64) for p in scenes.mlp_init(seed, 1)[0]]


def test_features_closed_forms():
    x = mlp.features(np.array([[0.0, 0.0], [2.0, 0.25]]))
    assert x.shape == (2, 32)
    assert np.allclose(x[0, 0::2], 0.0) and np.allclose(x[0, 1::2], 1.0)
    # u = 2 is an eighth of the period of w_0 = 2 pi / 16: sin = cos = 1 / sqrt 2
    assert np.isclose(x[1, 0], np.sqrt(0.5)) and np.isclose(x[1, 1], np.sqrt(0.5))
    # u = 2 is a quarter period of w_1 = 2 pi / 8: sin = 1, cos = 0
    assert np.isclose(x[1, 4], 1.0) and np.isclose(x[1, 5], 0.0, atol=1e-15)
    # v = 1/4 is a whole period of w_6 = 2 pi 4
    assert np.isclose(x[1, 4 * 6 + 2], 0.0, atol=1e-12) and np.isclose(x[1, 4 * 6 + 3], 1.0)
    # v = 1/8 is a whole period of the fastest feature, w_7 = 2 pi 8
    c = mlp.features(np.array([[0.0, 0.125]]))
    assert np.isclose(c[0, 30], 0.0, atol=1e-12) and np.isclose(c[0, 31], 1.0)
    # periodicity of the slowest feature: period 16
    a = mlp.features(np.array([[0.3, 0.7]]))
    b = mlp.features(np.array([[16.3, 16.7]]))
    assert np.allclose(a[0, :4], b[0, :4])


def test_zero_weights_give_the_output_bias():
    p = _params()
    p = [np.zeros_like(q) for q in p]
    p[5] = np.array([0.1, 0.2, 0.3, 0.4])
    y, _ = mlp.forward(p, mlp.features(np.random.default_rng(0).uniform(0, 4, (7, 2))))
    assert np.allclose(y, [0.1, 0.2, 0.3, 0.4])


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = _params(3)
    # shift the biases so every ReLU is away from its kink for this batch
    p[1] = p[1] + 0.05
    p[3] = p[3] + 0.05
    x = mlp.features(rng.uniform(0, 4, (16, 2)))
    t = rng.uniform(0, 1, (16, 4))
    mask = np.ones((16, 4))
    mask[:, 3] = 0.0
    loss, grads = mlp.loss_and_grads(p, x, t, mask)
    eps = 1e-6
    for k in range(6):
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(8, flat.size), replace=False):
            q = [a.copy() for a in p]
            q[k].ravel()[idx] += eps
            lp, _ = mlp.loss_and_grads(q, x, t, mask)
            q[k].ravel()[idx] -= 2 * eps
            lm, _ = mlp.loss_and_grads(q, x, t, mask)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grads[k].ravel()[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)
    # masked channel contributes nothing
    assert np.allclose(grads[4][3], 0.0) and grads[5][3] == 0.0


def test_fp16_rounding_points_change_little():
    rng = np.random.default_rng(2)
    p = _params(4)
    x = mlp.features(rng.uniform(0, 4, (64, 2)))
    t = rng.uniform(0, 1, (64, 4))
    m = np.ones((64, 4))
    _, g64 = mlp.loss_and_grads(p, x, t, m)
    _, g16 = mlp.loss_and_grads(p, x, t, m, round16=True)
    for a, b in zip(g64, g16):
        cos = float((a * b).sum() / (np.linalg.norm(a) * np.linalg.norm(b)))
        assert cos > 0.999


def test_adam_first_step_moves_by_lr_times_sign():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -0.25, 0.0])]
    z = [np.zeros(3)]
    q, m, v = mlp.adam_update(p, g, z, z, step=1, lr=0.01)
    assert np.allclose(q[0], [0.99, -1.99, 3.0], atol=1e-8)


def test_batch_sampler_is_reproducible_and_in_range():
    a = mlp.batch_indices(7, 3, 4096, 1000)
    b = mlp.batch_indices(7, 3, 4096, 1000)
    c = mlp.batch_indices(7, 4, 4096, 1000)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0 and a.max() < 1000
    counts = np.bincount(mlp.batch_indices(1, 0, 100000, 10), minlength=10)
    assert counts.min() > 9000 and counts.max() < 11000
