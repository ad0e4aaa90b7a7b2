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


def test_audit_rule_selects_one_in_64():
    h = np.arange(1 << 16)
    for frame in (0, 5):
        k = int(mlp.audited(frame, h).sum())
        n, p = len(h), 1.0 / 64
        assert abs(k - n * p) <= 4 * np.sqrt(n * p * (1 - p))
    # the rule depends on the frame
    assert not np.array_equal(mlp.audited(0, h), mlp.audited(1, h))


def test_targets_place_channels_by_ordinal():
    rec = np.zeros(3, dtype=[("ordinal", "<u4"), ("value", "<f4", (4,))])
    rec["ordinal"] = [0, 1, 2]
    rec["value"][0, :3] = [0.1, 0.2, 0.3]
    rec["value"][1, 0] = 0.7
    rec["value"][2, 0] = 0.9                     # ordinal 2 is not surrogated
    t, m = mlp.targets(rec, {0: (0, 3), 1: (3, 1)})
    assert np.allclose(t[0], [0.1, 0.2, 0.3, 0.0]) and np.array_equal(m[0], [1, 1, 1, 0])
    assert np.allclose(t[1], [0, 0, 0, 0.7]) and np.array_equal(m[1], [0, 0, 0, 1])
    assert not m[2].any()


def test_snapshot_substitution_with_a_constant_network():
    """A network with zero weights outputs its bias, so every substituted hit of
    the smooth material gets base colour = b3[0:3] and roughness = b3[3]
    (the sink takes both directly); audited hits keep their graph values and are
    inserted; substituted outputs are not."""
    from oracle import graph, render, table
    sc = scenes.smooth_scene(n_mats=1, width=80, height=40, frames=1)
    mat = sc.materials[0]
    cach = graph.cacheable_outputs(mat)
    assert [graph.output_type(mat, *c) for c in cach] == ["COLOR", "FLOAT"]
    params = [np.zeros((64, 32)), np.zeros(64), np.zeros((64, 64)), np.zeros(64),
              np.zeros((4, 64)), np.array([0.2, 0.3, 0.4, 0.5])]
    info = {0: dict(params=params, ordmap={0: (0, 3), 1: (3, 1)}, trusted=True)}
    h = sc.frame(0)
    t = table.Table(1 << 12, 8, 16)
    res = render.shade_snapshot_frame(sc.materials, sc.textures, h, t, 0, surrogate=info)
    sub = res.surrogate[:, 0] & res.surrogate[:, 1]
    aud = res.audited[:, 0]
    assert sub.sum() + aud.sum() == len(h)                  # empty table: every hit missed
    assert np.allclose(res.outputs["base_color"][sub], [0.2, 0.3, 0.4], rtol=0, atol=1e-12)
    assert np.allclose(res.outputs["roughness"][sub], 0.5, rtol=0, atol=1e-12)
    # only the audited hits' graph values were offered to the table
    assert res.stats["candidates"] == 2 * int(aud.sum())
    # and the live error is the distance of the graph values from the bias
    if aud.any():
        o = render.shade_uncached(sc.materials, sc.textures, h.take(np.nonzero(aud)[0]))
        e = max(np.abs(o["base_color"] - [0.2, 0.3, 0.4]).max(), np.abs(o["roughness"] - 0.5).max())
        assert abs(res.live_err[0] - e) < 1e-12
