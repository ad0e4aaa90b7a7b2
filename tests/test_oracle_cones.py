"""Pins of the ray-cone footprint oracle (oracle/cones.py): closed forms, a
least-squares solve for the barycentric map, the footprint ellipse sampled
from the cone's cross-section, invariances and degenerate inputs."""
import numpy as np

from oracle import cones, keys as K

XY = (np.array([[1.0, 0, 0]]), np.array([[0.0, 1, 0]]))       # unit right triangle, z = 0
UVXY = (np.array([[1.0, 0]]), np.array([[0.0, 1]]))           # uv = (x, y)


def _g(d, r, e=XY, t=UVXY):
    return cones.gradients(np.atleast_2d(d), np.atleast_1d(r), e[0], e[1], t[0], t[1])[0]


def test_head_on_identity_mapping_gives_radius():
    r = 1.0 / 64
    g = _g([0, 0, -1.0], r)
    assert np.allclose(g, [r, 0, 0, r], atol=1e-15)
    # Eq. 1 on it: the level of the tiny scene's footprints
    lv = K.compute_keys(0, 0, 0, np.array([[0.5, 0.5]], np.float32),
                        g[None].astype(np.float32), 8).level
    assert lv[0] == 6


def test_oblique_ray_stretches_along_its_projection():
    r = 0.01
    for th in (0.3, 1.0, 1.4):
        g = _g([np.sin(th), 0, -np.cos(th)], r)
        assert np.allclose(g, [r / np.cos(th), 0, 0, r], rtol=1e-13, atol=1e-16)


def test_grazing_ray_is_clamped():
    r = 0.01
    th = np.pi / 2 - 1e-6
    g = _g([np.sin(th), 0, -np.cos(th)], r)
    assert np.isclose(g[0], r * 1024.0, rtol=1e-12)


def test_uv_scale_and_rotation():
    r, s, phi = 0.02, 3.5, 0.7
    R = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
    t = (s * R @ UVXY[0][0], s * R @ UVXY[1][0])
    g = _g([0.3, -0.2, -1.0], r, t=(t[0][None], t[1][None]))
    g0 = _g([0.3, -0.2, -1.0], r)
    assert np.allclose(g[:2], s * R @ g0[:2]) and np.allclose(g[2:], s * R @ g0[2:])


def _random_case(rng, n):
    e1 = rng.normal(size=(n, 3))
    e2 = rng.normal(size=(n, 3))
    d = rng.normal(size=(n, 3))
    r = rng.uniform(1e-3, 0.1, n)
    t1 = rng.normal(size=(n, 2))
    t2 = rng.normal(size=(n, 2))
    return d, r, e1, e2, t1, t2


def test_barycentric_map_matches_a_least_squares_solve():
    rng = np.random.default_rng(1)
    d, r, e1, e2, t1, t2 = _random_case(rng, 200)
    n = np.cross(e1, e2)
    for i in range(200):
        a = rng.normal(size=3)
        a -= (a @ n[i]) / (n[i] @ n[i]) * n[i]                 # in the plane
        bc, *_ = np.linalg.lstsq(np.stack([e1[i], e2[i]], 1), a, rcond=None)
        want = bc[0] * t1[i] + bc[1] * t2[i]
        got = cones.uv_of_offset(a[None], e1[i:i + 1], e2[i:i + 1], t1[i:i + 1], t2[i:i + 1])[0]
        assert np.allclose(got, want, rtol=1e-9, atol=1e-12)


def test_axes_match_the_sampled_cone_cross_section():
    """Points of the cone's circular cross-section (radius r, perpendicular to the
    ray) projected along the ray onto the plane form the footprint ellipse: its
    longest and shortest radii are |a1| and |a2|, in their directions."""
    rng = np.random.default_rng(2)
    d, r, e1, e2, t1, t2 = _random_case(rng, 100)
    a1, a2, ok = cones.ellipse_axes(d, r, e1, e2)
    phi = np.linspace(0, 2 * np.pi, 20001)
    for i in range(100):
        m = np.cross(e1[i], e2[i])
        m /= np.linalg.norm(m)
        dh = d[i] / np.linalg.norm(d[i])
        if abs(dh @ m) < 1.0 / 1024:
            continue
        u = np.cross(dh, [0.3, 0.5, 0.8])
        u /= np.linalg.norm(u)
        w = np.cross(dh, u)
        q = r[i] * (np.cos(phi)[:, None] * u + np.sin(phi)[:, None] * w)
        p = q - ((q @ m) / (dh @ m))[:, None] * dh
        rad = np.linalg.norm(p, axis=1)
        # 20,001 samples: the extrema are found to ~1e-5 relative on these
        # ellipses (axis ratios below ~30)
        assert np.isclose(rad.max(), np.linalg.norm(a1[i]), rtol=1e-4)
        assert np.isclose(rad.min(), np.linalg.norm(a2[i]), rtol=1e-4)
        pmax = p[np.argmax(rad)] / rad.max()
        assert abs(abs(pmax @ a1[i]) / np.linalg.norm(a1[i]) - 1) < 1e-4


def test_rotation_of_the_world_leaves_gradients_unchanged():
    rng = np.random.default_rng(3)
    d, r, e1, e2, t1, t2 = _random_case(rng, 50)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.linalg.det(q))                             # a rotation
    g = cones.gradients(d, r, e1, e2, t1, t2)
    gq = cones.gradients(d @ q.T, r, e1 @ q.T, e2 @ q.T, t1, t2)
    assert np.allclose(g, gq, rtol=1e-9, atol=1e-12)


def test_vertex_order_flips_only_the_minor_axis():
    rng = np.random.default_rng(4)
    d, r, e1, e2, t1, t2 = _random_case(rng, 50)
    g = cones.gradients(d, r, e1, e2, t1, t2)
    gs = cones.gradients(d, r, e2, e1, t2, t1)
    assert np.allclose(gs[:, :2], g[:, :2], rtol=1e-9, atol=1e-12)
    assert np.allclose(gs[:, 2:], -g[:, 2:], rtol=1e-9, atol=1e-12)


def test_degenerate_inputs_give_nan():
    e1 = np.array([[1.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0]])
    e2 = np.array([[2.0, 0, 0], [0, 1.0, 0], [0, 1.0, 0], [0, 1.0, 0]])  # collinear, ok, ok, ok
    d = np.array([[0, 0, -1.0], [0, 0, 0], [0, 0, -1.0], [np.inf, 0, -1]])
    r = np.array([0.01, 0.01, np.nan, 0.01])
    t = np.array([[1.0, 0]] * 4), np.array([[0.0, 1]] * 4)
    g = cones.gradients(d, r, e1, e2, t[0], t[1])
    assert np.all(np.isnan(g))
