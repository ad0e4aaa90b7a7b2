"""Ray-cone footprints: texture-coordinate gradients g1, g2 of a hit (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 3.1: the intersection of a ray cone with the surface is an ellipse, and
the texture-coordinate gradients g1 and g2 are its two axes carried into UV
space (after Akenine-Moller et al. 2021, "Improved shader and texture level of
detail using ray cones"); Eq. 1 then takes the level from the shorter one.

Reading (the paper gives no formulas; this is the geometry restated):
  * inputs per hit: the ray direction d (any length), the cone radius r at the
    hit (the renderer tracks the cone's width along the path), the hit
    triangle's edges e1 = P1 - P0, e2 = P2 - P0 and its UV edges
    t1 = uv1 - uv0, t2 = uv2 - uv0;
  * the surface is the triangle's plane, unit normal m = (e1 x e2) / |e1 x e2|;
    a cone of radius r around the ray meets it in an ellipse whose semi-axes
    are a1 = r / |cos| along the ray direction projected onto the plane, and
    a2 = r along the plane direction perpendicular to it (cos = d.m / |d|);
    |cos| is clamped below at 1/1024, so a grazing ray stretches the footprint
    at most 1024 times;
  * when the ray is (within 1e-4 rad) perpendicular to the plane the projected
    direction is undefined; the axes are then r times the tangent frame of m of
    Duff et al. 2017 (JCGT 6(1)), the same frame the normal-map node uses;
  * an in-plane vector a moves the barycentric coordinates by
    du = ((a x e2) . n) / (n . n), dv = ((e1 x a) . n) / (n . n) with
    n = e1 x e2, hence the UV by du t1 + dv t2: g1 from a1, g2 from a2;
  * a degenerate triangle (n = 0), a zero direction, or any non-finite input
    gives NaN gradients, which make the hit bypass the cache.
"""
import numpy as np

MIN_COS = 1.0 / 1024.0
HEAD_ON = 1e-4


def _onb(m):
    sign = np.where(m[:, 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + m[:, 2])
    b = m[:, 0] * m[:, 1] * a
    t = np.stack([1.0 + sign * m[:, 0] * m[:, 0] * a, sign * b, -sign * m[:, 0]], 1)
    bb = np.stack([b, sign + m[:, 1] * m[:, 1] * a, -m[:, 1]], 1)
    return t, bb


def ellipse_axes(d, r, e1, e2):
    """Semi-axis vectors (a1, a2) of the footprint ellipse in world space, [n, 3]
    each, and a validity mask."""
    d = np.asarray(d, np.float64)
    r = np.asarray(r, np.float64)
    e1 = np.asarray(e1, np.float64)
    e2 = np.asarray(e2, np.float64)
    n = np.cross(e1, e2)
    nn = np.sum(n * n, axis=1)
    dl = np.sqrt(np.sum(d * d, axis=1))
    ok = (nn > 0) & (dl > 0) & np.isfinite(nn) & np.isfinite(dl) & np.isfinite(r)
    with np.errstate(all="ignore"):
        m = n / np.sqrt(nn)[:, None]
        dh = d / dl[:, None]
        c = np.sum(dh * m, axis=1)
        h = dh - c[:, None] * m
        hl = np.sqrt(np.sum(h * h, axis=1))
        head_on = hl < HEAD_ON
        t1 = h / np.where(head_on, 1.0, hl)[:, None]
        t2 = np.cross(m, t1)
        ft, fb = _onb(m)
        ac = np.maximum(np.abs(c), MIN_COS)
        a1 = np.where(head_on[:, None], ft * r[:, None], t1 * (r / ac)[:, None])
        a2 = np.where(head_on[:, None], fb * r[:, None], t2 * r[:, None])
    return a1, a2, ok


def uv_of_offset(a, e1, e2, t1, t2):
    """UV change of an in-plane world offset a (barycentric coordinates of the plane)."""
    e1 = np.asarray(e1, np.float64)
    e2 = np.asarray(e2, np.float64)
    n = np.cross(e1, e2)
    nn = np.sum(n * n, axis=1)
    with np.errstate(all="ignore"):
        du = np.sum(np.cross(a, e2) * n, axis=1) / nn
        dv = np.sum(np.cross(e1, a) * n, axis=1) / nn
    return du[:, None] * np.asarray(t1, np.float64) + dv[:, None] * np.asarray(t2, np.float64)


def gradients(d, r, e1, e2, t1, t2):
    """[n, 4] = g1.x, g1.y, g2.x, g2.y (the layout of the hits' duv); NaN rows for
    invalid inputs."""
    a1, a2, ok = ellipse_axes(d, r, e1, e2)
    g1 = uv_of_offset(a1, e1, e2, t1, t2)
    g2 = uv_of_offset(a2, e1, e2, t1, t2)
    g = np.concatenate([g1, g2], axis=1)
    fin = ok & np.all(np.isfinite(g), axis=1) & np.all(np.isfinite(np.asarray(t1)), axis=1) & \
        np.all(np.isfinite(np.asarray(t2)), axis=1)
    g[~fin] = np.nan
    return g
