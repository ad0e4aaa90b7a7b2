"""Node definitions, evaluated in FP64 over arrays of shading points.

The paper names no node types (Sec. 2 only says networks are evaluated "in
the standard way").  The node set below is the one the workloads use, each
stated once here and independently in the HIP interpreter:

  IMAGE_TEXTURE  bilinear RGBA8 lookup, repeat wrap, texel centres at
                 (i + 1/2) / W, linear UNORM8 (byte / 255), row 0 at v = 0.
  VALUE_NOISE    lattice value noise, smoothstep weights t^2 (3 - 2t),
                 octave o at frequency f0 * 2^o with weight 2^-o, normalised.
  PERLIN_NOISE   gradient noise (Perlin, "Improving Noise", SIGGRAPH 2002):
                 8 corner gradients, quintic fade 6t^5 - 15t^4 + 10t^3,
                 same octave sum, mapped to 0.5 + 0.5 n.
  MIX            a + clamp(fac, 0, 1) (b - a), per channel.
  MATH           ADD a + b, MUL a b, POW (a > 0 ? a^b : 0), optional clamp to [0, 1].
  COLOR_RAMP     8 stops, linear interpolation between neighbouring stops,
                 constant outside [pos_0, pos_7].
  NORMAL_MAP     tangent-space colour -> world normal with the orthonormal
                 basis of Duff et al. 2017 (JCGT 6(1)), strength blend.
  POSITION_NOISE value noise of the world position: octave o at frequency
                 f0 2^o, lattice corner (i, j, k) valued
                 hash32(((u32)i << 32 | (u32)j) ^ mix64((u32)k ^ (seed + o) G)) 2^-32
                 (G the 64-bit golden constant), trilinear interpolation with
                 smoothstep weights, octaves weighted 2^-o and normalised.
"""
import numpy as np

from .hashing import lattice_hash32

INV_2_32 = 2.0 ** -32


def lerp(a, b, t):
    return a + t * (b - a)


def image_texture(tex, uv):
    """tex: uint8 [H, W, 4]; uv: [n, 2].  Returns (rgb [n, 3], alpha [n])."""
    h, w = tex.shape[0], tex.shape[1]
    x = uv[:, 0] * w - 0.5
    y = uv[:, 1] * h - 0.5
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = (x - x0)[:, None]
    fy = (y - y0)[:, None]
    i0 = np.mod(x0.astype(np.int64), w)
    i1 = np.mod(x0.astype(np.int64) + 1, w)
    j0 = np.mod(y0.astype(np.int64), h)
    j1 = np.mod(y0.astype(np.int64) + 1, h)
    t = tex.astype(np.float64) / 255.0
    c = lerp(lerp(t[j0, i0], t[j0, i1], fx), lerp(t[j1, i0], t[j1, i1], fx), fy)
    return c[:, :3], c[:, 3]


def _octaves(uv, f0, octaves, seed, one_octave):
    total = np.zeros(uv.shape[0])
    norm = 0.0
    for o in range(octaves):
        freq = f0 * 2.0 ** o
        amp = 0.5 ** o
        total = total + amp * one_octave(uv[:, 0] * freq, uv[:, 1] * freq, seed + o)
        norm += amp
    return total / norm


def _value_octave(px, py, seed):
    i = np.floor(px)
    j = np.floor(py)
    fx, fy = px - i, py - j
    i = i.astype(np.int64)
    j = j.astype(np.int64)

    def corner(a, b):
        return lattice_hash32(a, b, seed).astype(np.float64) * INV_2_32

    sx = fx * fx * (3.0 - 2.0 * fx)
    sy = fy * fy * (3.0 - 2.0 * fy)
    return lerp(lerp(corner(i, j), corner(i + 1, j), sx),
                lerp(corner(i, j + 1), corner(i + 1, j + 1), sx), sy)


# the 8 corner gradients, indexed by hash & 7
GRADIENTS = np.array([(1, 0), (-1, 0), (0, 1), (0, -1),
                      (1, 1), (-1, 1), (1, -1), (-1, -1)], dtype=np.float64)


def _perlin_octave(px, py, seed):
    i = np.floor(px)
    j = np.floor(py)
    fx, fy = px - i, py - j
    i = i.astype(np.int64)
    j = j.astype(np.int64)

    def dot(a, b, dx, dy):
        g = GRADIENTS[(lattice_hash32(a, b, seed) & np.uint64(7)).astype(np.int64)]
        return g[:, 0] * dx + g[:, 1] * dy

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    qx, qy = fade(fx), fade(fy)
    return lerp(lerp(dot(i, j, fx, fy), dot(i + 1, j, fx - 1.0, fy), qx),
                lerp(dot(i, j + 1, fx, fy - 1.0), dot(i + 1, j + 1, fx - 1.0, fy - 1.0), qx), qy)


def value_noise(uv, f0, octaves, seed):
    return _octaves(uv, f0, octaves, seed, _value_octave)


def perlin_noise(uv, f0, octaves, seed):
    return 0.5 + 0.5 * _octaves(uv, f0, octaves, seed, _perlin_octave)


def mix(fac, a, b):
    t = np.clip(fac, 0.0, 1.0)[:, None]
    return a + t * (b - a)


def math_op(op, a, b, clamp):
    if op == "ADD":
        r = a + b
    elif op == "MUL":
        r = a * b
    elif op == "POW":
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            r = np.where(a > 0, np.power(np.where(a > 0, a, 1.0), b), 0.0)
    else:
        raise ValueError(op)
    if clamp:
        r = np.clip(r, 0.0, 1.0)
    return r


def color_ramp(fac, pos, rgba):
    """fac: [n]; pos: 8 ascending floats; rgba: [8, 4].  Returns (rgb, alpha)."""
    pos = np.asarray(pos, dtype=np.float64)
    rgba = np.asarray(rgba, dtype=np.float64)
    n = fac.shape[0]
    out = np.empty((n, 4))
    lo = fac <= pos[0]
    hi = fac >= pos[-1]
    out[lo] = rgba[0]
    out[hi & ~lo] = rgba[-1]
    mid = ~(lo | hi)
    if np.any(mid):
        f = fac[mid]
        k = np.searchsorted(pos, f, side="right") - 1      # pos[k] <= f < pos[k+1]
        t = ((f - pos[k]) / (pos[k + 1] - pos[k]))[:, None]
        out[mid] = lerp(rgba[k], rgba[k + 1], t)
    return out[:, :3], out[:, 3]


def _normalize(v, fallback):
    ln = np.sqrt(np.sum(v * v, axis=1))
    ok = ln >= 1e-12
    out = np.where(ok[:, None], v / np.where(ok, ln, 1.0)[:, None], fallback)
    return out


def onb_duff(n):
    """Tangent frame (t, b) of unit normal n after Duff et al. 2017 (JCGT 6(1)); sign = +1 when n.z >= 0."""
    sign = np.where(n[:, 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t = np.stack([1.0 + sign * n[:, 0] * n[:, 0] * a, sign * b, -sign * n[:, 0]], 1)
    bb = np.stack([b, sign + n[:, 1] * n[:, 1] * a, -n[:, 1]], 1)
    return t, bb


def normal_map(color, strength, n):
    """color: [n, 3] in [0, 1]; strength: [n]; n: [n, 3] unit hit normal."""
    t = 2.0 * color - 1.0
    tx, bx = onb_duff(n)
    v = t[:, 0:1] * tx + t[:, 1:2] * bx + t[:, 2:3] * n
    v = _normalize(v, n)
    return _normalize(n + strength[:, None] * (v - n), n)


def position_noise(p, f0, octaves, seed):
    """p: [n, 3] world positions; returns [n] in [0, 1)."""
    from .hashing import GOLDEN, mix64
    p = np.asarray(p, dtype=np.float64)
    total = np.zeros(p.shape[0])
    norm = 0.0
    for o in range(int(octaves)):
        freq = f0 * 2.0 ** o
        x = p * freq
        c0 = np.floor(x)
        f = x - c0
        w = f * f * (3.0 - 2.0 * f)
        ci = c0.astype(np.int64)
        sg = np.uint64((((int(seed) + o) & 0xFFFFFFFF) * int(GOLDEN)) & 0xFFFFFFFFFFFFFFFF)
        val = np.zeros(p.shape[0])
        for dz in (0, 1):
            kz = mix64((ci[:, 2] + dz).astype(np.uint32).astype(np.uint64) ^ sg)
            for dy in (0, 1):
                for dx in (0, 1):
                    ij = ((ci[:, 0] + dx).astype(np.uint32).astype(np.uint64) << np.uint64(32)) | \
                        (ci[:, 1] + dy).astype(np.uint32).astype(np.uint64)
                    h = (mix64(ij ^ kz) & np.uint64(0xFFFFFFFF)).astype(np.float64) * INV_2_32
                    wx = w[:, 0] if dx else 1.0 - w[:, 0]
                    wy = w[:, 1] if dy else 1.0 - w[:, 1]
                    wz = w[:, 2] if dz else 1.0 - w[:, 2]
                    val += wx * wy * wz * h
        total += 0.5 ** o * val
        norm += 0.5 ** o
    return total / norm
