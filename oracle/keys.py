"""Descriptor of a cacheable output at a shading point (Sec. 3.1, Eq. 1, Sec. 3.2).

Eq. 1: lambda = -log2(min(|g1|, |g2|)) from the ray-cone UV gradients.
The virtual texture at level lambda has 2^lambda texels per unit of UV on
each axis (Sec. 3.1: resolution grows with the level) and the texel indices
come from the UV value.  The descriptor holds material id, node id, the level
and the texel indices (Sec. 3.1); Hash(desc) % N_c picks the cell and
Hash2(desc) is the verification key (Sec. 3.2, Algorithm 1).

Readings (the paper fixes none of these):
  * |g|^2 = gx*gx + gy*gy evaluated in binary64 from the binary32 inputs
    (both products are exact; one rounding on the sum); m2 = min(|g1|^2, |g2|^2);
  * integer level L = floor(lambda) + level_bias clamped to [0, level_max],
    where floor(lambda) = max{k : 4^k * m2 <= 1}; m2 == 0 gives level_max;
  * x = u * 2^L, y = v * 2^L (exact), tx = floor(x), ty = floor(y) as int32;
    no wrapping (UV outside [0, 1] is legal);
  * any non-finite u, v or gradient component, or |x|, |y| beyond int32,
    bypasses the cache (evaluate, never probe or insert);
  * descriptor words k0 = mat << 32 | node << 16 | socket << 8 | L,
    k1 = (u32)tx << 32 | (u32)ty;
  * cell = hi32(H(SEED_CELL)) % N_c, hash2 = lo32(H(SEED_VERIFY)), 0 -> 1
    (a stored hash of 0 would read as an empty entry in Algorithm 1).

World-space cells (Sec. 3.1 names the world position as other shading-point
information a descriptor may hold; reading): a POS-class output is keyed by a
virtual 3D grid of 2^L cells per world unit on each axis, with the same level
rule as Eq. 1 applied to the hit's world footprint width w (m2 = w^2, binary64
from the binary32 width); cell indices qx, qy, qz = floor(p * 2^L) (exact
scaling, int32 range or bypass); k0 as above with bit 7 of its low byte set
(L <= 30 needs 5 bits), k1 = (qx mod 2^21) << 42 | (qy mod 2^21) << 21 |
(qz mod 2^21) (indices wrap every 2^21 cells: far-apart cells may share a
descriptor, which the verification hash cannot tell apart either).

``hash2_mask`` keeps only some bits of the verification hash before the
0 -> 1 step.  It exists to force the verification collisions that Sec. 3.2
says cannot be avoided (with the full 32 bits they are too rare to observe),
so that false hits can be produced and counted; the method itself uses all
32 bits.
"""
import numpy as np

from .hashing import SEED_CELL, SEED_VERIFY, descriptor_hash

LEVEL_MAX_DEFAULT = 20


def squared_norms(duv):
    g = np.asarray(duv, dtype=np.float32).astype(np.float64)
    s1 = g[:, 0] * g[:, 0] + g[:, 1] * g[:, 1]
    s2 = g[:, 2] * g[:, 2] + g[:, 3] * g[:, 3]
    return s1, s2


def floor_lambda(m2):
    """max{k in Z : 4^k * m2 <= 1} for finite m2 > 0 (Eq. 1 rounded down)."""
    m2 = np.asarray(m2, dtype=np.float64)
    k = np.floor(-0.5 * np.log2(m2)).astype(np.int64)
    # exact correction against powers of two (ldexp is exact here)
    for _ in range(2):
        k = np.where(np.ldexp(m2, 2 * k) > 1.0, k - 1, k)
        k = np.where(np.ldexp(m2, 2 * (k + 1)) <= 1.0, k + 1, k)
    return k


def levels(duv, level_bias=0, level_max=LEVEL_MAX_DEFAULT):
    s1, s2 = squared_norms(duv)
    m2 = np.minimum(s1, s2)
    pos = m2 > 0
    f = np.where(pos & np.isfinite(m2), floor_lambda(np.where(pos & np.isfinite(m2), m2, 1.0)), 0)
    lv = np.clip(f + int(level_bias), 0, int(level_max))
    return np.where(pos, lv, int(level_max)).astype(np.int64)


class Keys:
    """Per-(hit, cacheable) descriptor fields for one material's hits."""

    def __init__(self, bypass, level, tx, ty, k0, k1, cell, hash2):
        self.bypass, self.level, self.tx, self.ty = bypass, level, tx, ty
        self.k0, self.k1, self.cell, self.hash2 = k0, k1, cell, hash2


def compute_keys(mat_id, node, socket, uv, duv, n_cells, level_bias=0,
                 level_max=LEVEL_MAX_DEFAULT, hash2_mask=0xFFFFFFFF) -> Keys:
    uv32 = np.asarray(uv, dtype=np.float32)
    duv32 = np.asarray(duv, dtype=np.float32)
    finite = np.all(np.isfinite(uv32), axis=1) & np.all(np.isfinite(duv32), axis=1)
    safe_duv = np.where(finite[:, None], duv32, np.float32(1.0))
    safe_uv = np.where(finite[:, None], uv32, np.float32(0.0)).astype(np.float64)
    lv = levels(safe_duv, level_bias, level_max)
    x = np.ldexp(safe_uv[:, 0], lv)
    y = np.ldexp(safe_uv[:, 1], lv)
    lim = 2.0 ** 31
    inrange = (x >= -lim) & (x < lim) & (y >= -lim) & (y < lim)
    bypass = ~(finite & inrange)
    tx = np.where(bypass, 0, np.floor(np.where(inrange, x, 0.0))).astype(np.int64)
    ty = np.where(bypass, 0, np.floor(np.where(inrange, y, 0.0))).astype(np.int64)
    U = np.uint64
    k0 = (U(mat_id) << U(32)) | (U(node) << U(16)) | (U(socket) << U(8)) | lv.astype(U)
    k1 = (tx.astype(np.uint32).astype(U) << U(32)) | ty.astype(np.uint32).astype(U)
    hc = descriptor_hash(k0, k1, SEED_CELL)
    hv = descriptor_hash(k0, k1, SEED_VERIFY)
    cell = ((hc >> U(32)) % U(n_cells)).astype(np.int64)
    h2 = (hv & U(int(hash2_mask) & 0xFFFFFFFF)).astype(np.int64)
    h2 = np.where(h2 == 0, 1, h2)
    return Keys(bypass, lv, tx, ty, k0, k1, cell, h2)


SPATIAL_FLAG = 0x80
SPATIAL_BITS = 21


def compute_keys_spatial(mat_id, node, socket, pos, width, n_cells, level_bias=0,
                         level_max=LEVEL_MAX_DEFAULT, hash2_mask=0xFFFFFFFF) -> Keys:
    """Descriptor of a POS-class output at world positions pos [n, 3] with
    footprint widths width [n].  tx, ty of the result hold qx, qy."""
    p32 = np.asarray(pos, dtype=np.float32)
    w32 = np.asarray(width, dtype=np.float32)
    finite = np.all(np.isfinite(p32), axis=1) & np.isfinite(w32)
    w64 = np.where(finite, w32, np.float32(1.0)).astype(np.float64)
    m2 = w64 * w64
    ok = m2 > 0
    f = np.where(ok & np.isfinite(m2), floor_lambda(np.where(ok & np.isfinite(m2), m2, 1.0)), 0)
    lv = np.where(ok, np.clip(f + int(level_bias), 0, int(level_max)), int(level_max))
    lv = lv.astype(np.int64)
    safe = np.where(finite[:, None], p32, np.float32(0.0)).astype(np.float64)
    q = np.ldexp(safe, lv[:, None])
    lim = 2.0 ** 31
    inrange = np.all((q >= -lim) & (q < lim), axis=1)
    bypass = ~(finite & inrange)
    qi = np.where(bypass[:, None], 0, np.floor(np.where(inrange[:, None], q, 0.0))).astype(np.int64)
    U = np.uint64
    M = U((1 << SPATIAL_BITS) - 1)
    k0 = (U(mat_id) << U(32)) | (U(node) << U(16)) | (U(socket) << U(8)) | U(SPATIAL_FLAG) | \
        lv.astype(U)
    qu = qi.astype(np.uint32).astype(U) & M
    k1 = (qu[:, 0] << U(2 * SPATIAL_BITS)) | (qu[:, 1] << U(SPATIAL_BITS)) | qu[:, 2]
    hc = descriptor_hash(k0, k1, SEED_CELL)
    hv = descriptor_hash(k0, k1, SEED_VERIFY)
    cell = ((hc >> U(32)) % U(n_cells)).astype(np.int64)
    h2 = (hv & U(int(hash2_mask) & 0xFFFFFFFF)).astype(np.int64)
    h2 = np.where(h2 == 0, 1, h2)
    return Keys(bypass, lv, qi[:, 0], qi[:, 1], k0, k1, cell, h2)


def keys_for(material, mat_id, node, socket, hits, idx, n_cells, level_bias=0,
             level_max=LEVEL_MAX_DEFAULT, hash2_mask=0xFFFFFFFF) -> Keys:
    """Keys of cacheable output (node, socket) for hits[idx]: a UV texel, or a
    world-space cell for a POS-class output."""
    from . import graph
    if graph.key_kind(material, node) == graph.POS:
        return compute_keys_spatial(mat_id, node, socket, hits.position[idx], hits.width[idx],
                                    n_cells, level_bias, level_max, hash2_mask)
    return compute_keys(mat_id, node, socket, hits.uv[idx], hits.duv[idx], n_cells, level_bias,
                        level_max, hash2_mask)
