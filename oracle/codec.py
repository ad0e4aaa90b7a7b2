"""The 32-bit value encodings packed beside Hash2 in one 64-bit table word.

Sec. 3.3 encodes a cacheable node's output as one 32-bit value but does not
say how.  Reading used here:
  FLOAT output  -> the IEEE-754 binary32 bit pattern of the value;
  COLOR output  -> RGB9E5, the shared-exponent format of the Khronos
                   EXT_texture_shared_exponent extension (N = 9 mantissa bits,
                   B = 15 exponent bias, Emax = 31), restated from that
                   specification and evaluated exactly on the real input.
"""
import numpy as np

N_BITS = 9
BIAS = 15
EMAX = 31
MAX_RGB9E5 = (2 ** N_BITS - 1) / 2 ** N_BITS * 2.0 ** (EMAX - BIAS)   # 65408


def float_encode(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)


def float_decode(enc):
    return np.asarray(enc, dtype=np.uint64).astype(np.uint32).view(np.float32).astype(np.float64)


def _floor_log2(x):
    """Largest integer k with 2^k <= x, for finite x > 0 (exact via ldexp comparisons)."""
    x = np.asarray(x, dtype=np.float64)
    k = np.floor(np.log2(x)).astype(np.int64)
    # correct any libm rounding: enforce 2^k <= x < 2^(k+1) exactly
    k = np.where(np.ldexp(1.0, k) > x, k - 1, k)
    k = np.where(np.ldexp(1.0, k + 1) <= x, k + 1, k)
    return k


def rgb9e5_encode(rgb):
    """Encode [n, 3] real colours; returns uint64 codes (low 32 bits used)."""
    c = np.asarray(rgb, dtype=np.float64).reshape(-1, 3)
    c = np.where(np.isnan(c), 0.0, c)
    c = np.clip(c, 0.0, MAX_RGB9E5)
    maxc = c.max(axis=1)
    safe = np.where(maxc > 0, maxc, 1.0)
    fl = np.where(maxc > 0, _floor_log2(safe), -BIAS - 1)
    exp_p = np.maximum(-BIAS - 1, fl) + 1 + BIAS
    max_s = np.floor(maxc / np.ldexp(1.0, exp_p - BIAS - N_BITS) + 0.5)
    exp = np.where(max_s == 2 ** N_BITS, exp_p + 1, exp_p)
    m = np.floor(c / np.ldexp(1.0, exp - BIAS - N_BITS)[:, None] + 0.5).astype(np.uint64)
    code = m[:, 0] | (m[:, 1] << np.uint64(9)) | (m[:, 2] << np.uint64(18)) | \
        (exp.astype(np.uint64) << np.uint64(27))
    return code


def rgb9e5_decode(code):
    code = np.asarray(code, dtype=np.uint64).reshape(-1)
    m = np.stack([(code >> np.uint64(s)) & np.uint64(0x1FF) for s in (0, 9, 18)], 1)
    e = ((code >> np.uint64(27)) & np.uint64(0x1F)).astype(np.int64)
    return m.astype(np.float64) * np.ldexp(1.0, e - BIAS - N_BITS)[:, None]


def rgb9e5_step(code):
    """Size of one mantissa step at the code's shared exponent."""
    e = ((np.asarray(code, dtype=np.uint64) >> np.uint64(27)) & np.uint64(0x1F)).astype(np.int64)
    return np.ldexp(1.0, e - BIAS - N_BITS)
