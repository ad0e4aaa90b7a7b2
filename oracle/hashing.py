"""Integer hashing used by the descriptor and by the noise lattices.

The paper delegates its two hash functions to Binder et al. 2022 without
stating them (Sec. 3.2).  This reading uses the SplitMix64 output finalizer
(Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), re-stated here from that publication:

    z ^= z >> 30;  z *= 0xBF58476D1CE4E5B9
    z ^= z >> 27;  z *= 0x94D049BB133111EB
    z ^= z >> 31

All arithmetic is modulo 2^64 on numpy uint64 arrays (wrap-around is the
intended semantics).
"""
import numpy as np

U64 = np.uint64
GOLDEN = U64(0x9E3779B97F4A7C15)         # SplitMix64 state increment
SEED_CELL = U64(0x9E3779B97F4A7C15)      # seed of Hash  (cell index)
SEED_VERIFY = U64(0xC2B2AE3D27D4EB4F)    # seed of Hash2 (verification key)


def mix64(z):
    z = np.asarray(z, dtype=U64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> U64(30))
        z = z * U64(0xBF58476D1CE4E5B9)
        z = z ^ (z >> U64(27))
        z = z * U64(0x94D049BB133111EB)
        z = z ^ (z >> U64(31))
    return z


def splitmix64_sequence(seed: int, n: int):
    """The SplitMix64 generator itself (state += golden; output mix64(state))."""
    out = []
    state = U64(seed)
    with np.errstate(over="ignore"):
        for _ in range(n):
            state = U64(state + GOLDEN)
            out.append(int(mix64(state)))
    return out


def lattice_hash32(i, j, seed):
    """Noise corner hash: low 32 bits of mix64(((u32)i << 32 | (u32)j) ^ seed * golden)."""
    i = np.asarray(i, dtype=np.int64).astype(np.uint32).astype(U64)
    j = np.asarray(j, dtype=np.int64).astype(np.uint32).astype(U64)
    with np.errstate(over="ignore"):
        s = U64(int(seed) & 0xFFFFFFFF) * GOLDEN
    z = mix64(((i << U64(32)) | j) ^ s)
    return (z & U64(0xFFFFFFFF)).astype(np.uint64)


def descriptor_hash(k0, k1, seed):
    """H(seed) = mix64(k1 ^ mix64(k0 ^ seed)) over the two 64-bit descriptor words."""
    k0 = np.asarray(k0, dtype=U64)
    k1 = np.asarray(k1, dtype=U64)
    return mix64(k1 ^ mix64(k0 ^ U64(seed)))
