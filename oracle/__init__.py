"""CPU oracle for Progressive Material Caching (Fujieda & Harada 2022).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 restatement of
what the method computes, written from the paper's text: material networks
evaluated in the standard way (Sec. 2), cacheable nodes and their descriptors
(Sec. 3 and 3.1, Eq. 1), the two-hash fixed-size table and its update
(Sec. 3.2, 3.3, Algorithm 1).  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import it.  It shares no code, header,
constant table or helper with the HIP library, and never calls it.

Modules
  hashing  64-bit finalizer and the lattice / descriptor hashes
  codec    32-bit value encodings (raw float, RGB9E5)
  nodes    node definitions (FP64)
  graph    dependency classes, cacheable marking, memoised evaluation
  keys     descriptor pipeline: Eq. 1 level, virtual texel, cell and Hash2
  table    the fixed-size table: lookup and Algorithm 1 insert
  render   uncached evaluation and the snapshot-mode progressive frames
  check    invariants a nondeterministic (lock-free) run must satisfy
  mlp      reference forward/backward of the per-material surrogate
"""
