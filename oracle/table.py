"""The fixed-size two-hash table and its update (Sec. 3.2, Sec. 3.3, Algorithm 1).

Layout: N_c cells of N_e entries (Fig. 4 shows a 10 x 5 table); entry index
= cell * N_e + i.  Each entry holds one 64-bit word = hash2 << 32 | encoded
value (Sec. 3.3 packs the second hash with the 32-bit encoded value); a word
of 0 is an empty entry.  16-byte entries add a 32-bit stamp (frame + 1 of the
write) and a 32-bit reserved field that stays 0.

Readings:
  * the entry loop runs i = 0 .. N_e - 1 (the loop bound is exclusive; an
    inclusive bound would step into the next cell);
  * the condition is a logical OR: first entry whose hash equals hash2 or is 0;
  * lookup (which the paper does not list) is the same scan: a hit on the
    first entry whose hash equals hash2, a miss at the first empty entry or
    after N_e entries;
  * a failed compare-and-swap is not retried (the algorithm discards ``old``);
  * FIRST keeps the first inserted value (Sec. 3.2); OVERWRITE (beyond the
    paper, after its future-work remark in Sec. 5) replaces, when the scan
    finds neither the key nor an empty entry, the entry with the smallest
    stamp (lowest index on ties) if that stamp predates the current frame.
Everything here is sequential pure Python: the obviously-correct model.
"""
import numpy as np

FIRST, OVERWRITE = "FIRST", "OVERWRITE"


class Table:
    def __init__(self, n_cells: int, n_entries: int, entry_bytes: int = 16):
        if entry_bytes not in (8, 16):
            raise ValueError("entry_bytes must be 8 or 16")
        self.n_cells, self.n_entries, self.entry_bytes = int(n_cells), int(n_entries), entry_bytes
        size = self.n_cells * self.n_entries
        self.word = [0] * size
        self.stamp = [0] * size

    # --- raw views ---------------------------------------------------------
    def words(self) -> np.ndarray:
        return np.array(self.word, dtype=np.uint64)

    def stamps(self) -> np.ndarray:
        return np.array(self.stamp, dtype=np.uint32)

    def nbytes(self) -> int:
        return self.n_cells * self.n_entries * self.entry_bytes

    def copy(self) -> "Table":
        t = Table(self.n_cells, self.n_entries, self.entry_bytes)
        t.word = list(self.word)
        t.stamp = list(self.stamp)
        return t

    # --- lookup -------------------------------------------------------------
    def lookup(self, cell: int, hash2: int):
        """Returns (found, encoded value)."""
        base = cell * self.n_entries
        for i in range(self.n_entries):
            w = self.word[base + i]
            if (w >> 32) == hash2:
                return True, w & 0xFFFFFFFF
            if w == 0:
                return False, 0
        return False, 0

    # --- Algorithm 1 --------------------------------------------------------
    def cas(self, idx: int, expected: int, new: int) -> int:
        old = self.word[idx]
        if old == expected:
            self.word[idx] = new
        return old

    def insert(self, cell: int, hash2: int, enc: int, policy: str = FIRST, frame: int = 0) -> str:
        """Returns one of 'inserted', 'present', 'full', 'overwritten', 'cas_failed'."""
        base = cell * self.n_entries
        hash_idx = -1
        for i in range(self.n_entries):
            cur = self.word[base + i]
            if (cur >> 32) == hash2 or (cur >> 32) == 0:
                hash_idx = base + i
                break
        new = (hash2 << 32) | (enc & 0xFFFFFFFF)
        if hash_idx != -1:
            old = self.cas(hash_idx, 0, new)
            if old == 0:
                self.stamp[hash_idx] = frame + 1 if self.entry_bytes == 16 else 0
                return "inserted"
            return "present" if (old >> 32) == hash2 else "cas_failed"
        if policy == OVERWRITE:
            if self.entry_bytes != 16:
                raise ValueError("OVERWRITE needs 16-byte entries (stamps)")
            victim = min(range(self.n_entries), key=lambda i: (self.stamp[base + i], i))
            if self.stamp[base + victim] < frame + 1:
                observed = self.word[base + victim]
                if self.cas(base + victim, observed, new) == observed:
                    self.stamp[base + victim] = frame + 1
                    return "overwritten"
        return "full"

    # --- properties ---------------------------------------------------------
    def occupancy(self) -> int:
        return sum(1 for w in self.word if w != 0)
