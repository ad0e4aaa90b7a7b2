"""The fixed-size two-hash table and its update (Sec. 3.2, Sec. 3.3, Algorithm 1).

Layout: N_c cells of N_e entries (the paper's two-hash figure shows a 10 x 5
table); entry index = cell * N_e + i.  Each entry holds one 64-bit word =
hash2 << 32 | encoded value (Sec. 3.3 packs the second hash with the 32-bit
encoded value); a word of 0 is an empty entry.  16-byte entries add a 32-bit
stamp (frame + 1 of the write) and a 32-bit aux field: 0, except under the
PRIORITY policy, where it holds the bounce count of the sample that wrote
the entry.

What the paper fixes: the hash picks a cell, the second hash verifies the
key; a cell is searched entry by entry; a value is stored only in an empty
entry, with one compare-and-swap of the whole word, so the first value
stored for a key stays (Sec. 3.2 "keep the first", Sec. 3.3); when a cell has
no room the value is simply not stored.

Readings:
  * entries i = 0 .. N_e - 1 of the cell are searched (an inclusive bound
    would step into the next cell); the search stops at the first entry that
    holds hash2 or is empty (the paper's condition is a logical OR);
  * lookup (which the paper does not list) is the same search: hash2 found
    is a hit, an empty entry or the end of the cell a miss;
  * a failed compare-and-swap is not retried (the algorithm discards the old
    word); in this sequential model the swap fails exactly when the entry
    the search returned already holds the key;
  * FIRST keeps the first inserted value; OVERWRITE (beyond the paper, after
    its future-work remark in Sec. 5) replaces, when the search finds neither
    the key nor an empty entry, the entry with the smallest stamp (lowest
    index on ties) if that stamp predates the current frame;
  * PRIORITY (also beyond the paper: Sec. 5 suggests preferring directly
    visible samples when storage is limited): as OVERWRITE, but the victim is
    the entry with the largest bounce count, then the smallest stamp, then
    the lowest index; it is replaced when its bounce count is larger than the
    new sample's, or equal and its stamp predates the current frame.  A
    sample never displaces one of a smaller bounce count.

False hits (Sec. 3.2 notes that collisions of the verification hash cannot
be avoided): next to every entry the model keeps the full descriptor of the
sample that wrote it (a shadow map the device table does not have), so a
lookup that matches hash2 but not the descriptor is counted as a false hit.

Everything here is sequential pure Python: the obviously-correct model.
"""
import numpy as np

FIRST, OVERWRITE, PRIORITY = "FIRST", "OVERWRITE", "PRIORITY"


class Table:
    def __init__(self, n_cells: int, n_entries: int, entry_bytes: int = 16):
        if entry_bytes not in (8, 16):
            raise ValueError("entry_bytes must be 8 or 16")
        self.n_cells, self.n_entries, self.entry_bytes = int(n_cells), int(n_entries), entry_bytes
        size = self.n_cells * self.n_entries
        self.word = [0] * size
        self.stamp = [0] * size
        self.aux = [0] * size
        self.key = [None] * size          # shadow map: full descriptor of the writer
        self.false_hits = 0

    # --- raw views ---------------------------------------------------------
    def words(self) -> np.ndarray:
        return np.array(self.word, dtype=np.uint64)

    def stamps(self) -> np.ndarray:
        return np.array(self.stamp, dtype=np.uint32)

    def auxes(self) -> np.ndarray:
        return np.array(self.aux, dtype=np.uint32)

    def nbytes(self) -> int:
        return self.n_cells * self.n_entries * self.entry_bytes

    def copy(self) -> "Table":
        t = Table(self.n_cells, self.n_entries, self.entry_bytes)
        t.word, t.stamp, t.aux, t.key = list(self.word), list(self.stamp), list(self.aux), \
            list(self.key)
        t.false_hits = self.false_hits
        return t

    # --- the search shared by lookup and insert ----------------------------
    def _search(self, cell: int, hash2: int):
        """Entry index of the first entry of the cell whose hash is hash2 or that
        is empty, with True when it holds hash2; (None, False) when every entry
        holds another hash."""
        first = cell * self.n_entries
        for idx in range(first, first + self.n_entries):
            h = self.word[idx] >> 32
            if h == hash2:
                return idx, True
            if self.word[idx] == 0:
                return idx, False
        return None, False

    # --- lookup -------------------------------------------------------------
    def lookup(self, cell: int, hash2: int, key=None):
        """Returns (found, encoded value).  With the probing sample's full
        descriptor ``key``, a hit on an entry written for another descriptor is
        counted in ``false_hits``."""
        idx, holds = self._search(cell, hash2)
        if not holds:
            return False, 0
        if key is not None and self.key[idx] is not None and self.key[idx] != key:
            self.false_hits += 1
        return True, self.word[idx] & 0xFFFFFFFF

    def is_false_hit(self, cell: int, hash2: int, key) -> bool:
        idx, holds = self._search(cell, hash2)
        return bool(holds and self.key[idx] is not None and self.key[idx] != key)

    # --- update --------------------------------------------------------------
    def _store(self, idx, new, frame, key, bounce):
        self.word[idx] = new
        self.stamp[idx] = frame + 1 if self.entry_bytes == 16 else 0
        self.aux[idx] = bounce if self.entry_bytes == 16 else 0
        self.key[idx] = key

    def _victim(self, cell: int, policy: str):
        """Entry a full cell gives up: oldest stamp (OVERWRITE), or largest bounce
        count, then oldest stamp (PRIORITY); lowest index on ties."""
        first = cell * self.n_entries
        idxs = range(first, first + self.n_entries)
        if policy == PRIORITY:
            return min(idxs, key=lambda i: (-self.aux[i], self.stamp[i], i))
        return min(idxs, key=lambda i: (self.stamp[i], i))

    def insert(self, cell: int, hash2: int, enc: int, policy: str = FIRST, frame: int = 0,
               key=None, bounce: int = 0) -> str:
        """Store hash2 << 32 | enc in the cell.  Returns one of 'inserted',
        'present', 'full', 'overwritten' (a sequential model has no failed
        compare-and-swap).  ``key`` is the full descriptor for the shadow map;
        ``bounce`` the sample's bounce count (stored under PRIORITY)."""
        new = (hash2 << 32) | (enc & 0xFFFFFFFF)
        if policy == PRIORITY:
            bounce = int(bounce)
        else:
            bounce = 0
        idx, holds = self._search(cell, hash2)
        if idx is not None:
            # the compare-and-swap from the empty word: it succeeds iff the
            # entry is still empty, i.e. did not already hold the key
            if holds:
                return "present"
            self._store(idx, new, frame, key, bounce)
            return "inserted"
        if policy in (OVERWRITE, PRIORITY):
            if self.entry_bytes != 16:
                raise ValueError("OVERWRITE and PRIORITY need 16-byte entries (stamps)")
            v = self._victim(cell, policy)
            older = self.stamp[v] < frame + 1
            if policy == PRIORITY:
                ok = self.aux[v] > bounce or (self.aux[v] == bounce and older)
            else:
                ok = older
            if ok:
                self._store(v, new, frame, key, bounce)
                return "overwritten"
        return "full"

    # --- properties ---------------------------------------------------------
    def occupancy(self) -> int:
        return sum(1 for w in self.word if w != 0)
