"""Oracle depth digests for the full-size parity tests.

The digest files (tests/golden/depth_digests_*.txt) are written by
tests/golden/make_digests.py, which calls only the CPU oracle and the seeded
input generators. Each line holds a source, the size and edge count of its
component, its largest depth and the SHA-256 of the oracle's depth row as n
int32 values, little-endian. A GPU row hashed the same way is bit-identical to
the oracle's row iff the digests are equal.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def row_digest(depth: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(depth, dtype="<i4").data).hexdigest()


def load(name: str) -> dict:
    """{source: record} for an RMAT file, {(graph, source): record} for the
    served mix; record = dict(reached, edges_cc, max_depth, sha256, index)."""
    out = {}
    with open(os.path.join(GOLD, f"depth_digests_{name}.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, s, reached, ecc, maxd, h = line.split()
            rec = {"reached": int(reached), "edges_cc": int(ecc), "max_depth": int(maxd),
                   "sha256": h}
            if name == "served":
                out[(int(a), int(s))] = rec
            else:
                rec["index"] = int(a)
                out[int(s)] = rec
    return out


def sources_of(name: str) -> list:
    """Sources of an RMAT digest file, in file order."""
    recs = load(name)
    return [s for s, _ in sorted(recs.items(), key=lambda kv: kv[1]["index"])]


def threads() -> int:
    """Hashing threads: the host's cores, at most 16 (the GPU machine's share)."""
    return max(1, min(16, os.cpu_count() or 1))


class RowChecker:
    """Hashes host rows on a thread pool and compares them with the digests.

    submit() takes a host numpy row (owned by the checker from then on); at
    most `pending` rows wait at once, so host memory stays bounded.
    mismatches() waits for every row and returns [(key, got, want)]."""

    def __init__(self, expected: dict, pending: int = 16):
        self.expected = expected
        self.pool = cf.ThreadPoolExecutor(max_workers=threads())
        self.futs = []
        self.pending = pending
        self.bad = []
        self.checked = 0

    def _drain(self, keep: int):
        while len(self.futs) > keep:
            key, f = self.futs.pop(0)
            got = f.result()
            want = self.expected[key]["sha256"]
            self.checked += 1
            if got != want:
                self.bad.append((key, got, want))

    def submit(self, key, row: np.ndarray):
        self.futs.append((key, self.pool.submit(row_digest, row)))
        self._drain(self.pending)

    def mismatches(self):
        self._drain(0)
        self.pool.shutdown()
        return self.bad


def first_difference(got: np.ndarray, want: np.ndarray) -> str:
    diff = np.nonzero(got != want)[0]
    if len(diff) == 0:
        return "rows equal (digest of a different row?)"
    v = int(diff[0])
    return (f"{len(diff)} vertices differ; first at vertex {v}: gpu {int(got[v])}, "
            f"oracle {int(want[v])}")
