"""Reference of the learned filter's per-read decision and of the compaction
(test infrastructure only: imported by tests, never by the product path).

The paper's stage D keeps a merged seed region as a candidate location only
when enough seed evidence supports it, and stage E aligns every candidate that
survives (Sec. 2, "Stage D: CAL Seeker" and "Stage E", task iii).  The learned
filter replaces stage D's rule by a score per candidate (a logit z) and this
decision, written here directly from its definition, read by read:

  * a read id at or beyond the number of reads: the pair is never kept;
  * a read whose pairs do not form one contiguous run of the pair list, or
    that has more than 64 candidates: every candidate is kept, and the read
    counts as unsure;
  * otherwise, with mx the largest logit of the read:
      - mx < drop: no candidate is kept (the read is reported unmapped);
      - the read is unsure when mx < hi or some logit lies in [lo, hi):
        every candidate is kept;
      - else the candidates with z >= hi are kept.

The compaction lists the kept pairs in their original order (a stable
selection) with their windows.
"""
from __future__ import annotations

import numpy as np

MAX_CAND = 64


def decide(z, read_id, n_reads: int, lo: float, hi: float, drop: float = float("-inf"),
           max_cand: int = MAX_CAND):
    """Keep flag per pair (bool array) and the number of unsure reads.

    z: logits per pair (float32); read_id: read of each pair."""
    z = np.asarray(z, dtype=np.float32)
    rid = np.asarray(read_id, dtype=np.int64)
    keep = np.zeros(len(rid), dtype=bool)
    n_unsure = 0
    order = np.argsort(rid, kind="stable")
    bounds = np.searchsorted(rid[order], np.arange(n_reads + 1))
    lo32, hi32, drop32 = np.float32(lo), np.float32(hi), np.float32(drop)
    for r in range(n_reads):
        idx = order[bounds[r]:bounds[r + 1]]          # this read's pairs, ascending
        if len(idx) == 0:
            continue
        contiguous = int(idx[-1]) - int(idx[0]) + 1 == len(idx)
        if not contiguous or len(idx) > max_cand:
            keep[idx] = True
            n_unsure += 1
            continue
        zr = z[idx]
        mx = zr.max()
        if mx < drop32:
            continue
        if mx < hi32 or bool(((zr >= lo32) & (zr < hi32)).any()):
            keep[idx] = True
            n_unsure += 1
        else:
            keep[idx] = zr >= hi32
    return keep, n_unsure


def compact(keep, windows):
    """(kept pair ids in original order, their windows)."""
    ids = np.nonzero(np.asarray(keep, dtype=bool))[0].astype(np.uint32)
    return ids, np.asarray(windows)[ids]
