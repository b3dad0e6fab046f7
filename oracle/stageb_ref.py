"""Reference of stage B, whole-read mapping with at most one edit (test
infrastructure only: imported by tests, never by the product path).

Stage B of the paper (Sec. 2, "Stage B: BWT") maps each whole read onto the
reference allowing at most one error, insertion or deletion (EID) and writes
an alignment record (first and last reference base, strand) for each mapping;
reads it cannot map go on to the seeders.  The paper searches its BWT; here
the candidate places come from the exact seed regions of seeker_ref (the
same index, seeds and repeat cut-off), and each candidate is verified base by
base.  This module is the plain definition:

Candidates.  Of the read's regions (seeker_ref.regions order) the first
MAX_REGIONS count.  For each strand, every region's diagonal d = first - read
position (the read's first base on the reference if the region lies on an
error-free stretch) gives the candidate starts d - 1, d and d + 1 (an indel
before the region shifts its diagonal by one).

Verification of the query q (the read, or its reverse complement on strand 1;
m bases) at start p, in this order of preference:
  exact          q == ref[p : p + m]
  substitution   q differs from ref[p : p + m] at exactly one base j
  deletion       the reference holds one base the read lacks: for the
                 smallest i in [1, m - 1], q[:i] == ref[p : p + i] and
                 q[i:] == ref[p + i + 1 : p + m + 1]
  insertion      the read holds one base the reference lacks: for the
                 smallest i in [1, m - 2], q[:i] == ref[p : p + i] and
                 q[i + 1:] == ref[p + i : p + m - 1]
A variant whose reference span leaves [0, L) does not apply.  (Indels at the
read's first or last base are left out: they are the same as a shorter or
longer exact match.)

Records.  The read maps when some candidate verifies; only the candidates
with the fewest edits are reported (an exact match hides one-edit matches
elsewhere), sorted by (strand, start), at most MAX_RECORDS of them, as
(strand, first, last, edits, op, edit position) with op 0 exact, 1
substitution, 2 deletion, 3 insertion, and edit position j (substitution) or
i (indels) in query coordinates (-1 for exact).
"""
from __future__ import annotations

import numpy as np

from . import seeker_ref as sr

MAX_RECORDS = 16
MAX_REGIONS = sr.MAX_REGIONS
EXACT, SUBST, DEL, INS = 0, 1, 2, 3


def verify(q: np.ndarray, ref: np.ndarray, p: int):
    """(edits, op, position, last reference base) of q at start p, or None."""
    m, L = len(q), len(ref)
    if p < 0:
        return None
    if p + m <= L:
        mm = np.nonzero(q != ref[p:p + m])[0]
        if len(mm) == 0:
            return (0, EXACT, -1, p + m - 1)
        if len(mm) == 1:
            return (1, SUBST, int(mm[0]), p + m - 1)
    if p + m + 1 <= L:
        for i in range(1, m):
            if (q[:i] == ref[p:p + i]).all() and (q[i:] == ref[p + i + 1:p + m + 1]).all():
                return (1, DEL, i, p + m)
    if p + m - 1 <= L:
        for i in range(1, m - 1):
            if (q[:i] == ref[p:p + i]).all() and (q[i + 1:] == ref[p + i:p + m - 1]).all():
                return (1, INS, i, p + m - 2)
    return None


def map_read(read_codes, ref: np.ndarray, index: dict, k: int = sr.K, step: int = sr.STEP,
             offset: int = sr.OFFSET, max_occ: int = sr.MAX_OCC,
             max_records: int = MAX_RECORDS) -> list[tuple]:
    """Records of one read: [(strand, first, last, edits, op, position)], empty if
    stage B does not map it."""
    q0 = np.asarray(read_codes, dtype=np.uint8)
    regs = sr.regions(q0, index, k, step, offset, max_occ)[:MAX_REGIONS]
    ref = np.asarray(ref, dtype=np.uint8)
    recs = []
    for strand in (0, 1):
        q = q0 if strand == 0 else sr.revcomp(q0)
        diags = {f - rp for (s, f, _, rp) in regs if s == strand}
        for p in sorted({d + t for d in diags for t in (-1, 0, 1)}):
            v = verify(q, ref, p)
            if v is not None:
                recs.append((strand, p, v[3], v[0], v[1], v[2]))
    if not recs:
        return []
    e = min(r[3] for r in recs)
    return [r for r in recs if r[3] == e][:max_records]
