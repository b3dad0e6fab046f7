"""Pins of the stage B reference (oracle/stageb_ref.py): verification against
brute-force enumeration of every single edit on small random inputs, the
preference order and leftmost placement on hand-built cases, and whole-read
mapping of planted reads (exact, one substitution, one indel, two edits,
reverse strand, best stratum, repeat cut-off)."""
import numpy as np

from oracle import seeker_ref as sr
from oracle import stageb_ref as sb


def _edits_of(span, q):
    """Brute force: the ways q arises from span by one substitution, one
    deletion (a base of span dropped) or one insertion (a base added)."""
    subs = [j for j in range(len(span)) if len(q) == len(span) and
            np.sum(q != span) == 1 and q[j] != span[j]]
    dels = [i for i in range(len(span)) if len(q) == len(span) - 1 and
            (np.concatenate([span[:i], span[i + 1:]]) == q).all()]
    ins = [i for i in range(len(q)) if len(q) == len(span) + 1 and
           (np.concatenate([q[:i], q[i + 1:]]) == span).all()]
    return subs, dels, ins


def test_verify_against_brute_force():
    g = np.random.default_rng(5)
    seen = {sb.EXACT: 0, sb.SUBST: 0, sb.DEL: 0, sb.INS: 0, None: 0}
    for t in range(3000):
        L = int(g.integers(10, 30))
        ref = g.integers(0, 2 if t % 3 == 0 else 4, L).astype(np.uint8)
        m = int(g.integers(3, 9))
        p = int(g.integers(-1, L - m + 2))
        base = ref[max(p, 0):max(p, 0) + m].copy()
        if len(base) < m:
            base = np.concatenate([base, g.integers(0, 4, m - len(base)).astype(np.uint8)])
        u = g.random()
        q = base.copy()
        if u < 0.25:
            j = int(g.integers(0, m))
            q[j] = (q[j] + 1) % 4
        elif u < 0.45:
            q = np.delete(q, int(g.integers(0, m)))
            q = np.concatenate([q, ref[max(p, 0) + m:max(p, 0) + m + 1]])[:m]
        elif u < 0.65:
            q = np.insert(q, int(g.integers(0, m)), int(g.integers(0, 4)))[:m]
        elif u < 0.8:
            q = g.integers(0, 4, m).astype(np.uint8)
        if len(q) < m:
            q = np.concatenate([q, g.integers(0, 4, m - len(q)).astype(np.uint8)])
        v = sb.verify(q, ref, p)
        seen[None if v is None else v[1]] += 1
        if p < 0:
            assert v is None
            continue
        spans = {0: ref[p:p + m] if p + m <= L else None,
                 1: ref[p:p + m + 1] if p + m + 1 <= L else None,
                 -1: ref[p:p + m - 1] if p + m - 1 <= L else None}
        exact = spans[0] is not None and (spans[0] == q).all()
        subs = _edits_of(spans[0], q)[0] if spans[0] is not None else []
        dels = [i for i in _edits_of(spans[1], q)[1] if 1 <= i <= m - 1] \
            if spans[1] is not None else []
        ins = [i for i in _edits_of(spans[-1], q)[2] if 1 <= i <= m - 2] \
            if spans[-1] is not None else []
        if exact:
            assert v == (0, sb.EXACT, -1, p + m - 1)
        elif subs:
            assert v == (1, sb.SUBST, subs[0], p + m - 1)
        elif dels:
            assert v == (1, sb.DEL, min(dels), p + m)
        elif ins:
            assert v == (1, sb.INS, min(ins), p + m - 2)
        else:
            assert v is None
    assert min(seen.values()) > 100, seen


def test_verify_hand_cases():
    A, C, G, T = 0, 1, 2, 3
    ref = np.array([C, A, A, A, A, G, T, C], np.uint8)
    # deletion inside a homopolymer: leftmost placement (after the first A)
    q = np.array([C, A, A, A, G, T], np.uint8)
    assert sb.verify(q, ref, 0) == (1, sb.DEL, 1, 6)
    # insertion inside a homopolymer: leftmost placement
    q = np.array([C, A, A, A, A, A, G], np.uint8)
    assert sb.verify(q, ref, 0) == (1, sb.INS, 1, 5)
    # a substitution is preferred to an indel with the same start
    q = np.array([C, A, A, A, A, G, A], np.uint8)
    assert sb.verify(q, ref, 0) == (1, sb.SUBST, 6, 6)
    # an indel at either end is not counted
    assert sb.verify(np.array([A, A, A, A, G], np.uint8), ref, 0) is None
    assert sb.verify(np.array([C, A, A, A, A, G, T, C], np.uint8), ref, 1) is None
    # past the reference end
    assert sb.verify(np.array([T, C, A], np.uint8), ref, 6) is None


def test_map_planted_reads():
    g = np.random.default_rng(6)
    ref = g.integers(0, 4, 200_000).astype(np.uint8)
    idx = sr.build_index_fast(ref)
    p, m = 50_000, 100
    q = ref[p:p + m].copy()
    assert sb.map_read(q, ref, idx) == [(0, p, p + m - 1, 0, sb.EXACT, -1)]
    q1 = q.copy()
    q1[37] = (q1[37] + 2) % 4
    assert sb.map_read(q1, ref, idx) == [(0, p, p + m - 1, 1, sb.SUBST, 37)]
    q2 = np.delete(ref[p:p + m + 1], 60)                 # one reference base missing
    r2 = sb.map_read(q2, ref, idx)
    assert len(r2) == 1 and r2[0][:2] == (0, p) and r2[0][3:5] == (1, sb.DEL)
    q3 = np.insert(ref[p:p + m - 1], 5, 2)               # an extra read base near the start
    r3 = sb.map_read(q3, ref, idx)
    assert len(r3) == 1 and r3[0][:2] == (0, p) and r3[0][3:5] == (1, sb.INS)
    q4 = q1.copy()
    q4[80] = (q4[80] + 1) % 4                            # two edits: stage B does not map it
    assert sb.map_read(q4, ref, idx) == []
    rc = sr.revcomp(q1)                                  # the reverse strand
    assert sb.map_read(rc, ref, idx) == [(1, p, p + m - 1, 1, sb.SUBST, 37)]


def test_best_stratum_and_repeats():
    g = np.random.default_rng(7)
    ref = g.integers(0, 4, 100_000).astype(np.uint8)
    seg = ref[10_000:10_100].copy()
    ref[60_000:60_100] = seg
    ref[60_050] = (ref[60_050] + 1) % 4                  # a copy one substitution away
    idx = sr.build_index_fast(ref)
    assert sb.map_read(seg, ref, idx) == [(0, 10_000, 10_099, 0, sb.EXACT, -1)]
    seg2 = seg.copy()
    seg2[50] = (seg2[50] + 2) % 4                        # now both copies are one edit away
    r = sb.map_read(seg2, ref, idx)
    assert [x[:2] for x in r] == [(0, 10_000), (0, 60_000)] and all(x[3] == 1 for x in r)
    # a read all of whose seeds repeat beyond max_occ gets no candidates
    for c in range(6):
        ref[70_000 + 200 * c:70_000 + 200 * c + 100] = seg
    idx = sr.build_index_fast(ref)
    assert sb.map_read(seg, ref, idx, max_occ=5) == []
    assert len(sb.map_read(seg, ref, idx, max_occ=64)) == 7
