"""Exhaustive checker for local alignment on tiny inputs (test infrastructure).

It does not use the dynamic-programming recurrences at all.  It enumerates
every local alignment of the read q against the window r as an explicit path
and scores the path by summation, so it pins the oracle independently.

A path starts with an aligned pair (M) at some cell and continues with
  M      consume q_i and r_j, score s(q_i, r_j)
  D      consume r_j only (a deletion from the read)
  I      consume q_i only (an insertion in the read)
Every gap op is tagged "open" (scores gap_open; allowed after any op) or
"extend" (scores gap_extend; only directly after a gap op of the same kind),
which is the three-state automaton behind Gotoh's affine-gap model.  A path is
a complete alignment whenever its last op is M.

Selection rules checked against the oracle:
  score S  = max(0, best path score)
  end cell = among optimal paths, smallest window end j, then smallest read end i
  path     = among optimal paths ending there, the one whose backward decision
             string is lexicographically smallest, where walking back from the
             end the decisions are:
               at an aligned point: stop (path starts here) < M < D < I
               inside a gap run:    this gap op is an open < it is an extend
"""
from __future__ import annotations

M, I, D = 0, 1, 2


def _s(a, b, sc):
    return sc[0] if a == b else sc[1]


def enumerate_paths(q, r, sc, floor=None):
    """Yield (score, start_i, start_j, end_i, end_j, ops) for every local path.

    Coordinates are 1-based cells of the last consumed bases; ops is a tuple of
    (op, is_open) in forward order.

    Two exact prunings keep this usable beyond 5x5 inputs; neither can drop a
    path that ties the optimum:
      * a gap may re-open directly after a gap of the same kind only when
        gap_open == gap_extend; otherwise extending gives the same ops with a
        strictly higher score;
      * with `floor` (a list holding the best score seen so far), a path whose
        score plus the most it could still gain (match * remaining diagonal)
        is below floor[0] is abandoned.
    """
    m, n = len(q), len(r)
    ma, go, ge = sc[0], sc[2], sc[3]
    reopen = go == ge
    for i0 in range(1, m + 1):
        for j0 in range(1, n + 1):
            first = ((M, False),)
            stack = [(i0, j0, _s(q[i0 - 1], r[j0 - 1], sc), first)]
            while stack:
                i, j, score, ops = stack.pop()
                if floor is not None and score + ma * min(m - i, n - j) < floor[0]:
                    continue
                last = ops[-1][0]
                if last == M:
                    if floor is not None and score > floor[0]:
                        floor[0] = score
                    yield score, i0, j0, i, j, ops
                if i < m and j < n:
                    stack.append((i + 1, j + 1, score + _s(q[i], r[j], sc), ops + ((M, False),)))
                if j < n:
                    if last != D or reopen:
                        stack.append((i, j + 1, score + go, ops + ((D, True),)))
                    if last == D:
                        stack.append((i, j + 1, score + ge, ops + ((D, False),)))
                if i < m:
                    if last != I or reopen:
                        stack.append((i + 1, j, score + go, ops + ((I, True),)))
                    if last == I:
                        stack.append((i + 1, j, score + ge, ops + ((I, False),)))


def _decisions(ops):
    """Backward decision string of a path (see module docstring)."""
    out = []
    k = len(ops) - 1
    while True:
        if k < 0:
            out.append(0)            # stop
            return tuple(out)
        op, is_open = ops[k]
        if op == M:
            out.append(1)
            k -= 1
            continue
        out.append(2 if op == D else 3)
        # inside the gap run
        while True:
            op_k, open_k = ops[k]
            k -= 1
            if open_k:
                out.append(0)
                break
            out.append(1)


def brute_align(q, r, sc):
    """Returns dict(score, read_begin, read_end, ref_begin, ref_end, ops) with
    0-based inclusive coordinates (-1 when score is 0) and forward op list."""
    best = 0
    cands = []
    floor = [1]
    for score, i0, j0, i, j, ops in enumerate_paths(q, r, sc, floor):
        if score > best:
            best = score
            cands = [(i0, j0, i, j, ops)]
        elif score == best and score > 0:
            cands.append((i0, j0, i, j, ops))
    if best == 0:
        return dict(score=0, read_begin=-1, read_end=-1, ref_begin=-1, ref_end=-1, ops=())
    ej = min(c[3] for c in cands)
    ei = min(c[2] for c in cands if c[3] == ej)
    at_end = [c for c in cands if c[2] == ei and c[3] == ej]
    pick = min(at_end, key=lambda c: _decisions(c[4]))
    i0, j0, i, j, ops = pick
    return dict(score=best, read_begin=i0 - 1, read_end=i - 1, ref_begin=j0 - 1,
                ref_end=j - 1, ops=tuple(o for o, _ in ops))


def cigar_of(ops, read_begin, read_end, m):
    """Run-length CIGAR text with soft clips, e.g. '2S4M1D3M'."""
    names = "MID"
    parts = []
    if read_begin > 0:
        parts.append(f"{read_begin}S")
    k = 0
    while k < len(ops):
        j = k
        while j < len(ops) and ops[j] == ops[k]:
            j += 1
        parts.append(f"{j - k}{names[ops[k]]}")
        k = j
    if m - 1 - read_end > 0 and len(ops):
        parts.append(f"{m - 1 - read_end}S")
    return "".join(parts)


def rescore(ops, q, r, read_begin, ref_begin, sc):
    """Score of an op list placed at (read_begin, ref_begin), gap runs scored
    gap_open + (k-1)*gap_extend."""
    i, j = read_begin, ref_begin
    total = 0
    prev = None
    for op in ops:
        if op == M:
            total += _s(q[i], r[j], sc)
            i += 1
            j += 1
        elif op == D:
            total += sc[3] if prev == D else sc[2]
            j += 1
        else:
            total += sc[3] if prev == I else sc[2]
            i += 1
        prev = op
    return total
