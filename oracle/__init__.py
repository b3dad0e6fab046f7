"""CPU oracle for the batched Smith-Waterman hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the GPU path (see ``gotoh.c`` for the definition it implements, and
``brute.py`` for the exhaustive checker it is pinned against).

Contents
--------
* ``gotoh.c``   plain C full-matrix Gotoh local alignment + canonical traceback,
                and a two-row score/end variant (pthreads over pairs).
* ``brute.py``  enumeration of every local alignment on tiny inputs.
* ``mlp_ref.py`` float64/float32 reference of the candidate-filter MLP.
* ``features_ref.py`` reference of the per-candidate seed-hit features.
* ``filter_ref.py`` reference of the filter's per-read decision and compaction.

Parity status: the score, end cell, begin cell and CIGAR are pinned by brute
force, closed forms, hand-worked examples and invariants (tests/test_oracle_*);
the features by brute-force hit enumeration and hand-computed planted hits;
the MLP by float64 finite differences, Adam by hand-computed steps and a
closed form; the filter decision by hand-built cases.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

RESULT_DTYPE = np.dtype([("score", "<i4"), ("read_begin", "<i4"), ("read_end", "<i4"),
                         ("ref_begin", "<i4"), ("ref_end", "<i4"), ("n_ops", "<u4"),
                         ("status", "<u4")])
OPS = {0: "M", 1: "I", 2: "D", 3: "N", 4: "S"}
DEFAULT_SCORING = (5, -4, -10, -1)


class _Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


def build(force: bool = True) -> str:
    """Compile gotoh.c into liboracle.so (portable x86-64, no SIMD tuning)."""
    src = os.path.join(HERE, "gotoh.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-std=c11", "-Wall",
                               "-shared", "-fPIC", "-pthread", src, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_batch.argtypes = [P, ctypes.c_uint64, P, P, P, ctypes.c_uint32, P, P,
                                ctypes.c_uint32, ctypes.POINTER(_Scoring), ctypes.c_int, P, P,
                                ctypes.c_uint32, ctypes.c_int]
        L.orc_batch.restype = ctypes.c_int
        for name in ("orc_align_codes",):
            f = getattr(L, name)
            f.argtypes = [P, ctypes.c_int, P, ctypes.c_int, ctypes.POINTER(_Scoring), P, P,
                          ctypes.c_uint32]
            f.restype = ctypes.c_int
        L.orc_score_codes.argtypes = [P, ctypes.c_int, P, ctypes.c_int,
                                      ctypes.POINTER(_Scoring), P]
        L.orc_matrices.argtypes = [P, ctypes.c_int, P, ctypes.c_int, ctypes.POINTER(_Scoring),
                                   P, P, P]
        _lib = L
    return _lib


def _sc(scoring):
    return _Scoring(*[int(x) for x in scoring])


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def align_codes(q, r, scoring=DEFAULT_SCORING, ops_cap=None):
    """Full alignment of code sequences q (read) and r (window)."""
    q = np.ascontiguousarray(q, dtype=np.uint8)
    r = np.ascontiguousarray(r, dtype=np.uint8)
    cap = ops_cap if ops_cap is not None else len(q) + len(r) + 4
    ops = np.zeros(max(cap, 1), dtype=np.uint32)
    res = np.zeros(1, dtype=RESULT_DTYPE)
    lib().orc_align_codes(_ptr(q), len(q), _ptr(r), len(r), ctypes.byref(_sc(scoring)),
                          _ptr(res), _ptr(ops), cap)
    return res[0], ops[:int(res[0]["n_ops"])].copy()


def score_codes(q, r, scoring=DEFAULT_SCORING):
    q = np.ascontiguousarray(q, dtype=np.uint8)
    r = np.ascontiguousarray(r, dtype=np.uint8)
    res = np.zeros(1, dtype=RESULT_DTYPE)
    lib().orc_score_codes(_ptr(q), len(q), _ptr(r), len(r), ctypes.byref(_sc(scoring)), _ptr(res))
    return res[0]


def matrices(q, r, scoring=DEFAULT_SCORING):
    q = np.ascontiguousarray(q, dtype=np.uint8)
    r = np.ascontiguousarray(r, dtype=np.uint8)
    sh = (len(q) + 1, len(r) + 1)
    H = np.zeros(sh, np.int32)
    E = np.zeros(sh, np.int32)
    F = np.zeros(sh, np.int32)
    lib().orc_matrices(_ptr(q), len(q), _ptr(r), len(r), ctypes.byref(_sc(scoring)),
                       _ptr(H), _ptr(E), _ptr(F))
    return H, E, F


def align_batch(batch, scoring=DEFAULT_SCORING, mode=0, sel=None, ops_stride=None,
                nthreads=None):
    """Run the oracle on a synth.Batch (all pairs, or the pair indices in `sel`).

    mode 0: score + end coordinates.  mode 1: full alignment with CIGAR ops.
    Returns (results[RESULT_DTYPE], ops[n, ops_stride] or None).
    """
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    win = np.ascontiguousarray(batch.windows)
    seln = None if sel is None else np.ascontiguousarray(sel, dtype=np.uint32)
    n_work = batch.n_pairs if seln is None else len(seln)
    out = np.zeros(n_work, dtype=RESULT_DTYPE)
    ops = None
    if mode == 1:
        if ops_stride is None:
            ops_stride = int(batch.read_len.max(initial=0)) + int(win["len"].max(initial=0)) + 4
        ops = np.zeros((n_work, ops_stride), dtype=np.uint32)
    ref = np.ascontiguousarray(batch.ref, dtype=np.uint8)
    reads = np.ascontiguousarray(batch.reads, dtype=np.uint8)
    roff = np.ascontiguousarray(batch.read_off, dtype=np.uint64)
    rlen = np.ascontiguousarray(batch.read_len, dtype=np.uint16)
    rc = lib().orc_batch(_ptr(ref), len(ref), _ptr(reads), _ptr(roff), _ptr(rlen),
                         batch.n_reads, _ptr(win), _ptr(seln), n_work,
                         ctypes.byref(_sc(scoring)), mode, _ptr(out), _ptr(ops),
                         ops_stride or 0, int(nthreads))
    if rc != 0:
        raise ValueError("non-ACGT base in the input")
    return out, ops


def cigar_string(ops) -> str:
    return "".join(f"{int(o) >> 4}{OPS[int(o) & 15]}" for o in ops)


def codes(s) -> np.ndarray:
    """'ACGT' text -> codes 0..3."""
    lut = np.full(256, 255, dtype=np.uint8)
    for k, c in enumerate(b"ACGT"):
        lut[c] = k
    a = lut[np.frombuffer(s.encode() if isinstance(s, str) else bytes(s), dtype=np.uint8)]
    if (a == 255).any():
        raise ValueError("non-ACGT base")
    return a


def pack2b(ascii_bytes: np.ndarray) -> np.ndarray:
    """Reference encoding: base p at byte p>>2, bits 2*(p&3) (A0 C1 G2 T3), padded
    with zero bits to a whole number of 32-bit words."""
    c = codes(np.asarray(ascii_bytes, dtype=np.uint8).tobytes()).astype(np.uint32)
    nwords = (len(c) + 15) // 16
    out = np.zeros(nwords * 4, dtype=np.uint8)
    for p in range(4):
        sl = c[p::4]
        out[:len(sl)] |= (sl << (2 * p)).astype(np.uint8)
    return out


def best_per_read(hits_score: np.ndarray, read_id: np.ndarray, n_reads: int):
    """Per read: index of the highest-scoring pair (lowest index on ties) and its
    score; reads without pairs get (0xFFFFFFFF, -1)."""
    best_pair = np.full(n_reads, 0xFFFFFFFF, dtype=np.uint32)
    best_score = np.full(n_reads, -1, dtype=np.int64)
    order = np.lexsort((np.arange(len(read_id)), -hits_score.astype(np.int64), read_id))
    rid_sorted = read_id[order]
    first = np.ones(len(order), dtype=bool)
    first[1:] = rid_sorted[1:] != rid_sorted[:-1]
    sel = order[first]
    best_pair[read_id[sel]] = sel.astype(np.uint32)
    best_score[read_id[sel]] = hits_score[sel]
    return best_pair, best_score.astype(np.int32)
