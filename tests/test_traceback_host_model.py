"""The traceback kernel's own source, run on the CPU.

tests/host_model/traceback_model.cpp compiles the unmodified kernel file
(paper_1304_0681_amd/csrc/traceback.hip) as C++ for the host, against the
stand-in HIP header, on the lockstep wave model (lanes as threads meeting at a
barrier around every cross-lane operation: the whole wave during the DP, only
the lane group during the group's walk; DPP shifts, v_bitop3_b32,
v_alignbit_b32 and v_bfe_i32 emulated from their definitions).  Every tile the
library launches runs on pairs of lengths spread over its class, both strands,
windows at and past the reference ends, with and without the band of the score
pass's hits, with a last wave whose lane groups are partly idle, and with
selected ids that name no pair placed first.  Every array and the code scratch
lie against a guard page (after their end, then before their start);
coordinates, scores and CIGARs must equal the oracle's, and nothing outside the
class may be written."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HM = os.path.join(ROOT, "tests", "host_model")
CXX = os.environ.get("HOST_CXX", "/opt/rocm/llvm/bin/clang++")
SC = (5, -4, -10, -1)
NONE = 0xFFFFFFFF
ALN = np.dtype([("score", "<i4"), ("read_begin", "<i4"), ("read_end", "<i4"),
                ("ref_begin", "<i4"), ("ref_end", "<i4"), ("n_ops", "<u4"), ("status", "<u4")])


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("no host clang++ for the kernel model")
    out = str(tmp_path_factory.mktemp("model") / "libtb_model.so")
    subprocess.check_call([CXX, "-std=c++20", "-O2", "-shared", "-fPIC", "-pthread", "-w",
                           "-I", os.path.join(HM, "hip_stub"), "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1304_0681_amd", "csrc"),
                           os.path.join(HM, "traceback_model.cpp"), "-o", out])
    L = ctypes.CDLL(out)
    L.model_traceback.restype = ctypes.c_int
    return L


def _batch(seed, ms, ns, ref_len=40_000):
    g = np.random.default_rng(seed)
    ref = g.integers(0, 4, ref_len).astype(np.uint8)
    reads, wins = [], []
    for k, m in enumerate(ms):
        n = ns[k % len(ns)]
        st = k & 1
        b0 = int(g.integers(1000, ref_len - m - 1000))
        seg = ref[b0:b0 + m].copy()
        mut = g.random(m) < 0.03
        seg[mut] = (seg[mut] + 1) % 4
        if m > 45:      # a 3-base deletion
            k0 = int(g.integers(20, m - 20))
            seg = np.concatenate([seg[:k0], seg[k0 + 3:], g.integers(0, 4, 3).astype(np.uint8)])
        reads.append(synth.ASCII[(3 - seg[::-1]) if st else seg].tobytes())
        wins.append((len(reads) - 1, max(b0 - int(g.integers(0, max(1, n // 3))), 0), n, st))
    wins.append((0, 0, 300, 0))                       # at the reference start
    wins.append((1, ref_len - 150, 300, 1))           # running past its end
    return synth.custom(synth.ASCII[ref].tobytes(), reads, wins)


def _run(model, b, sel, ids, G, RPL, strip, at_end, hits, waves=2, codes_words=None):
    m = b.read_len[b.windows["read_id"][sel[ids]]].astype(np.int64)
    n = np.minimum(b.windows["len"][sel[ids]].astype(np.int64),
                   len(b.ref) - b.windows["ref_begin"][sel[ids]].astype(np.int64))
    nmax, mmax = int(n.max()), int(m.max())
    SR = G * RPL
    strips = (mmax + SR - 1) // SR if strip else 1
    wpl = (RPL + 7) // 8
    slot = strips * G * wpl * (nmax + G - 1) + (2 * nmax if strip else 0) + mmax + nmax + 8
    ref2b = oracle.pack2b(b.ref).view(np.uint32)
    reads2b = oracle.pack2b(b.reads).view(np.uint32)
    win = np.ascontiguousarray(b.windows)
    stride = mmax + nmax + 4
    aln = np.full(len(sel), -7, ALN)
    ops = np.full((len(sel), stride), 7, np.uint32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    sc = np.array(SC, np.int32)
    h = None if hits is None else np.ascontiguousarray(hits)
    rc = model.model_traceback(G, RPL, int(strip), waves, int(at_end), p(ref2b), ctypes.c_uint64(len(b.ref)),
                               p(reads2b), ctypes.c_uint64(len(reads2b)),
                               p(np.ascontiguousarray(b.read_off, np.uint64)),
                               p(np.ascontiguousarray(b.read_len, np.uint16)),
                               ctypes.c_uint32(b.n_reads), p(win), ctypes.c_uint32(b.n_pairs),
                               p(sel), ctypes.c_uint32(len(sel)), p(ids), ctypes.c_uint32(len(ids)),
                               ctypes.c_uint32(nmax), ctypes.c_uint32(mmax), p(sc),
                               None if h is None else p(h), ctypes.c_uint64(waves * (64 // G) * slot if codes_words is None else codes_words),
                               p(aln), p(ops), ctypes.c_uint32(stride))
    assert rc == 0
    return aln, ops


# (G, RPL, strip, class bounds lo < m <= hi): the library's traceback classes
SHAPES = [(2, 8, False, 0, 16), (4, 8, False, 16, 32), (8, 8, False, 32, 64),
          (8, 13, False, 64, 100), (16, 8, False, 100, 128), (8, 20, False, 128, 160),
          (32, 8, False, 160, 256), (64, 8, False, 256, 512), (64, 12, False, 512, 768),
          (64, 16, False, 768, 1024), (64, 32, True, 1024, 2400)]


@pytest.mark.parametrize("G,RPL,strip,lo,hi", SHAPES)
def test_traceback_on_host_equals_oracle(model, G, RPL, strip, lo, hi):
    ppw = 64 // G
    n_pairs = max(ppw + ppw // 2 + 1, 6)      # the last wave's groups partly idle
    ms = [int(x) for x in np.linspace(lo + 1, min(hi, 2300), n_pairs).round()]
    b = _batch(500 + 7 * G + RPL, ms, [max(hi // 2, 8), 40, hi + 200, 1000])
    pairs = np.arange(b.n_pairs, dtype=np.uint32)
    m = b.read_len[b.windows["read_id"]].astype(np.int64)
    cls = pairs[(m > lo) & (m <= hi)]
    # ids naming no pair come first in the selection; the class's pairs follow
    sel = np.concatenate([[NONE, b.n_pairs], cls, [NONE]]).astype(np.uint32)
    ids = np.arange(2, 2 + len(cls), dtype=np.uint32)
    ra, rops = oracle.align_batch(b, SC, mode=1, sel=cls)
    hits_all, _ = oracle.align_batch(b, SC, mode=0)
    hits = np.zeros(b.n_pairs, [("score", "<i4"), ("read_end", "<i4"), ("ref_end", "<i4")])
    for f in ("score", "read_end", "ref_end"):
        hits[f] = hits_all[f]
    for band, at_end in ((False, True), (True, False)):
        aln, ops = _run(model, b, sel, ids, G, RPL, strip, at_end, hits if band else None)
        got = aln[ids]
        for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
            assert (got[f] == ra[f]).all(), (G, RPL, band, f, got[f], ra[f])
        for k, i in enumerate(ids):
            nn = int(ra[k]["n_ops"])
            assert (ops[i, :nn] == rops[k, :nn]).all(), (G, RPL, band, k)
        others = np.setdiff1d(np.arange(len(sel)), ids)
        assert (aln["score"][others] == -7).all() and (ops[others] == 7).all()


@pytest.mark.parametrize("G,RPL,strip,lo,hi", [SHAPES[3], SHAPES[8]])
def test_traceback_on_host_without_room_marks_pairs(model, G, RPL, strip, lo, hi):
    """A code scratch too small for one wave's slots: every pair of the class is
    marked (status 4, score -1, no ops) and nothing is read or written beyond
    the scratch."""
    ms = [int(x) for x in np.linspace(lo + 1, hi, 9).round()]
    b = _batch(900 + G, ms, [200, 40, 1000])
    m = b.read_len[b.windows["read_id"]].astype(np.int64)
    cls = np.nonzero((m > lo) & (m <= hi))[0].astype(np.uint32)
    sel = np.concatenate([[NONE], cls]).astype(np.uint32)
    ids = np.arange(1, 1 + len(cls), dtype=np.uint32)
    aln, ops = _run(model, b, sel, ids, G, RPL, strip, True, None, codes_words=16)
    got = aln[ids]
    assert (got["status"] == 4).all() and (got["score"] == -1).all() and (got["n_ops"] == 0).all()
    assert aln["score"][0] == -7 and (ops == 7).all()
