"""The packed int16 scoring kernel's own source, run on the CPU.

The wave body of k_sw_score16 (paper_1304_0681_amd/csrc/score16_body.h) is
compiled for the host with its cross-lane and byte-permute instructions
emulated (tests/host_model/score16_model.cpp: lanes are threads meeting at a
barrier around every cross-lane operation) and run, for every tile shape the
kernel is instantiated with, on pairs of every query length the shape can hold
(1 to G*RPL, windows of 1 to 1,000 bases, both strands, windows at and past the
reference ends), with every input array against a guard page: once placed at
the end of its pages (reads past an array's end fault) and once at the start
(reads before it fault).  Scores must equal the oracle's.  This is how the
kernel's indexing and arithmetic are checked for the shapes the library does
not dispatch packed on the GPU."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from batches import EDGE_M, EDGE_N, edge_batch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_model", "score16_model.cpp")
CXX = os.environ.get("HOST_CXX", "/opt/rocm/llvm/bin/clang++")
SC = (5, -4, -10, -1)
SHAPES = [(1, 16), (1, 32), (2, 32), (4, 16), (4, 25), (4, 32), (8, 13), (8, 20), (8, 32),
          (16, 32), (32, 32), (64, 32)]


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("no host clang++ for the kernel model")
    out = str(tmp_path_factory.mktemp("model") / "libscore16_model.so")
    subprocess.check_call([CXX, "-std=c++20", "-O2", "-shared", "-fPIC", "-pthread",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1304_0681_amd", "csrc"), SRC, "-o", out])
    L = ctypes.CDLL(out)
    L.model_score16.restype = ctypes.c_int
    return L


def _batch(seed, ms, ns, ref_len=60_000):
    g = np.random.default_rng(seed)
    ref = g.integers(0, 4, ref_len).astype(np.uint8)
    reads, wins = [], []
    for m in ms:
        for n in ns:
            for st in (0, 1):
                b0 = int(g.integers(1500, ref_len - m - 1500))
                seg = ref[b0:b0 + m].copy()
                mut = g.random(m) < 0.04
                seg[mut] = (seg[mut] + 1) % 4
                if m > 20 and g.random() < 0.5:
                    k = int(g.integers(5, m - 5))
                    seg = np.concatenate([seg[:k], g.integers(0, 4, 2).astype(np.uint8), seg[k:]])[:m]
                reads.append(synth.ASCII[(3 - seg[::-1]) if st else seg].tobytes())
                wins.append((len(reads) - 1, b0 - int(g.integers(0, max(1, n // 2 + 1))), n, st))
    # windows at the reference start and running past its end
    for n in (5, 40, 300):
        wins.append((0, 0, n, 0))
        wins.append((0, ref_len - n // 2, n, 1))
    return synth.custom(synth.ASCII[ref].tobytes(), reads, wins)


def _run(model, b, ids, G, RPL, at_end, waves=2):
    ref2b = oracle.pack2b(b.ref).view(np.uint32)
    reads2b = oracle.pack2b(b.reads).view(np.uint32)
    win = np.ascontiguousarray(b.windows)
    hits = np.zeros(b.n_pairs, dtype=[("score", "<i4"), ("read_end", "<i4"), ("ref_end", "<i4")])
    sc = np.array(SC, np.int32)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = model.model_score16(G, RPL, waves, int(at_end), p(ref2b), ctypes.c_uint64(len(b.ref)),
                             p(reads2b), ctypes.c_uint64(len(reads2b)),
                             p(np.ascontiguousarray(b.read_off, np.uint64)),
                             p(np.ascontiguousarray(b.read_len, np.uint16)),
                             ctypes.c_uint32(b.n_reads), p(win), ctypes.c_uint32(b.n_pairs),
                             p(ids), ctypes.c_uint32(len(ids)), p(sc), p(hits))
    assert rc == 0
    return hits


def _class_ids(b, cap):
    """Pairs the bucketing would hand a class of queries up to `cap` bases:
    valid, non-empty, longest window first (as the bins order them)."""
    m = b.read_len[b.windows["read_id"]].astype(np.int64)
    n = np.minimum(b.windows["len"].astype(np.int64),
                   np.maximum(len(b.ref) - b.windows["ref_begin"].astype(np.int64), 0))
    ok = (m > 0) & (n > 0) & (m <= cap)
    idx = np.nonzero(ok)[0]
    return idx[np.argsort(-(n[idx] >> 3), kind="stable")]


@pytest.mark.parametrize("G,RPL", SHAPES)
def test_packed_body_on_host_equals_oracle(model, G, RPL):
    cap = min(G * RPL, 2048)
    ms = sorted({x for x in (1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 99, 100, 101, 127, 128,
                             129, 159, 160, 161, 255, 256, 257, 511, 513, 1023, 1025, 2047, 2048)
                 if x <= cap} | {cap, max(cap // 2, 1)})
    if len(ms) > 8:             # bound the runtime of the big shapes: a spread of lengths
        ms = sorted(set(ms[::2]) | {ms[-1], ms[-2], 1})
    ns = [1, 16, 17, 65, 333, 1000]
    b = _batch(100 + G * 7 + RPL, ms, ns)
    ids = _class_ids(b, cap)
    ref, _ = oracle.align_batch(b, SC, mode=0, sel=ids.astype(np.uint32))
    for at_end in (True, False):
        h = _run(model, b, ids, G, RPL, at_end)
        bad = np.nonzero(h["score"][ids] != ref["score"])[0]
        assert len(bad) == 0, (G, RPL, at_end, ids[bad[:5]], h["score"][ids[bad[:5]]],
                               ref["score"][bad[:5]])
        others = np.setdiff1d(np.arange(b.n_pairs), ids)
        assert (h["score"][others] == -7).all()      # nothing written outside the class


def test_skipped_gpu_case_on_host(model):
    """The exact batch of the GPU case that did not return (edge lengths 1-2,300 x
    windows 1-1,000, both strands), split by query-length class as the
    bucketing splits it, each class on its default packed shape."""
    b = edge_batch(11, EDGE_M, EDGE_N)
    bounds = [0, 16, 32, 64, 100, 128, 160, 256, 512, 1024, 2048]
    default = {16: (1, 16), 32: (1, 32), 64: (2, 32), 100: (4, 25), 128: (4, 32), 160: (8, 20),
               256: (8, 32), 512: (16, 32), 1024: (32, 32), 2048: (64, 32)}
    m = b.read_len[b.windows["read_id"]].astype(np.int64)
    ref, _ = oracle.align_batch(b, SC, mode=0)
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        ids = _class_ids(b, hi)
        ids = ids[m[ids] > lo]
        if not len(ids):
            continue
        G, RPL = default[hi]
        h = _run(model, b, ids, G, RPL, at_end=True)
        assert (h["score"][ids] == ref["score"][ids]).all(), (hi, G, RPL)
