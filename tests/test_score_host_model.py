"""The score kernels' own source, run on the CPU.

tests/host_model/score_model.cpp compiles the unmodified kernel file
(paper_1304_0681_amd/csrc/score.hip) as C++ for the host, against a stand-in
HIP header, with the lanes of a wave as threads meeting at a barrier around
every cross-lane operation and the DPP shifts, v_perm_b32, v_alignbit_b32 and
v_bfe_i32 emulated from their definitions.  Every instantiation (the packed
int16 kernel at each tile shape, the int32 kernel at each shape and result mode,
and the strip-mined kernel) scores pairs of every query length the tile holds
(windows of 1 to 1,000 bases, both strands, windows at and past the reference
ends) with every input array against a guard page, once after its end and once
before its start; scores (and end cells where computed) must equal the oracle's.
This checks the kernels' indexing, arithmetic and termination for every shape,
including the ones the library does not dispatch on the GPU."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from batches import EDGE_M, EDGE_N, edge_batch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HM = os.path.join(ROOT, "tests", "host_model")
CXX = os.environ.get("HOST_CXX", "/opt/rocm/llvm/bin/clang++")
SC = (5, -4, -10, -1)
SHAPES = [(1, 16), (1, 32), (2, 32), (4, 16), (4, 25), (4, 32), (8, 13), (8, 20), (8, 32),
          (16, 32), (32, 32), (64, 32)]


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("no host clang++ for the kernel model")
    out = str(tmp_path_factory.mktemp("model") / "libscore_model.so")
    subprocess.check_call([CXX, "-std=c++20", "-O2", "-shared", "-fPIC", "-pthread", "-w",
                           "-I", os.path.join(HM, "hip_stub"), "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1304_0681_amd", "csrc"),
                           os.path.join(HM, "score_model.cpp"), "-o", out])
    L = ctypes.CDLL(out)
    L.model_score.restype = ctypes.c_int
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
    for n in (5, 40, 300):            # windows at the reference start and past its end
        wins.append((0, 0, n, 0))
        wins.append((0, ref_len - n // 2, n, 1))
    return synth.custom(synth.ASCII[ref].tobytes(), reads, wins)


def run_model(model, b, ids, packed16, G, RPL, mode, strip, at_end, waves=2):
    ref2b = oracle.pack2b(b.ref).view(np.uint32)
    reads2b = oracle.pack2b(b.reads).view(np.uint32)
    win = np.ascontiguousarray(b.windows)
    hits = np.zeros(b.n_pairs, dtype=[("score", "<i4"), ("read_end", "<i4"), ("ref_end", "<i4")])
    sc = np.array(SC, np.int32)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = model.model_score(int(packed16), G, RPL, mode, int(strip), waves, int(at_end), p(ref2b),
                           ctypes.c_uint64(len(b.ref)), p(reads2b), ctypes.c_uint64(len(reads2b)),
                           p(np.ascontiguousarray(b.read_off, np.uint64)),
                           p(np.ascontiguousarray(b.read_len, np.uint16)),
                           ctypes.c_uint32(b.n_reads), p(win), ctypes.c_uint32(b.n_pairs),
                           p(ids), ctypes.c_uint32(len(ids)), p(sc), p(hits))
    assert rc == 0
    return hits


def class_ids(b, lo, hi):
    """Pairs the bucketing hands a class of queries lo < m <= hi: valid,
    non-empty, longest window first (as the bins order them)."""
    m = b.read_len[b.windows["read_id"]].astype(np.int64)
    n = np.minimum(b.windows["len"].astype(np.int64),
                   np.maximum(len(b.ref) - b.windows["ref_begin"].astype(np.int64), 0))
    ok = (m > lo) & (n > 0) & (m <= hi)
    idx = np.nonzero(ok)[0]
    return idx[np.argsort(-(n[idx] >> 3), kind="stable")]


def _lengths(cap):
    ms = sorted({x for x in (1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 99, 100, 101, 127, 128,
                             129, 159, 160, 161, 255, 256, 257, 511, 513, 1023, 1025, 2047, 2048)
                 if x <= cap} | {cap, max(cap // 2, 1)})
    if len(ms) > 8:             # bound the runtime of the big shapes: a spread of lengths
        ms = sorted(set(ms[::2]) | {ms[-1], ms[-2], 1})
    return ms


def _check(h, ref, ids, ends, what):
    bad = np.nonzero(h["score"][ids] != ref["score"])[0]
    assert len(bad) == 0, (what, ids[bad[:5]], h["score"][ids[bad[:5]]], ref["score"][bad[:5]])
    if ends:
        for f in ("read_end", "ref_end"):
            assert (h[f][ids] == ref[f]).all(), (what, f)


@pytest.mark.parametrize("G,RPL", SHAPES)
def test_packed_kernel_on_host_equals_oracle(model, G, RPL):
    cap = min(G * RPL, 2048)
    b = _batch(100 + G * 7 + RPL, _lengths(cap), [1, 16, 17, 65, 333, 1000])
    ids = class_ids(b, 0, cap)
    ref, _ = oracle.align_batch(b, SC, mode=0, sel=ids.astype(np.uint32))
    for at_end in (True, False):
        h = run_model(model, b, ids, True, G, RPL, 0, False, at_end)
        _check(h, ref, ids, False, ("packed", G, RPL, at_end))
        others = np.setdiff1d(np.arange(b.n_pairs), ids)
        assert (h["score"][others] == -7).all()      # nothing written outside the class


@pytest.mark.parametrize("G,RPL", SHAPES)
def test_int32_kernel_on_host_equals_oracle(model, G, RPL):
    cap = min(G * RPL, 2048)
    b = _batch(300 + G * 7 + RPL, _lengths(cap), [1, 17, 65, 333, 1000])
    ids = class_ids(b, 0, cap)
    ref, _ = oracle.align_batch(b, SC, mode=0, sel=ids.astype(np.uint32))
    for mode in (0, 1, 2):
        h = run_model(model, b, ids, False, G, RPL, mode, False, at_end=(mode != 1))
        _check(h, ref, ids, mode > 0, ("int32", G, RPL, mode))


def test_strip_kernel_on_host_equals_oracle(model):
    b = _batch(401, [2049, 2300, 4200], [17, 300, 1000], ref_len=80_000)
    ids = class_ids(b, 2048, 65535)
    ref, _ = oracle.align_batch(b, SC, mode=0, sel=ids.astype(np.uint32))
    for mode in (0, 1, 2):
        h = run_model(model, b, ids, False, 64, 32, mode, True, at_end=(mode != 2))
        _check(h, ref, ids, mode > 0, ("strip", mode))


def test_skipped_gpu_case_on_host(model):
    """The exact batch of the GPU case that did not return (edge lengths 1-2,300 x
    windows 1-1,000, both strands), split by query-length class as the
    bucketing splits it, each class on its default packed shape."""
    b = edge_batch(11, EDGE_M, EDGE_N)
    bounds = [0, 16, 32, 64, 100, 128, 160, 256, 512, 1024, 2048]
    default = {16: (1, 16), 32: (1, 32), 64: (2, 32), 100: (4, 25), 128: (4, 32), 160: (8, 20),
               256: (8, 32), 512: (16, 32), 1024: (32, 32), 2048: (64, 32)}
    ref, _ = oracle.align_batch(b, SC, mode=0)
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        ids = class_ids(b, lo, hi)
        if len(ids):
            G, RPL = default[hi]
            h = run_model(model, b, ids, True, G, RPL, 0, False, at_end=True)
            assert (h["score"][ids] == ref["score"][ids]).all(), (hi, G, RPL)
