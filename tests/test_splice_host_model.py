"""The spliced-read kernels' own source, run on the CPU.

tests/host_model/splice_model.cpp compiles the unmodified kernel file
(paper_1304_0681_amd/csrc/splice.hip) as C++ for the host against the
stand-in HIP header; its kernels have no cross-lane operations or barriers,
so the lanes of one block run one after another.  Every array lies against a
guard page (after its end, then before its start).  CALs, joined windows
(before the library's stable compaction, done here), rewritten CIGARs and
junction counts must equal the oracle's (oracle/junction_ref.py) on the
seeded inputs of tests/splice_inputs.py."""
import ctypes
import os
import subprocess
from collections import Counter

import numpy as np
import pytest

import oracle
import synth
from oracle import junction_ref as jr
from splice_inputs import ALN_DTYPE, CAL_DTYPE, WINDOW_DTYPE, planted_alignments, random_cals

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HM = os.path.join(ROOT, "tests", "host_model")
CXX = os.environ.get("HOST_CXX", "/opt/rocm/llvm/bin/clang++")
JUNC_DTYPE = np.dtype([("start", "<u8"), ("end", "<u8"), ("count", "<u4"), ("strand", "<u4")])
MIN_INTRON = 40


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("no host clang++ for the kernel model")
    out = str(tmp_path_factory.mktemp("smodel") / "libsplice_model.so")
    subprocess.check_call([CXX, "-std=c++20", "-O2", "-shared", "-fPIC", "-w",
                           "-I", os.path.join(HM, "hip_stub"), "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1304_0681_amd", "csrc"),
                           os.path.join(HM, "splice_model.cpp"), "-o", out])
    L = ctypes.CDLL(out)
    L.model_list.restype = ctypes.c_uint32
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cal_tuples(c):
    return [(int(x["read_id"]), int(x["first"]), int(x["last"]), int(x["strand"]), int(x["valid"]))
            for x in c]


@pytest.mark.parametrize("at_end", [1, 0])
def test_seed_cals(model, at_end):
    g = np.random.default_rng(11)
    n_pairs, n_seeds = 700, 500
    win = np.zeros(n_pairs, WINDOW_DTYPE)
    win["read_id"] = g.integers(0, n_seeds, n_pairs)
    win["ref_begin"] = g.integers(0, 2**32 - 1, n_pairs, dtype=np.uint64)
    win["ref_begin"][:600] = g.integers(0, 10**8, 600)
    win["len"] = g.integers(1, 1000, n_pairs)
    win["strand"] = g.integers(0, 2, n_pairs)
    best = g.integers(0, n_pairs + 50, n_seeds).astype(np.uint32)
    best[:5] = 0xFFFFFFFF
    aln = np.zeros(n_seeds, ALN_DTYPE)
    aln["score"] = g.integers(-1, 300, n_seeds)
    aln["ref_begin"] = g.integers(0, 500, n_seeds)
    aln["ref_end"] = aln["ref_begin"] + g.integers(0, 400, n_seeds)
    neg = aln["score"] <= 0
    aln["ref_begin"][neg] = -1
    aln["ref_end"][neg] = -1
    win["ref_begin"][650:660] = 2**32 - 100        # spans crossing 2^32
    best[10:20] = np.arange(650, 660)
    aln["score"][10:20] = 100
    aln["ref_begin"][10:20] = np.arange(90, 110, 2)
    aln["ref_end"][10:20] = aln["ref_begin"][10:20] + 5
    seed_read = np.sort(g.integers(0, 120, n_seeds)).astype(np.uint32)
    out = np.zeros(n_seeds, CAL_DTYPE)
    model.model_seed_cals(at_end, n_seeds, _p(win), n_pairs, _p(best), _p(aln), _p(seed_read),
                          ctypes.c_int32(60), _p(out))
    ref = jr.seed_cals(win, best, aln, seed_read, 60)
    assert _cal_tuples(out) == ref
    assert (out["reserved"] == 0).all()
    got_valid = int(out["valid"].sum())
    assert 100 < got_valid < n_seeds
    # spans crossing 2^32 are dropped, those below it kept
    assert out["valid"][10:13].all() and not out["valid"][13:20].any()


@pytest.mark.parametrize("at_end", [1, 0])
@pytest.mark.parametrize("ext,max_gap", [(30, 5000), (0, 1), (100, 0)])
def test_join(model, at_end, ext, max_gap):
    ref_len, n_reads = 3_000_000, 400
    cals = random_cals(12 + ext, n_reads, ref_len, ext, max_gap)
    n = len(cals)
    tmp = np.zeros(n, WINDOW_DTYPE)
    keep = np.zeros(n, np.uint8)
    model.model_join(at_end, n, _p(cals), n_reads, ctypes.c_uint64(ref_len), ext, max_gap, _p(tmp),
                     _p(keep))
    got = [(int(w["read_id"]), int(w["ref_begin"]), int(w["len"]), int(w["strand"]))
           for w in tmp[keep == 1]]
    assert (tmp[keep == 1]["flags"] == 0).all()
    ref = jr.join_cals(_cal_tuples(cals), n_reads, ref_len, ext=ext, max_gap=max_gap)
    assert got == ref
    assert len(ref) > 200


def _run_detect(model, at_end, seed, n_aln, cap=1 << 12, ops_stride=48, min_score=30):
    ref, win, aln, ops = planted_alignments(seed, n_aln, MIN_INTRON, ops_stride, min_score)
    ref2b = oracle.pack2b(synth.ASCII[ref]).view(np.uint32)
    pair_ids = np.arange(n_aln, dtype=np.uint32)
    keys = np.zeros(cap, np.uint64)
    counts = np.zeros(cap, np.uint32)
    nj = np.zeros(n_aln, np.uint32)
    dropped = np.zeros(1, np.uint32)
    got_ops = ops.copy()
    model.model_detect(at_end, n_aln, _p(pair_ids), _p(win), len(win), _p(ref2b),
                       ctypes.c_uint64(len(ref)), _p(aln), _p(got_ops), ops_stride,
                       ctypes.c_int32(min_score), MIN_INTRON, _p(keys), _p(counts), cap, _p(nj),
                       _p(dropped))
    return ref, win, aln, ops, got_ops, keys, counts, nj, int(dropped[0])


def _oracle_detect(ref, win, aln, ops, min_score):
    want_ops, want_nj, lists = ops.copy(), [], []
    for k in range(len(aln)):
        a = aln[k]
        if a["status"] or a["score"] < max(min_score, 1):
            want_nj.append(0)
            continue
        w = win[k]
        t = ref[int(w["ref_begin"]):int(w["ref_begin"]) + int(w["len"])]
        n = int(a["n_ops"])
        new, js = jr.detect(t, ops[k, :n], int(a["ref_begin"]), MIN_INTRON, int(w["ref_begin"]))
        want_ops[k, :n] = new
        want_nj.append(len(js))
        lists.append(js)
    return want_ops, np.array(want_nj), jr.count(lists)


def _table(keys, counts):
    occ = keys != 0
    return Counter({(int(k >> 17), int(k >> 17) + int((k >> 1) & 0xFFFF), int(k & 1)): int(c)
                    for k, c in zip(keys[occ], counts[occ])})


@pytest.mark.parametrize("at_end", [1, 0])
def test_detect_and_count(model, at_end):
    ref, win, aln, ops, got_ops, keys, counts, nj, dropped = _run_detect(model, at_end, 21, 600)
    want_ops, want_nj, want = _oracle_detect(ref, win, aln, ops, 30)
    assert (got_ops == want_ops).all()
    assert (nj == want_nj).all()
    assert dropped == 0
    assert _table(keys, counts) == want
    # the planted cases exercise the search: junctions on both motifs, shifted
    # placements, and runs left as deletions
    assert sum(want.values()) > 300 and {s for _, _, s in want} == {0, 1}
    n_shifted = sum(int((want_ops[k] != ops[k]).sum()) > 1 for k in range(len(ops)))
    assert n_shifted > 50
    assert any(((o & 15) == 2 and (o >> 4) >= MIN_INTRON) for o in want_ops.reshape(-1))
    # listing
    out = np.zeros(len(want) + 8, JUNC_DTYPE)
    n = model.model_list(at_end, _p(keys), _p(counts), len(keys), _p(out), len(out))
    assert n == len(want)
    listed = Counter({(int(r["start"]), int(r["end"]), int(r["strand"])): int(r["count"])
                      for r in out[:n]})
    assert listed == want
    small = np.zeros(3, JUNC_DTYPE)
    assert model.model_list(at_end, _p(keys), _p(counts), len(keys), _p(small), 3) == len(want)


def test_counts_accumulate_and_full_table(model):
    """The same alignments twice double every count; a table with fewer slots
    than distinct junctions keeps what fits and counts the rest as dropped."""
    ref, win, aln, ops, got_ops, keys, counts, nj, dropped = _run_detect(model, 1, 22, 200)
    _, _, want = _oracle_detect(ref, win, aln, ops, 30)
    ops2 = ops.copy()
    nj2 = np.zeros(len(aln), np.uint32)
    dr = np.zeros(1, np.uint32)
    ref2b = oracle.pack2b(synth.ASCII[ref]).view(np.uint32)
    model.model_detect(1, len(aln), _p(np.arange(len(aln), dtype=np.uint32)), _p(win), len(win),
                       _p(ref2b), ctypes.c_uint64(len(ref)), _p(aln), _p(ops2), 48,
                       ctypes.c_int32(30), MIN_INTRON, _p(keys), _p(counts), len(keys), _p(nj2),
                       _p(dr))
    assert _table(keys, counts) == Counter({k: 2 * v for k, v in want.items()})
    cap = 16
    assert len(want) > cap
    *_, keys_s, counts_s, nj_s, dropped_s = _run_detect(model, 1, 22, 200, cap=cap)
    tab = _table(keys_s, counts_s)
    assert len(tab) == cap
    assert all(want[k] == v for k, v in tab.items())
    assert dropped_s == sum(want.values()) - sum(tab.values())
