"""The region and CAL seeker kernels' own source, run on the CPU.

tests/host_model/seeker_model.cpp compiles the unmodified kernel file
(paper_1304_0681_amd/csrc/seeker.hip) as C++ for the host against the
stand-in HIP header; the lanes of a block are threads with barriers for
__syncthreads and the wave barrier, blocks run one after another, and every
array lies against a guard page (after its end, then before its start).  The
index (positions per k-mer), the regions (exact order) and the CALs must equal
the oracle's (oracle/seeker_ref.py) on the seeded inputs of
tests/seeker_inputs.py."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import seeker_ref as sr
from oracle import stageb_ref as sb
from seeker_inputs import one_edit_reads, reads_from, reference_with_repeats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HM = os.path.join(ROOT, "tests", "host_model")
CXX = os.environ.get("HOST_CXX", "/opt/rocm/llvm/bin/clang++")
REGION_DTYPE = np.dtype([("first", "<u4"), ("read_pos", "<u2"), ("strand", "u1"), ("reserved", "u1")])
CAL_DTYPE = np.dtype([("read_id", "<u4"), ("first", "<u4"), ("last", "<u4"), ("strand", "u1"),
                      ("valid", "u1"), ("reserved", "<u2")])
N_CALS = 16
BMAP_DTYPE = np.dtype([("first", "<u4"), ("last", "<u4"), ("strand", "u1"), ("edits", "u1"),
                       ("op", "u1"), ("reserved", "u1"), ("edit_pos", "<i4")])
N_MAPS = 16


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("no host clang++ for the kernel model")
    out = str(tmp_path_factory.mktemp("kmodel") / "libseeker_model.so")
    subprocess.check_call([CXX, "-std=c++20", "-O2", "-shared", "-fPIC", "-pthread", "-w",
                           "-I", os.path.join(HM, "hip_stub"), "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1304_0681_amd", "csrc"),
                           os.path.join(HM, "seeker_model.cpp"), "-o", out])
    return ctypes.CDLL(out)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pack(codes):
    return oracle.pack2b(synth.ASCII[codes]).view(np.uint32)


def _index(model, ref, k, at_end):
    n_pos = len(ref) - k + 1
    starts = np.zeros(4 ** k + 1, np.uint32)
    pos = np.zeros(max(n_pos, 1), np.uint32)
    model.model_index(at_end, _p(_pack(ref)), ctypes.c_uint64(len(ref)), k, _p(starts), _p(pos))
    return starts, pos


@pytest.mark.parametrize("k,at_end", [(6, 1), (9, 0), (10, 1)])
def test_index(model, k, at_end):
    ref = reference_with_repeats(7 + k, 40_000)
    starts, pos = _index(model, ref, k, at_end)
    want = sr.build_index_fast(ref, k)
    assert starts[-1] == len(ref) - k + 1 and (np.diff(starts.astype(np.int64)) >= 0).all()
    got = {c: sorted(pos[starts[c]:starts[c + 1]].tolist())
           for c in np.nonzero(np.diff(starts.astype(np.int64)))[0]}
    assert got == want


def _reads_arrays(reads):
    lens = np.array([len(q) for q in reads], np.uint16)
    off = np.zeros(len(reads), np.uint64)
    off[1:] = np.cumsum(lens[:-1], dtype=np.uint64)
    cat = np.concatenate(reads)
    return _pack(cat), len(cat), off, lens


def _regions(model, reads, starts, pos, k, step, offset, max_occ, cap, at_end):
    r2b, rl, off, lens = _reads_arrays(reads)
    out = np.zeros(max(cap, 1), REGION_DTYPE)
    end = np.zeros(len(reads), np.uint64)
    model.model_regions(at_end, _p(r2b), ctypes.c_uint64(rl), _p(off), _p(lens), len(reads),
                        _p(starts), _p(pos), ctypes.c_uint64(len(pos)), k, step, offset, max_occ,
                        _p(out), ctypes.c_uint64(cap), _p(end))
    return out[:cap], end


@pytest.mark.parametrize("k,step,offset,max_occ,at_end", [(9, 7, 4, 8, 1), (10, 12, 7, 3, 0),
                                                          (8, 5, 2, 40, 1)])
def test_regions(model, k, step, offset, max_occ, at_end):
    ref = reference_with_repeats(20 + k, 60_000)
    starts, pos = _index(model, ref, k, 1)
    reads, _, _ = reads_from(30 + k, ref, 300)
    regs, end = _regions(model, reads, starts, pos, k, step, offset, max_occ, 10**6, at_end)
    idx = sr.build_index_fast(ref, k)
    b = 0
    n_cut = 0
    for r, q in enumerate(reads):
        want = sr.regions(q, idx, k, step, offset, max_occ)
        e = int(end[r])
        got = [(int(x["strand"]), int(x["first"]), int(x["first"]) + k - 1, int(x["read_pos"]))
               for x in regs[b:e]]
        assert got == want, r
        b = e
        n_cut += any(len(idx.get(sr.kmer_code(q[s:s + k]), [])) > max_occ
                     for s in sr.seed_starts(len(q), k, step, offset))
    assert (regs["reserved"][:b] == 0).all()
    assert n_cut > 5 and b > 1000
    # a capacity below the total: counts unchanged, regions written up to it
    cap = b // 2
    regs2, end2 = _regions(model, reads, starts, pos, k, step, offset, max_occ, cap, at_end)
    assert (end2 == end).all() and (regs2 == regs[:cap]).all()


def _cal_rows(cals, n_reads):
    out = []
    for r in range(n_reads):
        row = cals[r * N_CALS:(r + 1) * N_CALS]
        v = [(int(c["read_id"]), int(c["first"]), int(c["last"]), int(c["strand"]), 1)
             for c in row if c["valid"]]
        assert all(c["read_id"] == r for c in row)
        k = len(v)
        assert row["valid"][:k].all() and not row["valid"][k:].any()
        assert (row["first"][k:] == 0).all() and (row["last"][k:] == 0).all()
        out.append(v)
    return out


@pytest.mark.parametrize("merge_gap,min_len,at_end", [(50, 20, 1), (0, 9, 0), (200, 40, 1)])
def test_cal_seek(model, merge_gap, min_len, at_end):
    k, step, offset, max_occ = 10, 12, 7, 6
    ref = reference_with_repeats(41, 80_000, families=3, copies=(3, 20))
    starts, pos = _index(model, ref, k, 1)
    reads, _, _ = reads_from(42, ref, 400)
    regs, end = _regions(model, reads, starts, pos, k, step, offset, max_occ, 10**6, 1)
    cals = np.zeros(len(reads) * N_CALS, CAL_DTYPE)
    model.model_cal_seek(at_end, _p(regs), ctypes.c_uint64(len(regs)), _p(end), len(reads),
                         ctypes.c_uint64(len(regs)), k, merge_gap, min_len, None, _p(cals), 3)
    got = _cal_rows(cals, len(reads))
    idx = sr.build_index_fast(ref, k)
    n = 0
    for r, q in enumerate(reads):
        want = sr.cals(r, sr.regions(q, idx, k, step, offset, max_occ), merge_gap, min_len)
        assert got[r] == want, r
        n += len(want)
    assert n > 200


def test_cal_seek_caps(model):
    """More regions than the seeker takes, more CALs than the slots, both
    strands, a capacity that cuts a read's regions."""
    g = np.random.default_rng(43)
    k = 15
    rows, ends = [], []
    for r in range(6):
        n = [3000, 40, 0, 700, 2049, 17][r]
        st = g.integers(0, 2, n)
        first = np.sort(g.integers(0, 10**6, n)) if r != 3 else np.arange(n) * 200
        rows += [(int(f), 0, int(s), 0) for f, s in zip(first, st)]
        ends.append(len(rows))
    regs = np.array(rows, REGION_DTYPE)
    end = np.array(ends, np.uint64)
    for cap in (len(regs), ends[3] + 100):
        cals = np.zeros(6 * N_CALS, CAL_DTYPE)
        model.model_cal_seek(1, _p(regs), ctypes.c_uint64(len(regs)), _p(end), 6,
                             ctypes.c_uint64(cap), k, 30, 10, None, _p(cals), 2)
        got = _cal_rows(cals, 6)
        b = 0
        for r in range(6):
            e = min(ends[r], cap)
            reg_r = [(int(x["strand"]), int(x["first"]), int(x["first"]) + k - 1, 0)
                     for x in regs[b:e]] if e > b else []
            assert got[r] == sr.cals(r, reg_r, 30, 10), (cap, r)
            b = ends[r]
    assert len(got[3]) == N_CALS


@pytest.mark.parametrize("at_end", [1, 0])
def test_stage_b(model, at_end):
    """Whole-read mapping with at most one edit: every read's records (fewest
    edits, by strand and start) equal the oracle's; reads with more edits and
    random reads get none; the skip mask empties their CAL slots."""
    k, step, offset, max_occ = 10, 12, 7, 6
    ref = reference_with_repeats(44, 60_000, families=3, copies=(2, 9))
    starts, pos = _index(model, ref, k, 1)
    reads = one_edit_reads(45, ref, 240) + reads_from(46, ref, 160)[0]
    regs, end = _regions(model, reads, starts, pos, k, step, offset, max_occ, 10**6, 1)
    r2b, rl, off, lens = _reads_arrays(reads)
    maps = np.zeros(len(reads) * N_MAPS, BMAP_DTYPE)
    n_maps = np.zeros(len(reads), np.uint32)
    model.model_stage_b(at_end, _p(r2b), ctypes.c_uint64(rl), _p(off), _p(lens), len(reads),
                        _p(_pack(ref)), ctypes.c_uint64(len(ref)), _p(regs),
                        ctypes.c_uint64(len(regs)), _p(end), ctypes.c_uint64(len(regs)), _p(maps),
                        _p(n_maps), 3)
    idx = sr.build_index_fast(ref, k)
    kinds = set()
    for r, q in enumerate(reads):
        want = sb.map_read(q, ref, idx, k, step, offset, max_occ)
        row = maps[r * N_MAPS:(r + 1) * N_MAPS]
        n = int(n_maps[r])
        got = [(int(x["strand"]), int(x["first"]), int(x["last"]), int(x["edits"]), int(x["op"]),
                int(x["edit_pos"])) for x in row[:n]]
        assert got == want, r
        assert (row[n:] == np.zeros(1, BMAP_DTYPE)).all()
        kinds |= {w[4] for w in want}
    assert kinds == {sb.EXACT, sb.SUBST, sb.DEL, sb.INS}
    assert (n_maps[:240] > 0).mean() > 0.95
    # reads stage B mapped get no CALs
    cals = np.zeros(len(reads) * N_CALS, CAL_DTYPE)
    model.model_cal_seek(at_end, _p(regs), ctypes.c_uint64(len(regs)), _p(end), len(reads),
                         ctypes.c_uint64(len(regs)), k, 50, 20, _p(n_maps), _p(cals), 2)
    got = _cal_rows(cals, len(reads))
    for r, q in enumerate(reads):
        want = [] if n_maps[r] else sr.cals(r, sr.regions(q, idx, k, step, offset, max_occ), 50, 20)
        assert got[r] == want
