"""Batch wrapper of the oracle: strands, clipping, invalid pairs, threading,
and the seeded generators it is fed with."""
import numpy as np

import synth


def _rc(codes):
    return (3 - codes[::-1]).astype(np.uint8)


def test_batch_matches_single_pairs(orc):
    b = synth.config1(n_reads=60)
    res, ops = orc.align_batch(b, mode=1)
    ref = orc.codes(b.ref.tobytes())
    for k in range(b.n_pairs):
        w = b.windows[k]
        q = orc.codes(b.read(int(w["read_id"])))
        if w["strand"]:
            q = _rc(q)
        r = ref[int(w["ref_begin"]):int(w["ref_begin"]) + int(w["len"])]
        one, one_ops = orc.align_codes(q, r)
        assert tuple(one)[:5] == tuple(res[k])[:5]
        assert list(one_ops) == list(ops[k, :int(res[k]["n_ops"])])
    lin, _ = orc.align_batch(b, mode=0)
    for f in ("score", "read_end", "ref_end"):
        assert (lin[f] == res[f]).all()


def test_true_windows_score_high(orc):
    b = synth.config1()
    res, _ = orc.align_batch(b, mode=0)
    # 100-nt reads with ~1 % substitutions and rare indels against their origin
    assert np.median(res["score"]) >= 5 * 100 - 2 * 9
    assert (res["score"] > 250).mean() > 0.97


def test_threads_agree(orc):
    b = synth.config2(n_reads=300, ref_len=200_000)
    a, _ = orc.align_batch(b, mode=0, nthreads=1)
    c, _ = orc.align_batch(b, mode=0, nthreads=8)
    assert (a == c).all()


def test_clipping_invalid_and_empty(orc):
    ref = b"ACGTACGTTTGCA"
    reads = [b"ACGTACG", b"TTGCA", b""]
    wins = [(0, 0, 13, 0), (1, 8, 50, 0), (1, 40, 10, 0), (5, 0, 5, 0), (2, 0, 13, 0),
            (0, 0, 0, 1)]
    b = synth.custom(ref, reads, wins)
    res, _ = orc.align_batch(b, mode=1)
    assert int(res[0]["score"]) == 35
    assert int(res[1]["score"]) == 25 and int(res[1]["ref_end"]) == 4     # clipped at the end
    assert int(res[2]["score"]) == 0 and int(res[2]["ref_end"]) == -1      # starts past the end
    assert int(res[3]["score"]) == -1 and int(res[3]["status"]) == 2       # read id out of range
    assert int(res[4]["score"]) == 0                                        # empty read
    assert int(res[5]["score"]) == 0                                        # empty window


def test_pack2b_reference_layout(orc):
    a = np.frombuffer(b"ACGTTGCAA", dtype=np.uint8)
    p = orc.pack2b(a)
    assert len(p) == 4                       # one 32-bit word holds 16 bases
    # byte 0: A C G T -> 0 | 1<<2 | 2<<4 | 3<<6
    assert p[0] == 0b11100100
    assert p[1] == (3 | 2 << 2 | 1 << 4 | 0 << 6)
    assert p[2] == 0 and p[3] == 0
    g = np.random.default_rng(0)
    x = synth.ASCII[g.integers(0, 4, 1001)]
    pk = orc.pack2b(x)
    unpacked = np.array([(pk[i >> 2] >> (2 * (i & 3))) & 3 for i in range(len(x))])
    assert (synth.ASCII[unpacked] == x).all()


def test_best_per_read_reference(orc):
    sc = np.array([5, 9, 9, 1, 7, 3], dtype=np.int32)
    rid = np.array([0, 0, 0, 2, 2, 2], dtype=np.uint32)
    bp, bs = orc.best_per_read(sc, rid, 4)
    assert bp.tolist() == [1, 0xFFFFFFFF, 4, 0xFFFFFFFF]
    assert bs.tolist() == [9, -1, 7, -1]


def test_synth_deterministic_and_shaped():
    a = synth.config2(n_reads=2000, ref_len=300_000)
    b = synth.config2(n_reads=2000, ref_len=300_000)
    assert (a.windows == b.windows).all() and (a.reads == b.reads).all()
    k = np.bincount(a.windows["read_id"], minlength=a.n_reads)
    assert k.min() >= 1 and k.max() <= 8
    assert a.windows["len"].min() >= 200 and a.windows["len"].max() <= 600
    true = (a.windows["flags"] & synth.FLAG_TRUE_ORIGIN) != 0
    assert 0.7 < true.sum() / a.n_reads < 0.82
    gc = np.isin(a.ref, np.frombuffer(b"CG", np.uint8)).mean()
    assert abs(gc - 0.40) < 0.01
    c = synth.config4(n_reads=100, ref_len=300_000)
    assert c.n_pairs == 1600
