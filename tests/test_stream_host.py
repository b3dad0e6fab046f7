"""Host logic of the stream's resume manifest (no GPU)."""
import json
import os

import pytest

from paper_1304_0681_amd.stream import ChunkManifest


def test_manifest_records_and_resumes(tmp_path):
    p = str(tmp_path / "run.json")
    m = ChunkManifest(p, 5, key={"chunk": 1000})
    assert m.pending() == [0, 1, 2, 3, 4] and not m.complete
    assert json.load(open(p)) == {"key": {"chunk": 1000}, "n_chunks": 5, "done": []}
    m.mark(0)
    m.mark(3)
    assert not os.path.exists(p + ".tmp")
    m2 = ChunkManifest(p, 5, key={"chunk": 1000})        # a restarted run
    assert m2.pending() == [1, 2, 4]
    for i in m2.pending():
        m2.mark(i)
    assert m2.complete and ChunkManifest(p, 5, key={"chunk": 1000}).pending() == []
    with pytest.raises(IndexError):
        m2.mark(5)


def test_manifest_of_another_run_is_refused(tmp_path):
    p = str(tmp_path / "run.json")
    ChunkManifest(p, 5, key="a").mark(2)
    with pytest.raises(ValueError):
        ChunkManifest(p, 6, key="a")
    with pytest.raises(ValueError):
        ChunkManifest(p, 5, key="b")


def test_interrupted_loop_resumes_exactly_once(tmp_path):
    """The resume protocol the stream follows (consume, then mark), driven by a
    host hook that fails once at chunk 4: every chunk is consumed exactly once
    over the two runs and the results equal an uninterrupted run's."""
    p = str(tmp_path / "run.json")
    n = 7
    got = {}

    def run(fail_at):
        m = ChunkManifest(p, n, key="loop")
        for i in m.pending():
            if i == fail_at:
                raise RuntimeError("injected")
            assert i not in got
            got[i] = i * i
            m.mark(i)

    with pytest.raises(RuntimeError):
        run(4)
    assert sorted(got) == [0, 1, 2, 3]
    run(None)
    assert got == {i: i * i for i in range(n)}


def test_write_bed_sorted_with_strands(tmp_path):
    """Junctions come out as BED lines sorted by position, with their counts as
    scores and + / - for the GT-AG / CT-AC motif."""
    import numpy as np

    from paper_1304_0681_amd import JUNCTION_DTYPE
    from paper_1304_0681_amd.splice import write_bed
    j = np.array([(500, 900, 3, 1), (100, 250, 7, 0), (100, 180, 1, 0)], JUNCTION_DTYPE)
    p = tmp_path / "j.bed"
    write_bed(str(p), j, chrom="chr1")
    rows = [ln.split("\t") for ln in p.read_text().splitlines()]
    assert [(r[0], int(r[1]), int(r[2]), int(r[4]), r[5]) for r in rows] == \
        [("chr1", 100, 180, 1, "+"), ("chr1", 100, 250, 7, "+"), ("chr1", 500, 900, 3, "-")]
    assert len({r[3] for r in rows}) == 3
