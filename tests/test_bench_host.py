"""bench.py's host-side contract, checked without a GPU: more than one GPU is
refused with a message (this build measures one GPU), and the stream's chunk
generators start, take their work later, and return chunks of the requested
shape."""
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stream_chunk_generation(tmp_path):
    code = (
        "import sys, types\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import bench\n"
        "if __name__ == '__main__':\n"
        "    a = types.SimpleNamespace(stream_distinct=3, stream_chunks=5, stream_frags=500)\n"
        "    w = bench.start_stream_workers(a)\n"
        "    ex, futs = bench.generate_stream_chunks(w, a)\n"
        "    out = [f.result() for f in futs]\n"
        "    ex.shutdown()\n"
        "    assert len(out) == 3\n"
        "    for reads, off, ln, win in out:\n"
        "        assert len(ln) == 1000 and (ln == 150).all() and len(win) == 16 * 1000\n"
        "        assert len(reads) == int(off[-1]) + int(ln[-1])\n"
        "    print('ok')\n")
    path = tmp_path / "gen_check.py"     # a script: the spawned workers import it as main
    path.write_text(code)
    r = subprocess.run([sys.executable, str(path)], capture_output=True, text=True, timeout=300,
                       cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")
