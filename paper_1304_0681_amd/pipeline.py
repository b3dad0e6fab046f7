"""One alignment pass over a batch with fixed device buffers.

Stage E of the paper aligns a read (or a split-read seed, stage D) against all
of its candidate windows, keeps the best-scoring one and reports its
alignment (Sec. 2, "Stage E", tasks iii and iv).  AlignPass runs that on the
device: sw_pack2b of the reads, sw_batch_score over every pair, sw_best_per_read
and sw_batch_traceback of the best pair of every read.  The same sequence can
be recorded once as a graph (sw_graph_*) and replayed on new inputs copied into
the same buffers, so a chunk costs one launch.
"""
from __future__ import annotations

import numpy as np

from . import (SW_WANT_ENDS, DeviceBatch, aln_to_numpy, sw_batch_score, sw_batch_traceback,
               sw_best_per_read, sw_graph_begin, sw_graph_destroy, sw_graph_end, sw_graph_launch)

SCORING = (5, -4, -10, -1)


class AlignPass:
    """`band`: score with end cells and let the traceback's DP cover only the
    columns each best alignment can reach (same results; pays where the reads
    score on the int32 path, i.e. reads longer than 100 nt)."""

    def __init__(self, ctx, db: DeviceBatch, scoring=SCORING, t_map: int = 0,
                 ops_stride: int | None = None, band: bool = False):
        import torch
        self.ctx, self.db, self.scoring, self.t_map = ctx, db, scoring, int(t_map)
        self.band = bool(band)
        n_pairs, n_reads = db.n_pairs, db.n_reads
        if ops_stride is None:       # m + n + 2 ops always suffice
            ops_stride = db.read_len_max + db.window_len_max + 2
        self.ops_stride = int(ops_stride)
        dev = "cuda"
        self.hits = torch.empty((n_pairs, 3), dtype=torch.int32, device=dev)
        self.best_pair = torch.empty(n_reads, dtype=torch.int32, device=dev)
        self.best_score = torch.empty(n_reads, dtype=torch.int32, device=dev)
        self.mapped = torch.empty(n_reads, dtype=torch.uint8, device=dev)
        self.aln = torch.empty((n_reads, 7), dtype=torch.int32, device=dev)
        self.ops = torch.empty((n_reads, self.ops_stride), dtype=torch.int32, device=dev)
        self.graph = None

    def run(self, stream=None, pack=True):
        """Encode (optional), score, best hit per read, traceback of the best hits."""
        if pack:
            self.db.pack_reads(stream)
        sw_batch_score(self.ctx, self.db, self.scoring, SW_WANT_ENDS if self.band else 0, self.hits,
                       stream)
        sw_best_per_read(self.ctx, self.db, self.hits, self.t_map, self.best_pair, self.best_score,
                         self.mapped, stream)
        sw_batch_traceback(self.ctx, self.db, self.scoring, self.best_pair, self.db.n_reads,
                           self.aln, self.ops, self.ops_stride, stream,
                           hits=self.hits if self.band else None)

    def capture(self, stream, pack=True):
        """Record run() as a graph on `stream` (a created torch.cuda.Stream).  One
        eager run first sizes every scratch buffer."""
        import torch
        with torch.cuda.stream(stream):
            self.run(stream, pack)
        stream.synchronize()
        sw_graph_begin(self.ctx, stream)
        try:
            self.run(stream, pack)
        finally:
            g = sw_graph_end(self.ctx, stream)
        if self.graph is not None:
            sw_graph_destroy(self.ctx, self.graph)
        self.graph = g

    def replay(self, stream):
        sw_graph_launch(self.ctx, self.graph, stream)

    def close(self):
        if self.graph is not None:
            sw_graph_destroy(self.ctx, self.graph)
            self.graph = None

    def results(self):
        """(best_pair, best_score, aln, ops) as numpy arrays."""
        return (self.best_pair.cpu().numpy().view(np.uint32), self.best_score.cpu().numpy(),
                aln_to_numpy(self.aln), self.ops.cpu().numpy().view(np.uint32))
