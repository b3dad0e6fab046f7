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
               sw_best_per_read, sw_graph_begin, sw_graph_destroy, sw_graph_end, sw_graph_launch,
               sw_merge_best, sw_select_windows, sw_sole_windows)

SCORING = (5, -4, -10, -1)


class BestBandTraceback:
    """Traceback of each read's best window over its band.

    The best window of every read (ids from sw_best_per_read) is copied into a
    window list of its own (sw_select_windows), those windows are scored again
    with their end cells (SW_WANT_ENDS: one pass over one window per read), and
    the traceback's DP then covers only the columns each best alignment can
    reach (sw_batch_traceback with the hits).  Results equal the traceback of the
    best pairs over their whole windows; the output rows are the reads.  Fixed
    device buffers, so a pass can be captured in a graph."""

    def __init__(self, ctx, db: DeviceBatch, n_reads: int, scoring=SCORING):
        import torch
        self.ctx, self.scoring, self.n_reads = ctx, scoring, int(n_reads)
        self.win = torch.empty(self.n_reads * 12, dtype=torch.uint8, device="cuda")
        self.hits = torch.empty((self.n_reads, 3), dtype=torch.int32, device="cuda")
        self.ids = torch.arange(self.n_reads, dtype=torch.int32, device="cuda")
        self.view = db.view(self.win, self.n_reads)

    def run(self, batch, best_pair, aln, ops, ops_stride, stream=None):
        """`batch`: the batch (or view) best_pair indexes into."""
        sw_select_windows(self.ctx, batch, best_pair, self.n_reads, self.win, stream)
        sw_batch_score(self.ctx, self.view, self.scoring, SW_WANT_ENDS, self.hits, stream)
        sw_batch_traceback(self.ctx, self.view, self.scoring, self.ids, self.n_reads, aln, ops,
                           ops_stride, stream, hits=self.hits)


class AlignPass:
    """`band`: trace back each read's best window over its band (BestBandTraceback:
    the best windows are scored again with their end cells, then the traceback's
    DP covers only the columns each alignment can reach); same results.

    `sole_first` (with `band`): a read with one window takes it without the
    first score pass (sw_sole_windows); only the windows of reads with several
    are scored, and their best merged in (sw_merge_best).  The rescoring of the
    best windows gives every read's best score, so results are unchanged; `hits`
    then holds the scores of the compacted list and `mapped` is not kept."""

    def __init__(self, ctx, db: DeviceBatch, scoring=SCORING, t_map: int = 0,
                 ops_stride: int | None = None, band: bool = False, sole_first: bool = False):
        import torch
        self.ctx, self.db, self.scoring, self.t_map = ctx, db, scoring, int(t_map)
        self.band = bool(band)
        if sole_first and not band:
            raise ValueError("sole_first takes the best scores from the band's rescoring")
        self.sole_first = bool(sole_first)
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
        self.bbt = BestBandTraceback(ctx, db, n_reads, scoring) if self.band else None
        if self.sole_first:
            self.sole = torch.empty(max(n_reads, 1), dtype=torch.int32, device=dev)
            self.multi_win = torch.empty(max(n_pairs, 1) * 12, dtype=torch.uint8, device=dev)
            self.multi_ids = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
            self.n_multi = torch.zeros(1, dtype=torch.int32, device=dev)
            self.multi_view = db.view(self.multi_win, n_pairs, self.n_multi)
            self.multi_best = torch.empty(max(n_reads, 1), dtype=torch.int32, device=dev)
        self.graph = None

    def run(self, stream=None, pack=True):
        """Encode (optional), score, best hit per read, traceback of the best hits."""
        if pack:
            self.db.pack_reads(stream)
        if self.sole_first:
            db, n = self.db, self.db.n_reads
            sw_sole_windows(self.ctx, db, self.sole, self.multi_win, self.multi_ids, self.n_multi,
                            stream)
            sw_batch_score(self.ctx, self.multi_view, self.scoring, 0, self.hits, stream)
            sw_best_per_read(self.ctx, self.multi_view, self.hits, self.t_map, self.multi_best,
                             self.best_score, self.mapped, stream)
            sw_merge_best(self.ctx, n, self.sole, self.multi_best, self.multi_ids, db.n_pairs,
                          self.best_pair, stream)
        else:
            sw_batch_score(self.ctx, self.db, self.scoring, 0, self.hits, stream)
            sw_best_per_read(self.ctx, self.db, self.hits, self.t_map, self.best_pair,
                             self.best_score, self.mapped, stream)
        if self.bbt is not None:
            self.bbt.run(self.db, self.best_pair, self.aln, self.ops, self.ops_stride, stream)
        else:
            sw_batch_traceback(self.ctx, self.db, self.scoring, self.best_pair, self.db.n_reads,
                               self.aln, self.ops, self.ops_stride, stream)

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
        bs = self.best_score.cpu().numpy()
        if self.sole_first:     # the rescoring of each read's best window has its score
            bs = self.bbt.hits[:, 0].cpu().numpy().copy()
        return (self.best_pair.cpu().numpy().view(np.uint32), bs, aln_to_numpy(self.aln),
                self.ops.cpu().numpy().view(np.uint32))
