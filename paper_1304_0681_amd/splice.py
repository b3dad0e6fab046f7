"""Spliced long reads on the device: seeds, CALs, joined windows, whole-read
alignment and splice junctions (Sec. 2, "Stage E: SWA + Splice Junctions").

SplicedPass runs, for one batch of long reads and their seeds, with fixed
device buffers and no host round trip:

  seeds      every seed against its candidate windows (sw_batch_score), the
             best window per seed (sw_best_per_read) and its alignment
             (sw_batch_traceback over the band of the best hit)
  CALs       the reference span of each seed's best alignment scoring at least
             min_seed_score (sw_seed_cals)
  joining    CALs extended by `ext` and joined within `max_gap` (the longest
             intron) into windows of the long reads (sw_join_cals, tasks i, ii)
  alignment  every long read against its joined windows (sw_batch_score with
             a gap extension of 0, so that an intron costs one gap open), the
             best window per read and its alignment (task iii); a read with
             one joined window (most of them) skips the score pass
             (sw_sole_windows, sw_merge_best)
  junctions  deletion runs of at least min_intron bases with an intron motif
             become N ops and are counted in a device hash table that
             accumulates over batches (sw_detect_junctions, task iv)

SeekerSplicedPass finds the seeds' candidate windows on the device first
(regions, CALs and joining of the seeds: stages C and D), so that nothing but
the reads and the reference enters the pass.

The junction table is read out with junctions() (sorted) and written as BED
with write_bed().
"""
from __future__ import annotations

import numpy as np

from . import (SW_OPT_TB_SCRATCH_MB, SW_WANT_ENDS, DeviceBatch, _ptr, aln_to_numpy,
               sw_batch_score, sw_batch_traceback, sw_best_per_read, sw_ctx_set_option,
               sw_detect_junctions, sw_join_cals, sw_junctions_clear, sw_list_junctions,
               sw_merge_best, sw_seed_cals, sw_sole_windows, junctions_to_numpy)
from .pipeline import AlignPass

SEED_SCORING = (5, -4, -10, -1)
LONG_SCORING = (5, -4, -20, 0)


class SplicedPass:
    """`seed_db`: the seeds with their candidate windows; `seed_read[s]`: the long
    read of seed s (seeds of one read contiguous); `long_db`: the long reads
    (its own windows are not used).  `tb_scratch_mb`: traceback scratch of the
    context (the whole-read alignments cover windows of several kb)."""

    def __init__(self, ctx, seed_db: DeviceBatch, seed_read, long_db: DeviceBatch,
                 seed_scoring=SEED_SCORING, long_scoring=LONG_SCORING, min_seed_score: int = 100,
                 ext: int = 30, max_gap: int = 5000, min_score: int = 100, min_intron: int = 40,
                 table_capacity: int = 1 << 20, ops_stride: int = 256,
                 tb_scratch_mb: int | None = 16384, seed_ops_stride: int | None = None):
        import torch
        self.ctx, self.seed_db, self.long_db = ctx, seed_db, long_db
        self.long_scoring = long_scoring
        self.min_seed_score, self.ext, self.max_gap = int(min_seed_score), int(ext), int(max_gap)
        self.min_score, self.min_intron = int(min_score), int(min_intron)
        self.capacity = int(table_capacity)
        self.ops_stride = int(ops_stride)
        if tb_scratch_mb is not None:
            sw_ctx_set_option(ctx, SW_OPT_TB_SCRATCH_MB, tb_scratch_mb)
        dev = "cuda"
        n_seeds, n_long = seed_db.n_reads, long_db.n_reads
        self.n_seeds, self.n_long = n_seeds, n_long
        # (a seed's CAL reads its alignment's span only, so truncated seed CIGARs
        # change nothing downstream)
        self.seeds = AlignPass(ctx, seed_db, seed_scoring, band=True, ops_stride=seed_ops_stride)
        sr = np.ascontiguousarray(seed_read, dtype=np.uint32)
        assert len(sr) == n_seeds
        self.seed_read = torch.from_numpy(sr.view(np.int32)).to(dev)
        self.cals = torch.empty(max(n_seeds, 1) * 16, dtype=torch.uint8, device=dev)
        # at most one window per CAL
        self.win = torch.empty(max(n_seeds, 1) * 12, dtype=torch.uint8, device=dev)
        self.n_win = torch.zeros(1, dtype=torch.int32, device=dev)
        self.long_view = long_db.view(self.win, n_seeds, self.n_win)
        self.hits = torch.empty((max(n_seeds, 1), 3), dtype=torch.int32, device=dev)
        # reads with one joined window go straight to the traceback; the windows
        # of the others are scored to pick each read's best
        self.sole = torch.empty(max(n_long, 1), dtype=torch.int32, device=dev)
        self.multi_win = torch.empty(max(n_seeds, 1) * 12, dtype=torch.uint8, device=dev)
        self.multi_ids = torch.empty(max(n_seeds, 1), dtype=torch.int32, device=dev)
        self.n_multi = torch.zeros(1, dtype=torch.int32, device=dev)
        self.multi_view = long_db.view(self.multi_win, n_seeds, self.n_multi)
        self.multi_best = torch.empty(n_long, dtype=torch.int32, device=dev)
        self.best_pair = torch.empty(n_long, dtype=torch.int32, device=dev)
        self.best_score = torch.empty(n_long, dtype=torch.int32, device=dev)
        self.aln = torch.empty((n_long, 7), dtype=torch.int32, device=dev)
        self.ops = torch.empty((n_long, self.ops_stride), dtype=torch.int32, device=dev)
        self.n_junc = torch.empty(n_long, dtype=torch.int32, device=dev)
        self.dropped = torch.zeros(1, dtype=torch.int32, device=dev)
        self.keys = torch.empty(self.capacity, dtype=torch.int64, device=dev)
        self.counts = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.clear()

    def clear(self, stream=None):
        """Empty the junction table (counts accumulate over run() calls)."""
        sw_junctions_clear(self.ctx, self.keys, self.counts, self.capacity, stream)
        self.dropped.zero_()

    def run_seeds(self, stream=None):
        self.seeds.run(stream)

    def run_cals(self, stream=None):
        sw_seed_cals(self.ctx, self.seed_db, self.seeds.best_pair, self.seeds.aln, self.seed_read,
                     self.n_seeds, self.min_seed_score, self.cals, stream)
        sw_join_cals(self.ctx, self.cals, self.n_seeds, self.n_long, self.long_db.ref_len,
                     self.ext, self.max_gap, self.win, self.n_win, stream)

    def run_long_best(self, stream=None):
        """Best joined window of every read.  A read with one window has it
        (the traceback then finds its score); the windows of the others are
        scored and their best merged in."""
        sw_sole_windows(self.ctx, self.long_view, self.sole, self.multi_win, self.multi_ids,
                        self.n_multi, stream)
        sw_batch_score(self.ctx, self.multi_view, self.long_scoring, 0, self.hits, stream)
        sw_best_per_read(self.ctx, self.multi_view, self.hits, self.min_score, self.multi_best,
                         self.best_score, None, stream)
        sw_merge_best(self.ctx, self.n_long, self.sole, self.multi_best, self.multi_ids,
                      self.n_seeds, self.best_pair, stream)

    def run_long_traceback(self, stream=None):
        sw_batch_traceback(self.ctx, self.long_view, self.long_scoring, self.best_pair,
                           self.n_long, self.aln, self.ops, self.ops_stride, stream)

    def run_long(self, stream=None):
        self.run_long_best(stream)
        self.run_long_traceback(stream)

    def run_junctions(self, stream=None):
        sw_detect_junctions(self.ctx, self.long_view, self.best_pair, self.n_long, self.aln,
                            self.ops, self.ops_stride, self.min_score, self.min_intron, self.keys,
                            self.counts, self.capacity, self.n_junc, self.dropped, stream)

    def run(self, stream=None):
        self.run_seeds(stream)
        self.run_cals(stream)
        self.run_long(stream)
        self.run_junctions(stream)

    def windows(self) -> np.ndarray:
        """The joined windows of the last run (host copy)."""
        from . import WINDOW_DTYPE
        n = int(self.n_win.item())
        return self.win.cpu().numpy().view(WINDOW_DTYPE)[:n].copy()

    def junctions(self, stream=None) -> np.ndarray:
        """The table's junctions sorted by (start, end, strand) (host copy)."""
        import torch
        out = torch.empty(self.capacity * 24, dtype=torch.uint8, device="cuda")
        n = torch.zeros(1, dtype=torch.int32, device="cuda")
        sw_list_junctions(self.ctx, self.keys, self.counts, self.capacity, out, self.capacity, n,
                          stream)
        torch.cuda.synchronize()
        j = junctions_to_numpy(out)[:int(n.item())]
        return np.sort(j, order=("start", "end", "strand"))

    def results(self):
        """(best_pair, best_score, aln, ops, junctions per read) of the long reads
        (a read with one window has its alignment's score as best score)."""
        aln = aln_to_numpy(self.aln)
        bs = self.best_score.cpu().numpy()
        sole = self.sole.cpu().numpy()[:self.n_long] != -1
        bs[sole] = aln["score"][sole]
        return (self.best_pair.cpu().numpy().view(np.uint32), bs, aln,
                self.ops.cpu().numpy().view(np.uint32), self.n_junc.cpu().numpy().view(np.uint32))


class SeekerSplicedPass(SplicedPass):
    """SplicedPass with the seeds' candidate windows found on the device: the
    seeds' regions, CALs and joined windows (CandidateSeeker: stages C and D,
    then stage E tasks i and ii on the seeds) run ahead of the seed alignment,
    so the reads and the reference are the whole input.

    `seed_db`: the seeds (its own windows are not used); `index`: the k-mer
    index of the reference (KmerIndex); max_occ, merge_gap and min_len are the
    seeker's, seed_ext and seed_max_gap the joining of a seed's CALs (a seed
    that crosses an intron has a CAL on each side).  The remaining arguments
    are SplicedPass's."""

    def __init__(self, ctx, seed_db: DeviceBatch, index, seed_read, long_db: DeviceBatch,
                 max_occ: int = 64, merge_gap: int = 50, min_len: int = 20, seed_ext: int = 30,
                 seed_max_gap: int = 5000, seed_ops_stride: int = 64, **kw):
        from .seeker import CandidateSeeker
        self.seeker = CandidateSeeker(ctx, seed_db, index, max_occ=max_occ, merge_gap=merge_gap,
                                      min_len=min_len, ext=seed_ext, max_gap=seed_max_gap)
        super().__init__(ctx, self.seeker.view, seed_read, long_db,
                         seed_ops_stride=seed_ops_stride, **kw)

    def run_seeker(self, stream=None):
        self.seeker.run(stream)

    def run(self, stream=None):
        self.run_seeker(stream)
        super().run(stream)


def write_bed(path: str, junctions: np.ndarray, chrom: str = "ref") -> None:
    """Junctions as BED lines (chrom, start, end, name, score = count, strand),
    sorted by position; the paper writes its junction list in this format."""
    j = np.sort(junctions, order=("start", "end", "strand"))
    with open(path, "w") as f:
        for k, r in enumerate(j):
            f.write(f"{chrom}\t{int(r['start'])}\t{int(r['end'])}\tJ{k:08d}\t{int(r['count'])}\t"
                    f"{'+' if int(r['strand']) == 0 else '-'}\n")
