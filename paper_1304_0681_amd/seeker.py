"""Candidate windows found on the device: k-mer index, seeds, regions, CALs
(Sec. 2, "Stage C: Region Seeker", "Stage D: CAL Seeker"), then the extension
and joining of stage E (tasks i, ii) into the windows sw_batch_score aligns.

KmerIndex builds the exact k-mer index of a packed reference once
(sw_kmer_index_build); CandidateSeeker turns the reads of a DeviceBatch into
joined windows with fixed device buffers and no host round trip:

  sw_seed_regions   two-phase seeds of every read, looked up on both strands
  sw_cal_seeker     each read's regions merged into CALs
  sw_join_cals      CALs extended and joined into windows

With stage_b=True the whole-read mapping of stage B (sw_stage_b, at most one
edit, from the same regions) runs between the two seekers, and the reads it
maps get no CALs: as in the paper, only the reads stage B cannot map go on to
stages C-E.

The windows come back as a batch view (`view`) whose pair count stays on the
device, ready for sw_batch_score / sw_best_per_read / sw_batch_traceback.
"""
from __future__ import annotations

import numpy as np

from . import (BMAP_DTYPE, REGION_DTYPE, SW_BMAP_MAX, SW_SEEKER_MAX_CALS, WINDOW_DTYPE,
               DeviceBatch, sw_cal_seeker, sw_join_cals, sw_kmer_index_build, sw_kmer_index_bytes,
               sw_seed_regions, sw_stage_b)

K, STEP, OFFSET, MAX_OCC = 15, 12, 7, 64


class KmerIndex:
    """Exact k-mer index of the batch's reference in one device buffer."""

    def __init__(self, ctx, ref2b, ref_len: int, k: int = K, stream=None):
        import torch
        self.k, self.ref_len = int(k), int(ref_len)
        self.nbytes = sw_kmer_index_bytes(ref_len, k)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        sw_kmer_index_build(ctx, ref2b, ref_len, k, self.buf, self.nbytes, stream)

    def arrays(self):
        """(starts[4^k + 1], positions) as device int32 views."""
        import torch
        n_codes = 4 ** self.k + 1
        off = (4 * n_codes + 255) & ~255
        n_pos = max(self.ref_len - self.k + 1, 0)
        return (self.buf[:4 * n_codes].view(torch.int32),
                self.buf[off:off + 4 * n_pos].view(torch.int32))


class CandidateSeeker:
    """Regions, CALs and joined windows for the reads of `db`.

    region_cap: regions kept (default 64 per read on average); a read whose
    regions lie beyond it gets CALs from those below it only."""

    def __init__(self, ctx, db: DeviceBatch, index: KmerIndex, step: int = STEP,
                 offset: int = OFFSET, max_occ: int = MAX_OCC, merge_gap: int = 50,
                 min_len: int = 20, ext: int = 30, max_gap: int = 5000,
                 region_cap: int | None = None, stage_b: bool = False):
        import torch
        self.ctx, self.db, self.index = ctx, db, index
        self.params = (index.k, int(step), int(offset), int(max_occ))
        self.merge_gap, self.min_len = int(merge_gap), int(min_len)
        self.ext, self.max_gap = int(ext), int(max_gap)
        n = db.n_reads
        self.n_reads = n
        self.cap = int(region_cap if region_cap is not None else 64 * max(n, 1))
        dev = "cuda"
        self.regions = torch.empty(max(self.cap, 1) * 8, dtype=torch.uint8, device=dev)
        self.read_end = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        self.n_cals = n * SW_SEEKER_MAX_CALS
        self.cals = torch.empty(max(self.n_cals, 1) * 16, dtype=torch.uint8, device=dev)
        self.win = torch.empty(max(self.n_cals, 1) * 12, dtype=torch.uint8, device=dev)
        self.n_win = torch.zeros(1, dtype=torch.int32, device=dev)
        self.view = db.view(self.win, max(self.n_cals, 1), self.n_win)
        self.stage_b = bool(stage_b)
        self.maps = self.n_maps = None
        if self.stage_b:
            self.maps = torch.empty(max(n, 1) * SW_BMAP_MAX * 16, dtype=torch.uint8, device=dev)
            self.n_maps = torch.empty(max(n, 1), dtype=torch.int32, device=dev)

    def run_regions(self, stream=None):
        sw_seed_regions(self.ctx, self.db, self.index.buf, self.params, self.regions, self.cap,
                        self.read_end, stream)

    def run_stage_b(self, stream=None):
        sw_stage_b(self.ctx, self.db, self.regions, self.read_end, self.cap, self.maps,
                   self.n_maps, stream)

    def run_cals(self, stream=None):
        sw_cal_seeker(self.ctx, self.regions, self.read_end, self.n_reads, self.cap, self.index.k,
                      self.merge_gap, self.min_len, self.cals, stream,
                      d_skip=self.n_maps if self.stage_b else None)

    def run_join(self, stream=None):
        sw_join_cals(self.ctx, self.cals, self.n_cals, self.n_reads, self.db.ref_len, self.ext,
                     self.max_gap, self.win, self.n_win, stream)

    def run(self, stream=None):
        self.run_regions(stream)
        if self.stage_b:
            self.run_stage_b(stream)
        self.run_cals(stream)
        self.run_join(stream)

    def stage_b_maps(self):
        """(records[n_reads, SW_BMAP_MAX], counts) of the last run (host copies)."""
        n = self.n_reads
        recs = self.maps.cpu().numpy().view(BMAP_DTYPE)[:n * SW_BMAP_MAX].reshape(n, SW_BMAP_MAX)
        return recs.copy(), self.n_maps.cpu().numpy().view(np.uint32)[:n].copy()

    def region_list(self):
        """(regions, read_end) of the last run (host copies)."""
        end = self.read_end.cpu().numpy().view(np.uint64)[:self.n_reads]
        n = int(min(end[-1], self.cap)) if self.n_reads else 0
        return self.regions.cpu().numpy().view(REGION_DTYPE)[:n].copy(), end.copy()

    def windows(self) -> np.ndarray:
        n = int(self.n_win.item())
        return self.win.cpu().numpy().view(WINDOW_DTYPE)[:n].copy()
