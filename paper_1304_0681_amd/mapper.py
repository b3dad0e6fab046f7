"""Short-read mapping through every device stage (Sec. 2, stages B-E).

ShortReadMapper takes a batch of reads and the k-mer index of its reference and
runs, with fixed device buffers and no host round trip:

  stage B    whole-read mapping with at most one edit (sw_stage_b), from the
             reads' exact seed regions (sw_seed_regions)
  stages C-D the reads stage B did not map: their regions merged into CALs
             (sw_cal_seeker), extended and joined into windows (sw_join_cals)
  stage E    SW of those reads against their windows, the best window per read
             and its alignment with CIGAR (AlignPass with the band of the best
             hit)

results() merges the two sources into one record per read: the stage B
record (the first of its best stratum, with the CIGAR of its one edit) or the
SW alignment of the best window, or unmapped.
"""
from __future__ import annotations

import numpy as np

from . import SW_OP_D, SW_OP_I, SW_OP_M, DeviceBatch
from .pipeline import AlignPass
from .seeker import CandidateSeeker

SCORING = (5, -4, -10, -1)

# where a read's record comes from
UNMAPPED, STAGE_B, STAGE_E = 0, 1, 2

RECORD_DTYPE = np.dtype([("source", "u1"), ("strand", "u1"), ("n_records", "u1"),
                         ("edits", "i1"), ("score", "<i4"), ("ref_begin", "<i8"),
                         ("ref_end", "<i8"), ("read_begin", "<i4"), ("read_end", "<i4")])


def _stage_b_cigar(m: int, op: int, pos: int) -> list[int]:
    """CIGAR ops ((len << 4) | code) of a stage B record of an m-base read."""
    if op == 2:                       # deletion before query base pos
        return [(pos << 4) | SW_OP_M, (1 << 4) | SW_OP_D, ((m - pos) << 4) | SW_OP_M]
    if op == 3:                       # query base pos inserted
        return [(pos << 4) | SW_OP_M, (1 << 4) | SW_OP_I, ((m - pos - 1) << 4) | SW_OP_M]
    return [(m << 4) | SW_OP_M]       # exact or one substitution


class ShortReadMapper:
    """`db`: the reads and the reference (its own windows are not used);
    `index`: KmerIndex of that reference.  `t_map`: the SW score a best window
    must reach for the read to count as mapped by stage E."""

    def __init__(self, ctx, db: DeviceBatch, index, scoring=SCORING, t_map: int = 200,
                 max_occ: int = 64, merge_gap: int = 50, min_len: int = 20, ext: int = 30,
                 max_gap: int = 5000, ops_stride: int = 64):
        self.ctx, self.db, self.t_map = ctx, db, int(t_map)
        self.seeker = CandidateSeeker(ctx, db, index, max_occ=max_occ, merge_gap=merge_gap,
                                      min_len=min_len, ext=ext, max_gap=max_gap, stage_b=True)
        self.align = AlignPass(ctx, self.seeker.view, scoring, t_map=self.t_map,
                               ops_stride=ops_stride, band=True)

    def run(self, stream=None):
        """Stages B-E for every read (the reads are already encoded)."""
        self.seeker.run(stream)
        self.align.run(stream, pack=False)

    def results(self):
        """(records, cigars): one RECORD_DTYPE row per read, and each read's CIGAR
        ops (a list per read; stage E CIGARs include soft clips)."""
        n = self.db.n_reads
        maps, n_maps = self.seeker.stage_b_maps()
        bp, bs, aln, ops = self.align.results()
        win = self.seeker.windows()
        m = self.db.read_len.cpu().numpy().view(np.uint16).astype(np.int64)[:n]
        rec = np.zeros(n, RECORD_DTYPE)
        rec["score"] = -1
        rec["ref_begin"] = rec["ref_end"] = -1
        rec["read_begin"] = rec["read_end"] = -1
        rec["edits"] = -1
        cigars: list[list[int]] = [[] for _ in range(n)]
        for r in range(n):
            k = int(n_maps[r])
            if k:
                x = maps[r, 0]
                rec[r] = (STAGE_B, int(x["strand"]), k, int(x["edits"]), -1, int(x["first"]),
                          int(x["last"]), 0, int(m[r]) - 1)
                cigars[r] = _stage_b_cigar(int(m[r]), int(x["op"]), int(x["edit_pos"]))
            elif (bp[r] != 0xFFFFFFFF and int(bs[r]) >= self.t_map
                  and (int(aln["status"][r]) & ~1) == 0):
                # (status bit 0: CIGAR cut at ops_stride; the coordinates stand)
                w = win[bp[r]]
                a = aln[r]
                rec[r] = (STAGE_E, int(w["strand"]), 1, -1, int(a["score"]),
                          int(w["ref_begin"]) + int(a["ref_begin"]),
                          int(w["ref_begin"]) + int(a["ref_end"]), int(a["read_begin"]),
                          int(a["read_end"]))
                cigars[r] = [int(o) for o in ops[r, :int(a["n_ops"])]]
        return rec, cigars


def cigar_string(ops) -> str:
    """'12M1D88M'-style text of CIGAR ops."""
    letters = "MIDNS"
    return "".join(f"{int(o) >> 4}{letters[int(o) & 15]}" for o in ops)


__all__ = ["ShortReadMapper", "RECORD_DTYPE", "UNMAPPED", "STAGE_B", "STAGE_E", "cigar_string"]
