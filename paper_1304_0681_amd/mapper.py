"""Short-read mapping through every device stage (Sec. 2, stages B-E).

ShortReadMapper takes a batch of reads and the k-mer index of its reference and
runs, with fixed device buffers and no host round trip:

  stage B    whole-read mapping with at most one edit (sw_stage_b), from the
             reads' exact seed regions (sw_seed_regions)
  stages C-D the reads stage B did not map: their regions merged into CALs
             (sw_cal_seeker), extended and joined into windows (sw_join_cals)
  stage E    SW of those reads against their windows, the best window per read
             and its alignment with CIGAR (AlignPass with the band of the best
             hit; a read with one window takes it without the score pass)

results() merges the two sources into one record per read (arrays, no
per-read host loop): the stage B record (the first of its best stratum, with
the CIGAR of its one edit) or the SW alignment of the best window, or
unmapped.
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
                               ops_stride=ops_stride, band=True, sole_first=True)

    def run(self, stream=None):
        """Stages B-E for every read (the reads are already encoded)."""
        self.seeker.run(stream)
        self.align.run(stream, pack=False)

    def results(self):
        """(records, ops, n_ops): one RECORD_DTYPE row per read, and its CIGAR ops
        ((length << 4) | code, ops[r, :n_ops[r]]; stage E CIGARs include soft
        clips and stop at ops_stride ops)."""
        n = self.db.n_reads
        maps, n_maps = self.seeker.stage_b_maps()
        bp, bs, aln, ops = self.align.results()
        win = self.seeker.windows()
        m = self.db.read_len.cpu().numpy().view(np.uint16).astype(np.int64)[:n]
        rec = np.zeros(n, RECORD_DTYPE)
        for f, v in (("score", -1), ("ref_begin", -1), ("ref_end", -1), ("read_begin", -1),
                     ("read_end", -1), ("edits", -1)):
            rec[f] = v
        out = np.zeros((n, ops.shape[1]), np.uint32)
        n_ops = np.zeros(n, np.int64)
        # stage B: the first record of the best stratum, the CIGAR of its one edit
        isb = n_maps > 0
        x = maps[:, 0]
        rec["source"][isb] = STAGE_B
        rec["strand"][isb] = x["strand"][isb]
        rec["n_records"][isb] = n_maps[isb]
        rec["edits"][isb] = x["edits"][isb]
        rec["ref_begin"][isb] = x["first"][isb]
        rec["ref_end"][isb] = x["last"][isb]
        rec["read_begin"][isb] = 0
        rec["read_end"][isb] = m[isb] - 1
        op, pos = x["op"].astype(np.int64), x["edit_pos"].astype(np.int64)
        gap = isb & ((op == 2) | (op == 3))
        code = np.where(op == 2, SW_OP_D, SW_OP_I)
        tail = np.where(op == 2, m - pos, m - pos - 1)
        plain = isb & ~gap
        out[plain, 0] = (m[plain] << 4) | SW_OP_M
        n_ops[plain] = 1
        out[gap, 0] = (pos[gap] << 4) | SW_OP_M
        out[gap, 1] = (1 << 4) | code[gap]
        out[gap, 2] = (tail[gap] << 4) | SW_OP_M
        n_ops[gap] = 3
        # stage E: the best window's alignment (status bit 0: CIGAR cut at
        # ops_stride; the coordinates stand)
        ise = (~isb & (bp != 0xFFFFFFFF) & (bs >= self.t_map)
               & ((aln["status"].astype(np.int64) & ~1) == 0))
        w = win[bp[ise]]
        a = aln[ise]
        rec["source"][ise] = STAGE_E
        rec["strand"][ise] = w["strand"]
        rec["n_records"][ise] = 1
        rec["score"][ise] = a["score"]
        rec["ref_begin"][ise] = w["ref_begin"].astype(np.int64) + a["ref_begin"]
        rec["ref_end"][ise] = w["ref_begin"].astype(np.int64) + a["ref_end"]
        rec["read_begin"][ise] = a["read_begin"]
        rec["read_end"][ise] = a["read_end"]
        out[ise] = ops[ise]
        n_ops[ise] = a["n_ops"]
        return rec, out, n_ops


def write_sam(path: str, rec: np.ndarray, ops: np.ndarray, n_ops: np.ndarray, reads: np.ndarray,
              read_off: np.ndarray, read_len: np.ndarray, ref_len: int, chrom: str = "ref",
              names=None) -> None:
    """Mapper records as SAM text (one line per read, in read order): flag 16 for
    the reverse strand (SEQ then holds the reverse complement, as aligned), 4
    for unmapped reads; POS is 1-based; AS:i carries the SW score, NM:i the
    edits of a stage B record; MAPQ is 255 (not computed).  reads / read_off /
    read_len: the batch's ASCII reads."""
    comp = bytes.maketrans(b"ACGTacgtN", b"TGCAtgcaN")
    with open(path, "w") as f:
        f.write(f"@HD\tVN:1.6\tSO:unsorted\n@SQ\tSN:{chrom}\tLN:{int(ref_len)}\n"
                f"@PG\tID:hpgsw\tPN:paper_1304_0681_amd\n")
        for r in range(len(rec)):
            x = rec[r]
            o, m = int(read_off[r]), int(read_len[r])
            seq = bytes(reads[o:o + m])
            name = names[r] if names is not None else f"r{r}"
            if int(x["source"]) == UNMAPPED:
                f.write(f"{name}\t4\t*\t0\t0\t*\t*\t0\t0\t{seq.decode()}\t*\n")
                continue
            rev = int(x["strand"]) == 1
            if rev:
                seq = seq.translate(comp)[::-1]
            tag = (f"AS:i:{int(x['score'])}" if int(x["source"]) == STAGE_E
                   else f"NM:i:{int(x['edits'])}")
            f.write(f"{name}\t{16 if rev else 0}\t{chrom}\t{int(x['ref_begin']) + 1}\t255\t"
                    f"{cigar_string(ops[r, :int(n_ops[r])])}\t*\t0\t0\t{seq.decode()}\t*\t{tag}\n")


def cigar_string(ops) -> str:
    """'12M1D88M'-style text of CIGAR ops."""
    letters = "MIDNS"
    return "".join(f"{int(o) >> 4}{letters[int(o) & 15]}" for o in ops)


__all__ = ["ShortReadMapper", "RECORD_DTYPE", "UNMAPPED", "STAGE_B", "STAGE_E", "cigar_string",
           "write_sam"]
