"""Streaming of read chunks through the filtered alignment path on one GPU.

The paper's pipeline moves reads through its stages in batches, with stages
overlapping each other (Sec. 3, the batch queues between stages).  Here a chunk
of reads (with all of their candidate windows) is one batch.  Each chunk is:

  host -> device copy of the reads, read offsets/lengths and windows
  encode (sw_pack2b), learned filter (sw_filter_candidates: features, MLP,
  per-read decision, compaction), SW on the kept pairs (sw_batch_score), best
  hit per read (sw_best_per_read with the mapping threshold), traceback of the
  best hit (sw_batch_traceback)
  device -> host copy of the per-read results

Two device buffer sets and three streams (host-to-device copies, compute,
device-to-host copies) overlap the copies of chunks i + 1 and i - 1 with the
compute of chunk i.  The results of chunk i - 1 are copied out once chunk i has
passed its filter stage, so that those copies (kernels writing to host memory)
run beside the arithmetic-bound scoring instead of the memory-bound filter
kernels they would slow down.  The reference stays resident (packed once); host
buffers are pinned allocations so that the copies are asynchronous.  The overlap
needs the three streams on different hardware queues: the runtime maps streams
onto a few queues per process (GPU_MAX_HW_QUEUES, 4 by default), and in a process
that has created other streams before, two of these can share one, which
serializes copies and compute (results stay the same).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import (ALN_DTYPE, SW_WANT_ENDS, WINDOW_DTYPE, _ptr, sw_batch, sw_batch_score,
               sw_batch_traceback, sw_best_per_read, sw_filter_candidates, sw_pack2b)

SCORING = (5, -4, -10, -1)


class ChunkManifest:
    """Which chunks of a stream have been handed out, kept in a JSON file so
    that a stopped run (a failure, a kill) resumes where it stopped.

    The file holds the run's identity (`key`, any JSON value the caller picks,
    e.g. the input file names and chunk size), the number of chunks and the
    sorted indices of the chunks whose results the consumer has received.  It
    is rewritten after every chunk through a temporary file and an atomic
    rename, so it is always either the old or the new record.  A chunk is
    marked after its consumer returns: a run that stops between the two hands
    that one chunk out again on resume (at least once), so a consumer should
    treat a repeated chunk index as a replacement.  Opening an existing file of
    another run (other key or chunk count) raises ValueError."""

    def __init__(self, path: str, n_chunks: int, key=None):
        self.path, self.n_chunks, self.key = path, int(n_chunks), key
        self.done: set[int] = set()
        if os.path.exists(path):
            with open(path) as f:
                rec = json.load(f)
            if rec.get("n_chunks") != self.n_chunks or rec.get("key") != key:
                raise ValueError(f"{path} records another run "
                                 f"({rec.get('n_chunks')} chunks, key {rec.get('key')!r})")
            self.done = {int(i) for i in rec.get("done", [])}
        else:
            self._write()

    def pending(self) -> list[int]:
        return [i for i in range(self.n_chunks) if i not in self.done]

    @property
    def complete(self) -> bool:
        return len(self.done) == self.n_chunks

    def mark(self, i: int):
        if not 0 <= i < self.n_chunks:
            raise IndexError(i)
        self.done.add(int(i))
        self._write()

    def _write(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"key": self.key, "n_chunks": self.n_chunks, "done": sorted(self.done)}, f)
            f.flush()
            os.fsync(f.fileno())
        os.replace(tmp, self.path)


class _View:
    """A batch over device buffers (the object the binding functions take)."""

    def __init__(self, c, n_reads, n_pairs):
        self.c, self.n_reads, self.n_pairs = c, n_reads, n_pairs


class HostChunk:
    """One chunk's inputs in pinned host memory."""

    def __init__(self, b):
        import torch
        self.n_reads, self.n_pairs, self.n_bases = b.n_reads, b.n_pairs, len(b.reads)
        self.reads = torch.empty(self.n_bases, dtype=torch.uint8, pin_memory=True)
        self.reads.numpy()[:] = b.reads
        self.read_off = torch.empty(self.n_reads, dtype=torch.int64, pin_memory=True)
        self.read_off.numpy()[:] = b.read_off.view(np.int64)
        self.read_len = torch.empty(self.n_reads, dtype=torch.int16, pin_memory=True)
        self.read_len.numpy()[:] = b.read_len.view(np.int16)
        self.win = torch.empty(self.n_pairs * WINDOW_DTYPE.itemsize, dtype=torch.uint8,
                               pin_memory=True)
        self.win.numpy()[:] = np.ascontiguousarray(b.windows).view(np.uint8)


class _DeviceSet:
    def __init__(self, reads_cap, bases_cap, pairs_cap, ops_stride):
        import torch
        d = "cuda"
        self.reads = torch.empty(bases_cap, dtype=torch.uint8, device=d)
        self.reads2b = torch.empty((bases_cap + 15) // 16, dtype=torch.int32, device=d)
        self.read_off = torch.empty(reads_cap, dtype=torch.int64, device=d)
        self.read_len = torch.empty(reads_cap, dtype=torch.int16, device=d)
        self.win = torch.empty(pairs_cap * WINDOW_DTYPE.itemsize, dtype=torch.uint8, device=d)
        self.bad = torch.zeros(1, dtype=torch.int32, device=d)
        self.feat = torch.empty((pairs_cap, 64), dtype=torch.int16, device=d)
        self.logits = torch.empty(pairs_cap, dtype=torch.float32, device=d)
        self.keep = torch.empty(pairs_cap, dtype=torch.uint8, device=d)
        self.win_out = torch.empty(pairs_cap * WINDOW_DTYPE.itemsize, dtype=torch.uint8, device=d)
        self.sel = torch.empty(pairs_cap, dtype=torch.int32, device=d)
        self.n_sel = torch.zeros(1, dtype=torch.int32, device=d)
        self.n_unsure = torch.zeros(1, dtype=torch.int32, device=d)
        self.hits = torch.empty((pairs_cap, 3), dtype=torch.int32, device=d)
        self.best_pair = torch.empty(reads_cap, dtype=torch.int32, device=d)
        self.best_score = torch.empty(reads_cap, dtype=torch.int32, device=d)
        self.mapped = torch.empty(reads_cap, dtype=torch.uint8, device=d)
        self.aln = torch.empty((reads_cap, 7), dtype=torch.int32, device=d)
        self.ops = torch.empty((reads_cap, ops_stride), dtype=torch.int32, device=d)
        self.pair = torch.empty(reads_cap, dtype=torch.int32, device=d)
        self.h2d = torch.cuda.Event()
        self.filtered = torch.cuda.Event()   # the chunk's filter stage has finished
        self.done = torch.cuda.Event()
        self.free = None           # event after which the set may be overwritten


class _HostOut:
    def __init__(self, reads_cap, ops_stride):
        import torch
        self.best_score = torch.empty(reads_cap, dtype=torch.int32, pin_memory=True)
        self.mapped = torch.empty(reads_cap, dtype=torch.uint8, pin_memory=True)
        self.pair = torch.empty(reads_cap, dtype=torch.int32, pin_memory=True)
        self.aln = torch.empty((reads_cap, 7), dtype=torch.int32, pin_memory=True)
        self.ops = torch.empty((reads_cap, ops_stride), dtype=torch.int32, pin_memory=True)
        self.n_sel = torch.empty(1, dtype=torch.int32, pin_memory=True)
        self.d2h = torch.cuda.Event()
        self.pending = None        # (chunk index, n_reads) waiting to be handed out


class StreamAligner:
    """Filtered alignment of a stream of chunks against one resident reference.

    `thresholds` = (drop, lo, hi) of the filter's decision rule; `t_map` is the
    mapping threshold of sw_best_per_read.  With `band` the kept pairs are scored
    with their end cells and the traceback's DP covers only the columns each best
    alignment can reach (same results; worth it when the reads score on the int32
    path, i.e. reads longer than 100 nt, where ends cost about one instruction per
    cell).  run() hands every chunk's results to `consume(index, results)` as numpy
    arrays: best_score, mapped, pair (index of the best window in the chunk's
    window list, -1 if none), aln, ops, kept (pairs aligned)."""

    def __init__(self, ctx, ref_ascii: np.ndarray, mlp, thresholds, t_map: int, reads_cap: int,
                 bases_cap: int, pairs_cap: int, ops_stride: int = 64, scoring=SCORING,
                 band: bool = True):
        import torch
        self.ctx, self.mlp, self.scoring, self.t_map = ctx, mlp, scoring, int(t_map)
        self.band = bool(band)
        self.drop, self.lo, self.hi = (float(x) for x in thresholds)
        self.ops_stride = int(ops_stride)
        self.caps = (reads_cap, bases_cap, pairs_cap)
        d = "cuda"
        self.ref_ascii = torch.from_numpy(np.ascontiguousarray(ref_ascii)).to(d)
        self.ref_len = len(ref_ascii)
        self.ref2b = torch.empty((self.ref_len + 15) // 16, dtype=torch.int32, device=d)
        bad = torch.zeros(1, dtype=torch.int32, device=d)
        sw_pack2b(ctx, self.ref_ascii, self.ref_len, self.ref2b, bad)
        torch.cuda.synchronize()
        del self.ref_ascii
        self.sets = [_DeviceSet(reads_cap, bases_cap, pairs_cap, ops_stride) for _ in range(2)]
        self.outs = [_HostOut(reads_cap, ops_stride) for _ in range(2)]
        self.s_h2d, self.s_comp, self.s_d2h = (torch.cuda.Stream() for _ in range(3))

    def _batch(self, ds, hc, win, n_pairs_dev=None):
        c = sw_batch(_ptr(self.ref2b), self.ref_len, _ptr(ds.reads2b), hc.n_bases, _ptr(ds.read_off),
                     _ptr(ds.read_len), hc.n_reads, _ptr(win), hc.n_pairs, _ptr(n_pairs_dev))
        return _View(c, hc.n_reads, hc.n_pairs)

    def _compute(self, ds, hc):
        s = self.s_comp
        full = self._batch(ds, hc, ds.win)
        sw_pack2b(self.ctx, ds.reads, hc.n_bases, ds.reads2b, ds.bad, s)
        ds.n_unsure.zero_()
        sw_filter_candidates(self.ctx, full, self.mlp, self.lo, self.hi, ds.feat, ds.logits, ds.keep,
                             ds.win_out, ds.sel, ds.n_sel, ds.n_unsure, s, logit_drop=self.drop)
        kept = self._batch(ds, hc, ds.win_out, ds.n_sel)
        ds.filtered.record(s)
        sw_batch_score(self.ctx, kept, self.scoring, SW_WANT_ENDS if self.band else 0, ds.hits, s)
        sw_best_per_read(self.ctx, kept, ds.hits, self.t_map, ds.best_pair, ds.best_score,
                         ds.mapped, s)
        sw_batch_traceback(self.ctx, kept, self.scoring, ds.best_pair, hc.n_reads, ds.aln, ds.ops,
                           self.ops_stride, s, hits=ds.hits if self.band else None)
        # index of the best window in the chunk's own window list (data movement only)
        n = hc.n_reads
        bp = ds.best_pair[:n].long()
        ds.pair[:n] = ds.sel[bp.clamp(min=0)].where(bp >= 0, bp.new_full((), -1)).int()

    def _hand_out(self, ho, consume):
        idx, n = ho.pending
        ho.d2h.synchronize()
        consume(idx, dict(best_score=ho.best_score[:n].numpy().copy(),
                          mapped=ho.mapped[:n].numpy().astype(bool),
                          pair=ho.pair[:n].numpy().copy(),
                          aln=ho.aln[:n].numpy().copy().view(ALN_DTYPE).reshape(-1),
                          ops=ho.ops[:n].numpy().copy().view(np.uint32),
                          kept=int(ho.n_sel[0])))
        ho.pending = None

    def _copy_out(self, ds, ho, idx, n, after=None):
        """Device -> host copy of a computed chunk's results (on the d2h stream)."""
        import torch
        self.s_d2h.wait_event(ds.done)
        if after is not None:
            self.s_d2h.wait_event(after)
        with torch.cuda.stream(self.s_d2h):
            ho.best_score[:n].copy_(ds.best_score[:n], non_blocking=True)
            ho.mapped[:n].copy_(ds.mapped[:n], non_blocking=True)
            ho.pair[:n].copy_(ds.pair[:n], non_blocking=True)
            ho.aln[:n].copy_(ds.aln[:n], non_blocking=True)
            ho.ops[:n].copy_(ds.ops[:n], non_blocking=True)
            ho.n_sel.copy_(ds.n_sel, non_blocking=True)
            ho.d2h.record(self.s_d2h)
        ho.pending = (idx, n)
        ds.free = ho.d2h

    def run(self, chunks, consume=None, manifest: ChunkManifest | None = None, hook=None):
        """Process the HostChunk sequence `chunks` in order.

        manifest: skip the chunks it records as handed out and record each chunk
        once `consume` has returned, so that a run stopped by an exception can
        be started again with the same manifest and only redoes the rest
        (results are handed out with their index in `chunks`).  hook(i), when
        given, is called on the host before chunk i's copies are issued (e.g. to
        inject a failure); an exception from it, from `consume` or from a call
        stops the run after the device has finished the work already issued."""
        import torch
        try:
            self._run(chunks, consume, manifest, hook)
        except BaseException:
            torch.cuda.synchronize()      # no copy or kernel still uses the buffers
            for ho in self.outs:
                ho.pending = None
            for ds in self.sets:
                ds.free = None
            raise

    def _run(self, chunks, consume, manifest, hook):
        import torch
        user = consume or (lambda i, r: None)
        if manifest is not None:
            if manifest.n_chunks != len(chunks):
                raise ValueError("the manifest is for another number of chunks")

            def consume(i, r):
                user(i, r)
                manifest.mark(i)
            todo = manifest.pending()
        else:
            consume = user
            todo = list(range(len(chunks)))
        rc, bc, pc = self.caps
        prev = None            # (device set, chunk index, reads) computed, not yet copied out
        for k, i in enumerate(todo):
            hc = chunks[i]
            if hc.n_reads > rc or hc.n_bases > bc or hc.n_pairs > pc:
                raise ValueError("chunk exceeds the stream's capacity")
            if hook is not None:
                hook(i)
            ds = self.sets[k % 2]
            # host -> device, once the set's previous chunk has been copied out
            if ds.free is not None:
                self.s_h2d.wait_event(ds.free)
            with torch.cuda.stream(self.s_h2d):
                ds.reads[:hc.n_bases].copy_(hc.reads, non_blocking=True)
                ds.read_off[:hc.n_reads].copy_(hc.read_off, non_blocking=True)
                ds.read_len[:hc.n_reads].copy_(hc.read_len, non_blocking=True)
                ds.win[:hc.win.numel()].copy_(hc.win, non_blocking=True)
                ds.h2d.record(self.s_h2d)
            self.s_comp.wait_event(ds.h2d)
            with torch.cuda.stream(self.s_comp):
                self._compute(ds, hc)
                ds.done.record(self.s_comp)
            if prev is not None:
                pds, pk, pidx, pn = prev
                ho = self.outs[pk % 2]
                # the pinned output set still holds the chunk before: hand it out first
                if ho.pending is not None:
                    self._hand_out(ho, consume)
                self._copy_out(pds, ho, pidx, pn, after=ds.filtered)
            prev = (ds, k, i, hc.n_reads)
        if prev is not None:
            pds, pk, pidx, pn = prev
            ho = self.outs[pk % 2]
            if ho.pending is not None:
                self._hand_out(ho, consume)
            self._copy_out(pds, ho, pidx, pn)
        for k in range(len(todo), len(todo) + 2):
            ho = self.outs[k % 2]
            if ho.pending is not None:
                self._hand_out(ho, consume)
        torch.cuda.synchronize()
