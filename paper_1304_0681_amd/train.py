"""Training and calibration of the learned candidate filter.

The network, its gradients and Adam all run in the library's kernels (C ABI:
sw_features, sw_mlp_labels, sw_mlp_train_step, sw_mlp_forward).  This module
only drives them: it builds labels from plain Smith-Waterman scores (a
candidate is positive when its score is within `margin` of the best score of
its read), draws minibatches, and calibrates the two decision thresholds on
held-out data so that the filtered best hit equals the plain one for a target
fraction of reads.  Calibration is host logic on the logits (numpy).

The filter replaces the paper's stage D rule (a merged seed region becomes a
candidate only when it is long enough; Sec. 2, "Stage D: CAL Seeker") by a
learned score, and keeps stage E's exhaustive alignment (Sec. 2, "Stage E",
task iii) as the fallback for every read the network is unsure about.
"""
from __future__ import annotations

import numpy as np

from . import (SW_MLP_PARAMS, DeviceBatch, sw_batch_score, sw_best_per_read, sw_features,
               sw_filter_candidates, sw_mlp_create, sw_mlp_forward, sw_mlp_labels,
               sw_mlp_set_params, sw_mlp_train_step)

SCORING = (5, -4, -10, -1)
D_IN, D_H = 64, 128


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the library's parameter layout."""
    g = np.random.default_rng(seed)
    parts = [g.normal(0, np.sqrt(2 / D_IN), D_IN * D_H), np.zeros(D_H),
             g.normal(0, np.sqrt(2 / D_H), D_H * D_H), np.zeros(D_H),
             g.normal(0, np.sqrt(1 / D_H), D_H), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == SW_MLP_PARAMS
    return p


class PlainResult:
    def __init__(self, hits, best_pair, best_score):
        self.hits, self.best_pair, self.best_score = hits, best_pair, best_score


def plain_scores(ctx, db: DeviceBatch, scoring=SCORING):
    """Plain Smith-Waterman on every pair + best hit per read (device tensors)."""
    import torch
    hits = torch.empty((db.n_pairs, 3), dtype=torch.int32, device="cuda")
    bp = torch.empty(db.n_reads, dtype=torch.int32, device="cuda")
    bs = torch.empty(db.n_reads, dtype=torch.int32, device="cuda")
    sw_batch_score(ctx, db, scoring, 0, hits)
    sw_best_per_read(ctx, db, hits, 0, bp, bs)
    return PlainResult(hits, bp, bs)


def features_and_labels(ctx, db: DeviceBatch, plain: PlainResult, margin: int = 10,
                        min_best: int | None = None):
    """Features of every pair and labels: within `margin` of the read's best plain
    score (and, with min_best, only for reads whose best score reaches it)."""
    import torch
    feat = torch.empty((db.n_pairs, 64), dtype=torch.int16, device="cuda")
    y = torch.empty(db.n_pairs, dtype=torch.float32, device="cuda")
    sw_features(ctx, db, feat)
    sw_mlp_labels(ctx, db, plain.hits, plain.best_score, margin, y,
                  min_best=-(1 << 31) if min_best is None else min_best)
    return feat, y


def train(ctx, feat, y, steps: int = 1500, batch: int = 4096, lr: float = 2e-3,
          seed: int = 1, log_every: int = 0):
    """Train a fresh network on (feat, y) (device tensors); returns (mlp, losses)."""
    import torch
    mlp = sw_mlp_create(ctx)
    sw_mlp_set_params(ctx, mlp, init_params(seed))
    n = feat.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    perm = torch.randperm(n, device="cuda", generator=gen)
    pos = 0
    for step in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, device="cuda", generator=gen)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb = feat.index_select(0, idx).contiguous()
        yb = y.index_select(0, idx).contiguous()
        # cosine decay of the learning rate
        lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / steps))
        sw_mlp_train_step(ctx, mlp, xb, yb, batch, max(lr_t, lr * 0.02), loss)
        if log_every and (step % log_every == 0 or step == steps - 1):
            losses.append((step, float(loss.item())))
    return mlp, losses


def logits_of(ctx, mlp, feat):
    import torch
    z = torch.empty(feat.shape[0], dtype=torch.float32, device="cuda")
    sw_mlp_forward(ctx, mlp, feat, feat.shape[0], z)
    return z


def read_segments_host(read_id: np.ndarray):
    """(first, count) of contiguous pair runs of each read id."""
    starts = np.concatenate([[0], np.nonzero(np.diff(read_id))[0] + 1])
    counts = np.diff(np.concatenate([starts, [len(read_id)]]))
    return starts, counts


def filter_outcome(z, scores, best, read_id, lo, hi, drop=float("-inf")):
    """Apply the decision rule on host arrays: returns (kept mask, hit per read,
    unsure per read) where hit = the kept pairs contain a best-scoring pair.
    Reads whose best logit is below `drop` keep nothing (and are not unsure)."""
    starts, counts = read_segments_host(read_id)
    mx = np.maximum.reduceat(z, starts)
    band = np.add.reduceat(((z >= lo) & (z < hi)).astype(np.int64), starts) > 0
    dropped = mx < drop
    unsure = ((mx < hi) | band) & ~dropped
    un_pair = np.repeat(unsure, counts)
    keep = (un_pair | (z >= hi)) & ~np.repeat(dropped, counts)
    is_best = scores == best[read_id]
    hit = np.add.reduceat((keep & is_best).astype(np.int64), starts) > 0
    return keep, hit, unsure


def calibrate(z, scores, best, read_id, target: float = 0.9995, gaps=(0.0, 0.5, 1.0, 2.0, 4.0),
              n_grid: int = 120):
    """Thresholds (lo, hi) with the fewest kept pairs whose best-hit recall on
    this data is at least `target`."""
    qs = np.quantile(z, np.linspace(0.5, 0.9995, n_grid))
    best_cfg = None
    for hi in qs:
        for gap in gaps:
            lo = hi - gap
            keep, hit, _ = filter_outcome(z, scores, best, read_id, lo, hi)
            rec = hit.mean()
            if rec >= target:
                k = int(keep.sum())
                if best_cfg is None or k < best_cfg[0]:
                    best_cfg = (k, float(lo), float(hi), float(rec))
    if best_cfg is None:          # no threshold reaches the target: keep everything
        return float(-np.inf), float(np.inf), 1.0
    return best_cfg[1], best_cfg[2], best_cfg[3]


def calibrate_output(z, scores, best, read_id, t_map: int, target: float = 0.9995,
                     gaps=(0.0, 0.5, 1.0, 2.0, 4.0), n_grid: int = 120):
    """Thresholds (drop, lo, hi) with the fewest kept pairs whose recall on the
    aligner's output is at least `target`.

    Only alignments scoring at least t_map become records (Sec. 2, stage E task
    iv); the others leave their read unmapped.  Recall is therefore taken over
    the mapped reads (plain best score >= t_map): a mapped read is recalled
    when the filtered best score equals the plain one.  An unmapped read stays
    unmapped whatever the filter keeps, so reads whose best logit is below
    `drop` are not aligned at all.  For each (lo, hi) of the grid, `drop` is
    the highest value whose extra misses keep the recall at the target."""
    starts, counts = read_segments_host(read_id)
    mx = np.maximum.reduceat(z, starts)
    mapped = best >= t_map
    n_map = max(int(mapped.sum()), 1)
    need = int(np.ceil(target * n_map))
    qs = np.quantile(z, np.linspace(0.5, 0.9995, n_grid))
    best_cfg = None
    for hi in qs:
        for gap in gaps:
            lo = hi - gap
            keep, hit, _ = filter_outcome(z, scores, best, read_id, lo, hi)
            hm = hit & mapped
            slack = int(hm.sum()) - need
            if slack < 0:
                continue
            mx_hm = np.sort(mx[hm])
            drop = float(mx_hm[slack]) if slack < len(mx_hm) else float("inf")
            drop = min(drop, float(lo))
            dropped = mx < drop
            k = int(keep[~np.repeat(dropped, counts)].sum())
            if best_cfg is None or k < best_cfg[0]:
                rec = float((hm & ~dropped).sum() / n_map)
                best_cfg = (k, drop, float(lo), float(hi), rec)
    if best_cfg is None:
        return float("-inf"), float("-inf"), float("inf"), 1.0
    return best_cfg[1:]


class FilterBuffers:
    """Device buffers of the filtered pipeline for one batch size."""

    def __init__(self, n_pairs: int, n_reads: int):
        import torch
        self.feat = torch.empty((n_pairs, 64), dtype=torch.int16, device="cuda")
        self.logits = torch.empty(n_pairs, dtype=torch.float32, device="cuda")
        self.keep = torch.empty(n_pairs, dtype=torch.uint8, device="cuda")
        self.win_out = torch.empty(n_pairs * 12, dtype=torch.uint8, device="cuda")
        self.sel = torch.empty(n_pairs, dtype=torch.int32, device="cuda")
        self.n_sel = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.n_unsure = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.hits = torch.empty((n_pairs, 3), dtype=torch.int32, device="cuda")
        self.best_pair = torch.empty(n_reads, dtype=torch.int32, device="cuda")
        self.best_score = torch.empty(n_reads, dtype=torch.int32, device="cuda")


def filtered_pass(ctx, mlp, db: DeviceBatch, lo: float, hi: float, buf: FilterBuffers,
                  scoring=SCORING, drop: float = float("-inf")):
    """Features -> logits -> decision -> compaction -> SW on the kept pairs ->
    best hit per read; everything stays on the device."""
    buf.n_unsure.zero_()
    sw_filter_candidates(ctx, db, mlp, lo, hi, buf.feat, buf.logits, buf.keep, buf.win_out,
                         buf.sel, buf.n_sel, buf.n_unsure, logit_drop=drop)
    kept = db.view(buf.win_out, db.n_pairs, buf.n_sel)
    sw_batch_score(ctx, kept, scoring, 0, buf.hits)
    sw_best_per_read(ctx, kept, buf.hits, 0, buf.best_pair, buf.best_score)
    return kept
