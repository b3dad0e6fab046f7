"""Reference of the per-candidate seed-hit features (test infrastructure).

Stage D of the paper (Sec. 2, "Stage D: CAL Seeker") turns the exact matches
of a read's short seeds (stage C, "Region Seeker") into candidate alignment
locations when enough of them fall close together.  The learned filter scores
each candidate window from the same kind of evidence; this module is the
plain definition of those 64 features, written directly from it:

  query q   the read, or its reverse complement for a strand-1 window, cut to
            its first MF = 256 bases; m = len(q)
  window t  the reference window clipped to the reference, cut to its first
            NF = 1024 bases; n = len(t)
  k-mers    every k = 12 base substring, q at p = 0..P-1 (P = m-k+1), t at
            j = 0..J-1 (J = n-k+1)
  hits      all (p, j) with q[p:p+k] == t[j:j+k]; diagonal d = j - p, bin
            b = (d + m) >> 4

Per candidate (nh = number of hits, Pd = max(P, 1)):
  f0   distinct hit positions p / Pd
  f1   min(nh, 4 Pd) / Pd
  f2   hits in the modal bin / Pd        (modal bin: most hits, smallest on ties)
  f3   hits in the modal bin and its two neighbours / Pd   ("nmode3")
  f4   min(distinct bins, 64) / 16
  f5   (16 * modal bin + 8 - m) / max(n, 1), 0 without hits
  f6   1 if nh > 0
  f7..22   histogram of hit p over 16 equal bins ((16 p) // Pd) / Pd
  f23..38  histogram of hit j over 16 bins ((16 j) // max(J, 1)) / Pd
Per read (over the K candidates of the read, K <= 64):
  f39  (nmode3 - max nmode3) / Pd
  f40  (distinct p - max distinct p) / Pd
  f41  1 if nmode3 equals the maximum
  f42  candidates with a strictly larger nmode3 / K
  f43  (largest - second largest nmode3, over the sorted list) / Pd
  f44  K / 16
  f45  n / 1000,   f46  m / 1000,   f47  strand,   f48  G+C of the window / max(n, 1)
  f49..63 zero
Each feature is computed in float32 (one correctly rounded division or
product) and rounded to bfloat16 (round to nearest even).
"""
from __future__ import annotations

import numpy as np

K = 12
MF = 256
NF = 1024
NFEAT = 64


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def _kmers(codes: np.ndarray) -> np.ndarray:
    L = len(codes) - K + 1
    if L <= 0:
        return np.zeros(0, dtype=np.int64)
    v = np.zeros(L, dtype=np.int64)
    for i in range(K):
        v |= codes[i:i + L].astype(np.int64) << (2 * i)
    return v


def candidate_stats(q: np.ndarray, t: np.ndarray) -> dict:
    """Seed-hit statistics of one (query, window) pair (codes 0..3)."""
    q = q[:MF]
    t = t[:NF]
    m, n = len(q), len(t)
    kq, kt = _kmers(q), _kmers(t)
    P, J = len(kq), len(kt)
    hits_p, hits_j = [], []
    if P and J:
        for p in range(P):
            js = np.nonzero(kt == kq[p])[0]
            hits_p.extend([p] * len(js))
            hits_j.extend(js.tolist())
    hp = np.array(hits_p, dtype=np.int64)
    hj = np.array(hits_j, dtype=np.int64)
    nh = len(hp)
    st = dict(m=m, n=n, P=P, J=J, nh=nh, ndp=len(set(hits_p)))
    if nh:
        bins = (hj - hp + m) >> 4
        cnt = np.bincount(bins, minlength=int(bins.max()) + 2)
        mode = int(np.argmax(cnt))
        st["nmode"] = int(cnt[mode])
        st["nmode3"] = int(cnt[mode] + (cnt[mode - 1] if mode > 0 else 0) + cnt[mode + 1])
        st["nbins"] = int((cnt > 0).sum())
        st["mode"] = mode
        Pd = max(P, 1)
        st["hist_p"] = np.bincount((16 * hp) // Pd, minlength=16)[:16]
        st["hist_j"] = np.bincount((16 * hj) // max(J, 1), minlength=16)[:16]
    else:
        st.update(nmode=0, nmode3=0, nbins=0, mode=0, hist_p=np.zeros(16, np.int64),
                  hist_j=np.zeros(16, np.int64))
    st["gc"] = int(((t == 1) | (t == 2)).sum())
    return st


def read_features(stats: list[dict], strands: list[int]) -> np.ndarray:
    """Features [K, 64] (bf16 values as float32) of one read's candidates."""
    Kc = len(stats)
    f = np.zeros((Kc, NFEAT), dtype=np.float32)
    nm3 = np.array([s["nmode3"] for s in stats], dtype=np.int64)
    ndp = np.array([s["ndp"] for s in stats], dtype=np.int64)
    mx3 = nm3.max() if Kc else 0
    mxd = ndp.max() if Kc else 0
    srt = np.sort(nm3)[::-1]
    second = srt[1] if Kc > 1 else 0
    f32 = np.float32
    for c, s in enumerate(stats):
        Pd = f32(max(s["P"], 1))
        f[c, 0] = f32(s["ndp"]) / Pd
        f[c, 1] = f32(min(s["nh"], 4 * int(Pd))) / Pd
        f[c, 2] = f32(s["nmode"]) / Pd
        f[c, 3] = f32(s["nmode3"]) / Pd
        f[c, 4] = f32(min(s["nbins"], 64)) / f32(16)
        f[c, 5] = (f32(16 * s["mode"] + 8 - s["m"]) / f32(max(s["n"], 1))) if s["nh"] else f32(0)
        f[c, 6] = f32(1) if s["nh"] else f32(0)
        f[c, 7:23] = s["hist_p"].astype(np.float32) / Pd
        f[c, 23:39] = s["hist_j"].astype(np.float32) / Pd
        f[c, 39] = f32(s["nmode3"] - mx3) / Pd
        f[c, 40] = f32(s["ndp"] - mxd) / Pd
        f[c, 41] = f32(1) if s["nmode3"] == mx3 else f32(0)
        f[c, 42] = f32(int((nm3 > s["nmode3"]).sum())) / f32(Kc)
        f[c, 43] = f32(mx3 - second) / Pd
        f[c, 44] = f32(Kc) / f32(16)
        f[c, 45] = f32(s["n"]) / f32(1000)
        f[c, 46] = f32(s["m"]) / f32(1000)
        f[c, 47] = f32(strands[c])
        f[c, 48] = f32(s["gc"]) / f32(max(s["n"], 1))
    return bf16_round(f)


def batch_features(batch, pairs=None) -> np.ndarray:
    """Features of the given pairs (default all) of a synth.Batch; every read's
    candidates are all its pairs, which must be contiguous in the batch."""
    from oracle import codes as to_codes
    ref = to_codes(batch.ref.tobytes())
    win = batch.windows
    rid = win["read_id"].astype(np.int64)
    out = np.zeros((batch.n_pairs, NFEAT), dtype=np.float32)
    want = np.ones(batch.n_pairs, bool) if pairs is None else np.isin(np.arange(batch.n_pairs), pairs)
    starts = np.concatenate([[0], np.nonzero(np.diff(rid))[0] + 1, [batch.n_pairs]])
    for a, b in zip(starts[:-1], starts[1:]):
        if not want[a:b].any():
            continue
        r = int(rid[a])
        read = to_codes(batch.read(r))
        stats, strands = [], []
        for p in range(a, b):
            w = win[p]
            q = (3 - read[::-1]).astype(np.uint8) if w["strand"] else read
            n = min(int(w["len"]), max(len(ref) - int(w["ref_begin"]), 0))
            t = ref[int(w["ref_begin"]):int(w["ref_begin"]) + n]
            stats.append(candidate_stats(q, t))
            strands.append(int(w["strand"]))
        out[a:b] = read_features(stats, strands)
    return out
