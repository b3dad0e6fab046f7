"""Seeded test batches shared by the GPU parity tests and the kernel's host model."""
import numpy as np

import synth


def edge_batch(seed, ms, ns, strands=(0, 1), ref_len=300_000, div=0.04):
    """Pairs of every (m, n) combination: a mutated copy of a reference segment as
    the read, a window that overlaps it."""
    g = np.random.default_rng(seed)
    ref = g.integers(0, 4, size=ref_len).astype(np.uint8)
    reads, wins = [], []
    for m in ms:
        for n in ns:
            for st in strands:
                b0 = int(g.integers(5000, ref_len - m - n - 5000))
                seg = ref[b0:b0 + m].copy()
                mut = g.random(m) < div
                seg[mut] = (seg[mut] + 1) % 4
                if m > 20 and g.random() < 0.5:         # an indel
                    k = int(g.integers(5, m - 5))
                    seg = np.concatenate([seg[:k], g.integers(0, 4, 2).astype(np.uint8), seg[k:]])[:m]
                read = (3 - seg[::-1]) if st else seg
                wb = b0 - int(g.integers(0, max(1, n // 2 + 1)))
                reads.append(synth.ASCII[read].tobytes())
                wins.append((len(reads) - 1, wb, n, st))
    return synth.custom(synth.ASCII[ref].tobytes(), reads, wins)


EDGE_M = [1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 99, 100, 101, 127, 128, 129, 150, 159, 160,
          161, 255, 256, 257, 511, 513, 1023, 1025, 2047, 2048, 2049, 2300]
EDGE_N = [1, 5, 16, 17, 63, 64, 65, 150, 333, 1000]
