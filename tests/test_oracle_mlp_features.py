"""Pins of the MLP and feature references: float64 finite differences for the
gradients, closed forms for the loss and Adam, brute-force and invariant checks
for the seed-hit features."""
import numpy as np

from oracle import features_ref as fr
from oracle import mlp_ref as mr


def test_bf16_round_known_values():
    x = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.0e-5, 0.0], dtype=np.float32)
    r = fr.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even mantissa (1.0);
    # 1 + 1.5 * 2^-8 rounds up to 1 + 2^-7
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0078125)
    assert r[3] == -2.5 and r[5] == 0.0
    assert abs(r[4] - 3.0e-5) / 3.0e-5 < 2 ** -8


def test_param_count():
    assert mr.N_PARAMS == 64 * 128 + 128 + 128 * 128 + 128 + 128 + 1 == 24961


def test_bce_closed_form():
    z = np.array([0.0, 2.0, -3.0, 40.0])
    y = np.array([1.0, 0.0, 1.0, 1.0])
    exp = np.mean([np.log(2), 2 + np.log1p(np.exp(-2)), 3 + np.log1p(np.exp(-3)),
                   np.log1p(np.exp(-40))])
    assert abs(mr.bce_with_logits(z, y) - exp) < 1e-12


def test_gradients_match_finite_differences():
    g = np.random.default_rng(0)
    theta = mr.init(3).astype(np.float64)
    theta[mr.N_PARAMS - 1 - 128 - 128:] += 0.1     # non-zero biases in the tail
    X = g.normal(0, 1, (37, 64))
    y = (g.random(37) < 0.4).astype(np.float64)
    L, grad = mr.grads(theta, X, y, rounding=False)
    assert abs(L - mr.loss(theta, X, y)) < 1e-12
    idx = np.concatenate([g.choice(8192, 40, replace=False),              # W1
                          8192 + g.choice(128, 10, replace=False),        # b1
                          8320 + g.choice(16384, 40, replace=False),      # W2
                          24704 + g.choice(128, 10, replace=False),       # b2
                          24832 + g.choice(128, 10, replace=False),       # w3
                          [24960]])                                       # b3
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mr.loss(tp, X, y) - mr.loss(tm, X, y)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, grad[i])


def test_rounded_gradients_close_to_exact():
    g = np.random.default_rng(1)
    theta = mr.init(4)
    X = fr.bf16_round(g.normal(0, 1, (256, 64)).astype(np.float32))
    y = (g.random(256) < 0.5).astype(np.float64)
    _, g64 = mr.grads(theta, X, y, rounding=False)
    _, g16 = mr.grads(theta, X, y, rounding=True)
    assert np.abs(g16 - g64).max() <= 0.02 * np.abs(g64).max()


def test_adam_first_step_is_signed_lr():
    theta = np.zeros(5, np.float32)
    g = np.array([1.0, -2.0, 0.5, 0.0, 3.0], np.float32)
    t, m, v = mr.adam(theta, np.zeros(5, np.float32), np.zeros(5, np.float32), g, 1, 0.01)
    # bias-corrected first step: -lr * g / |g|
    assert np.allclose(t[[0, 1, 2, 4]], [-0.01, 0.01, -0.01, -0.01], atol=1e-6)
    assert t[3] == 0.0


def test_adam_three_steps_hand_computed():
    """Moments, bias correction and parameter after each of three steps with
    gradients 1, -2, 0.5 (lr 0.1, beta1 0.9, beta2 0.999, eps 1e-8), worked out
    by hand:
      t=1: m = 0.1,    v = 0.001,     m/(1-0.9) = 1, v/(1-0.999) = 1, theta = -0.1
      t=2: m = -0.11,  v = 0.004999,  m/0.19 = -0.5789474, v/0.001999 = 2.5007504,
           theta = -0.1 + 0.1 * 0.5789474 / 1.5813761 = -0.0633896
      t=3: m = -0.049, v = 0.005244001, m/0.271 = -0.1808118,
           v/0.002997001 = 1.7497494, theta = -0.0633896 + 0.0136691 = -0.0497206"""
    th = np.zeros(1, np.float32)
    m = np.zeros(1, np.float32)
    v = np.zeros(1, np.float32)
    exp = [(0.1, 0.001, -0.1), (-0.11, 0.004999, -0.0633896465),
           (-0.049, 0.005244001, -0.0497205803)]
    for t, (g, (em, ev, eth)) in enumerate(zip([1.0, -2.0, 0.5], exp), start=1):
        th, m, v = mr.adam(th, m, v, np.array([g], np.float32), t, 0.1)
        assert abs(float(m[0]) - em) <= 1e-7 * max(1, abs(em)), (t, m)
        assert abs(float(v[0]) - ev) <= 1e-6 * ev, (t, v)
        assert abs(float(th[0]) - eth) <= 2e-7, (t, th)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments are g and g^2 at
    every step, so each step moves every parameter by lr against the sign of
    its gradient: theta_t = -t * lr * sign(g).  A wrong moment decay or a bias
    correction that does not follow the step count breaks this from step 2."""
    g = np.array([0.3, -2.0, 1e-3, 7.0], np.float32)
    th = np.zeros(4, np.float32)
    m = np.zeros(4, np.float32)
    v = np.zeros(4, np.float32)
    for t in range(1, 8):
        th, m, v = mr.adam(th, m, v, g, t, 0.01)
        assert np.allclose(th, -t * 0.01 * np.sign(g), rtol=0, atol=2e-6 * t), (t, th)


def test_training_reduces_loss():
    g = np.random.default_rng(2)
    X = g.normal(0, 1, (512, 64)).astype(np.float32)
    y = (X[:, 0] + 0.5 * X[:, 1] > 0).astype(np.float64)
    theta = mr.init(5)
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    L0 = mr.loss(theta, X, y)
    for step in range(1, 61):
        _, gr = mr.grads(theta, X, y, rounding=True)
        theta, m, v = mr.adam(theta, m, v, gr.astype(np.float32), step, 3e-3)
    assert mr.loss(theta, X, y) < 0.5 * L0


# ---- features ----------------------------------------------------------------

def _brute_hits(q, t):
    k = fr.K
    return [(p, j) for p in range(len(q) - k + 1) for j in range(len(t) - k + 1)
            if (q[p:p + k] == t[j:j + k]).all()]


def test_hits_match_brute_force():
    g = np.random.default_rng(3)
    for _ in range(30):
        q = g.integers(0, 2, int(g.integers(10, 40))).astype(np.uint8)   # binary: many hits
        t = g.integers(0, 2, int(g.integers(10, 60))).astype(np.uint8)
        st = fr.candidate_stats(q, t)
        hits = _brute_hits(q, t)
        assert st["nh"] == len(hits)
        assert st["ndp"] == len({p for p, _ in hits})


def test_feature_closed_forms():
    g = np.random.default_rng(4)
    read = g.integers(0, 4, 100).astype(np.uint8)
    t = np.concatenate([g.integers(0, 4, 37), read, g.integers(0, 4, 50)]).astype(np.uint8)
    st = fr.candidate_stats(read, t)
    P = 100 - 12 + 1
    assert st["ndp"] == P and st["nmode3"] >= P
    disjoint = fr.candidate_stats(np.zeros(100, np.uint8), np.full(300, 1, np.uint8))
    assert disjoint["nh"] == 0
    f = fr.read_features([st, disjoint], [0, 1])
    assert f[0, 0] == 1.0 and f[0, 6] == 1.0 and f[1, 6] == 0.0
    assert f[0, 41] == 1.0 and f[1, 41] == 0.0        # argmax flag
    assert f[1, 42] == 0.5                            # one of two candidates is better
    assert f[0, 47] == 0.0 and f[1, 47] == 1.0        # strand
    assert (f[:, 49:] == 0).all()
    # modal diagonal bin of an exact copy at window offset 37: d = 37 for every hit
    assert st["mode"] == (37 + 100) >> 4


def test_strand_symmetry():
    """A strand-1 candidate of a read has the features of the reverse
    complement of that read on strand 0, apart from the strand flag."""
    import synth
    g = np.random.default_rng(5)
    refc = g.integers(0, 4, 5000).astype(np.uint8)
    read = refc[1000:1100].copy()
    rc = (3 - read[::-1]).astype(np.uint8)
    b1 = synth.custom(synth.ASCII[refc].tobytes(), [synth.ASCII[rc].tobytes()],
                      [(0, 950, 300, 1), (0, 3000, 300, 0)])
    b0 = synth.custom(synth.ASCII[refc].tobytes(), [synth.ASCII[read].tobytes()],
                      [(0, 950, 300, 0), (0, 3000, 300, 1)])
    f1, f0 = fr.batch_features(b1), fr.batch_features(b0)
    keep = [i for i in range(64) if i != 47]
    assert (f1[:, keep] == f0[:, keep]).all()
    assert f1[0, 3] > 0.9 and f1[1, 3] < 0.1


def _planted_pair(seed):
    """A read of 100 bases holding four 12-mers copied from a 300-base window at
    (read position p, window position j) = (0, 10), (20, 150), (44, 288),
    (88, 200), the rest random; the brute-force hit list must be exactly those."""
    g = np.random.default_rng(seed)
    t = g.integers(0, 4, 300).astype(np.uint8)
    q = g.integers(0, 4, 100).astype(np.uint8)
    for p, j in ((0, 10), (20, 150), (44, 288), (88, 200)):
        q[p:p + 12] = t[j:j + 12]
    return q, t


def test_planted_hit_histograms_and_diagonals():
    """Histograms of planted hits, worked out by hand.  P = 100 - 11 = 89 read
    positions, J = 300 - 11 = 289 window positions.
      read bins (16 p) // 89:   0 -> 0, 20 -> 3, 44 -> 7, 88 -> 15
      window bins (16 j) // 289: 10 -> 0, 150 -> 8, 288 -> 15, 200 -> 11
      diagonal bins (j - p + 100) >> 4: 110 -> 6, 230 -> 14, 344 -> 21, 212 -> 13
    so 4 hits, 4 distinct read positions, 4 diagonal bins, the modal bin is 6
    (all bins hold one hit; the smallest wins) with nmode = nmode3 = 1, and
    f5 = (16 * 6 + 8 - 100) / 300.  Binning by m or n instead of P or J moves
    p = 20 to bin 3 (still), p = 88 to bin 14 and j = 200 to bin 10."""
    for seed in range(40):
        q, t = _planted_pair(seed)
        if sorted(_brute_hits(q, t)) == [(0, 10), (20, 150), (44, 288), (88, 200)]:
            break
    else:
        raise AssertionError("no seed without chance hits")
    st = fr.candidate_stats(q, t)
    f = fr.read_features([st], [0])[0]
    f32 = np.float32
    one = fr.bf16_round(f32(1) / f32(89))
    four = fr.bf16_round(f32(4) / f32(89))
    hp = np.zeros(16, np.float32)
    hp[[0, 3, 7, 15]] = one
    hj = np.zeros(16, np.float32)
    hj[[0, 8, 11, 15]] = one
    assert (f[7:23] == hp).all(), f[7:23]
    assert (f[23:39] == hj).all(), f[23:39]
    assert f[0] == four and f[1] == four and f[2] == one and f[3] == one
    assert f[4] == fr.bf16_round(f32(4) / f32(16)) and f[6] == 1.0
    assert f[5] == fr.bf16_round(f32(16 * 6 + 8 - 100) / f32(300))
    assert st["mode"] == 6 and st["nbins"] == 4


def test_per_read_features_hand_computed():
    """Three candidates of one read: A (the four planted hits above), B (the
    whole read copied at offset 37 of a 187-base window: 89 hits on one
    diagonal), C (a 240-base periodic window GGCA..., no hits, strand 1).
      nmode3 = [1, 89, 0], distinct read positions = [4, 89, 0], so
      f39 = (nmode3 - 89) / 89, f40 = (ndp - 89) / 89, f41 = [0, 1, 0],
      f42 = [1/3, 0, 2/3], f43 = (89 - 1) / 89, f44 = 3/16,
      f45 = n / 1000 = [0.3, 0.187, 0.24], f46 = 0.1, f47 = [0, 0, 1],
      f48(C) = 180 / 240 G+C (two G and one C in every four bases)."""
    for seed in range(40):
        q, tA = _planted_pair(seed)
        if sorted(_brute_hits(q, tA)) == [(0, 10), (20, 150), (44, 288), (88, 200)]:
            break
    g = np.random.default_rng(99)
    tB = np.concatenate([g.integers(0, 4, 37), q, g.integers(0, 4, 50)]).astype(np.uint8)
    tC = np.tile(np.array([2, 2, 1, 0], np.uint8), 60)
    qC = (3 - q[::-1]).astype(np.uint8)
    assert len(_brute_hits(q, tB)) == 89 and not _brute_hits(qC, tC)
    sts = [fr.candidate_stats(q, tA), fr.candidate_stats(q, tB), fr.candidate_stats(qC, tC)]
    assert [s["nmode3"] for s in sts] == [1, 89, 0]
    f = fr.read_features(sts, [0, 0, 1])
    f32 = np.float32
    b = fr.bf16_round
    assert f[0, 39] == b(f32(-88) / f32(89)) and f[1, 39] == 0 and f[2, 39] == -1
    assert f[0, 40] == b(f32(-85) / f32(89)) and f[1, 40] == 0 and f[2, 40] == -1
    assert f[:, 41].tolist() == [0, 1, 0]
    assert f[0, 42] == b(f32(1) / f32(3)) and f[1, 42] == 0 and f[2, 42] == b(f32(2) / f32(3))
    assert (f[:, 43] == b(f32(88) / f32(89))).all()
    assert (f[:, 44] == b(f32(3) / f32(16))).all()
    assert f[:, 45].tolist() == b(np.array([0.3, 0.187, 0.24], np.float32)).tolist()
    assert (f[:, 46] == b(f32(0.1))).all()
    assert f[:, 47].tolist() == [0, 0, 1]
    assert f[2, 48] == b(f32(180) / f32(240))


def test_features_without_kmers_are_zero():
    """A read shorter than 12 bases (P = 0) or a window shorter than 12 (J = 0)
    has no hits: every hit feature is 0 (no division by P or J = 0), and the
    single candidate is its read's argmax."""
    g = np.random.default_rng(7)
    t = g.integers(0, 4, 300).astype(np.uint8)
    short = t[40:51].copy()                          # 11 bases: no 12-mer
    st = fr.candidate_stats(short, t)
    st2 = fr.candidate_stats(t[:100].copy(), t[:11].copy())
    for s, m in ((st, 11), (st2, 100)):
        f = fr.read_features([s], [0])[0]
        assert np.isfinite(f).all()
        # the only candidate holds the read's maximum (0), so f41 = 1
        assert (f[:41] == 0).all() and f[41] == 1 and f[42] == 0 and f[43] == 0
        assert f[44] == np.float32(1) / np.float32(16)
        assert f[46] == fr.bf16_round(np.float32(m) / np.float32(1000))
