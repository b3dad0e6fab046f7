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
