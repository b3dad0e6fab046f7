"""GPU tests of the learned filter: seed-hit features (bit-exact), MLP forward,
gradients and Adam (against the bf16-rounded reference), determinism, and the
end-to-end filter (decision, compaction, recall against plain SW)."""
import numpy as np
import pytest
import torch

import synth
from oracle import features_ref as fr
from oracle import mlp_ref as mr
import paper_1304_0681_amd as sw
from paper_1304_0681_amd import train as tr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = sw.sw_ctx_create(0)
    yield c
    sw.sw_ctx_destroy(c)


def bf16_bits(f32):
    return (np.ascontiguousarray(f32, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def test_features_bitexact(ctx):
    b = synth.config4(n_reads=400, ref_len=300_000, seed=77)
    db = sw.DeviceBatch.from_synth(ctx, b)
    feat = torch.zeros((b.n_pairs, 64), dtype=torch.int16, device="cuda")
    sw.sw_features(ctx, db, feat)
    torch.cuda.synchronize()
    got = feat.cpu().numpy().view(np.uint16)
    exp = bf16_bits(fr.batch_features(b))
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} rows differ, first {bad[:3]}: cols " \
                          f"{np.nonzero(got[bad[0]] != exp[bad[0]])[0]}"


def test_features_edge_cases(ctx):
    """Short reads (no 12-mer), short and clipped windows, windows around the 1,024-base
    feature limit and beyond it, both strands, repeats."""
    g = np.random.default_rng(8)
    refc = g.integers(0, 4, 20_000).astype(np.uint8)
    refc[5000:5300] = 0                                    # a homopolymer run
    reads, wins = [], []
    for m in (5, 11, 12, 13, 60, 100, 255, 256, 300):
        o = int(g.integers(0, 15_000))
        seg = refc[o:o + m]
        reads.append(synth.ASCII[seg].tobytes())
        r = len(reads) - 1
        for (b0, n, st) in [(o - 20, 200, 0), (o, 11, 0), (o, 12, 1), (19_950, 400, 0),
                            (5000, 280, 0), (int(g.integers(0, 19_000)), 600, 1),
                            (o - 100, 1023, 0), (o - 200, 1024, 1), (o - 300, 1025, 0),
                            (max(o - 900, 0), 2000, 1)]:
            wins.append((r, max(b0, 0), n, st))
    reads.append(synth.ASCII[np.zeros(90, np.uint8)].tobytes())      # poly-A read
    wins += [(len(reads) - 1, 4990, 400, 0), (len(reads) - 1, 100, 300, 1)]
    b = synth.custom(synth.ASCII[refc].tobytes(), reads, wins)
    db = sw.DeviceBatch.from_synth(ctx, b)
    feat = torch.zeros((b.n_pairs, 64), dtype=torch.int16, device="cuda")
    sw.sw_features(ctx, db, feat)
    torch.cuda.synchronize()
    got = feat.cpu().numpy().view(np.uint16)
    exp = bf16_bits(fr.batch_features(b))
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert len(bad) == 0, f"rows {bad[:5]} differ in cols {np.nonzero(got[bad[0]] != exp[bad[0]])[0]}"


def test_features_bitexact_spliced_seeds(ctx):
    """Spliced-read seeds: 100-nt seeds against 4-12 windows of 200-1,000 nt."""
    b = synth.spliced(n_reads=120, seed=synth.BASE_SEED + 91, ref_len=2_000_000)
    assert int(b.windows["len"].max()) >= 990
    db = sw.DeviceBatch.from_synth(ctx, b)
    feat = torch.zeros((b.n_pairs, 64), dtype=torch.int16, device="cuda")
    sw.sw_features(ctx, db, feat)
    torch.cuda.synchronize()
    got = feat.cpu().numpy().view(np.uint16)
    exp = bf16_bits(fr.batch_features(b))
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} rows differ, first {bad[:3]}"


def _mlp(ctx, theta):
    m = sw.sw_mlp_create(ctx)
    sw.sw_mlp_set_params(ctx, m, theta)
    return m


def _random_theta(seed):
    g = np.random.default_rng(seed)
    th = mr.init(seed)
    th[8192:8320] = g.normal(0, 0.1, 128)          # b1
    th[24576:24704] = g.normal(0, 0.1, 128)        # b2
    th[-1] = 0.3
    return th.astype(np.float32)


def _random_x(seed, n):
    g = np.random.default_rng(seed)
    return fr.bf16_round(g.normal(0, 1, (n, 64)).astype(np.float32))


def test_mlp_forward_matches_reference(ctx):
    th = _random_theta(11)
    X = _random_x(12, 1000)
    m = _mlp(ctx, th)
    try:
        xd = torch.from_numpy(bf16_bits(X).view(np.int16)).cuda()
        z = torch.empty(1000, dtype=torch.float32, device="cuda")
        sw.sw_mlp_forward(ctx, m, xd, 1000, z)
        torch.cuda.synchronize()
        got = z.cpu().numpy()
    finally:
        sw.sw_mlp_destroy(ctx, m)
    ref = mr.forward(th, X, rounding=True)["z"]
    err = np.abs(got - ref)
    assert np.median(err) < 2e-3 and err.max() < 0.05 * max(1.0, np.abs(ref).max()), \
        (np.median(err), err.max())


def test_mlp_gradients_match_reference(ctx):
    th = _random_theta(13)
    X = _random_x(14, 512)
    y = (np.random.default_rng(15).random(512) < 0.3).astype(np.float32)
    m = _mlp(ctx, th)
    try:
        xd = torch.from_numpy(bf16_bits(X).view(np.int16)).cuda()
        yd = torch.from_numpy(y).cuda()
        gd = torch.empty(sw.SW_MLP_PARAMS, dtype=torch.float32, device="cuda")
        ld = torch.empty(1, dtype=torch.float32, device="cuda")
        sw.sw_mlp_grad(ctx, m, xd, yd, 512, gd, ld)
        torch.cuda.synchronize()
        g_gpu, l_gpu = gd.cpu().numpy(), float(ld.item())
    finally:
        sw.sw_mlp_destroy(ctx, m)
    l_ref, g_ref = mr.grads(th, X, y, rounding=True)
    assert abs(l_gpu - l_ref) <= 1e-4 * max(1.0, abs(l_ref))
    tol = 1e-2 * np.abs(g_ref).max() + 1e-4
    for name, (a, b) in {"W1": (0, 8192), "b1": (8192, 8320), "W2": (8320, 24704),
                         "b2": (24704, 24832), "w3": (24832, 24960), "b3": (24960, 24961)}.items():
        e = np.abs(g_gpu[a:b] - g_ref[a:b]).max()
        assert e <= tol, (name, e, tol)


def test_train_step_is_adam(ctx):
    th = _random_theta(16)
    X = _random_x(17, 256)
    y = (np.random.default_rng(18).random(256) < 0.5).astype(np.float32)
    m = _mlp(ctx, th)
    try:
        xd = torch.from_numpy(bf16_bits(X).view(np.int16)).cuda()
        yd = torch.from_numpy(y).cuda()
        sw.sw_mlp_train_step(ctx, m, xd, yd, 256, 1e-3)
        after = sw.sw_mlp_get_params(ctx, m)
    finally:
        sw.sw_mlp_destroy(ctx, m)
    _, g = mr.grads(th, X, y, rounding=True)
    exp, _, _ = mr.adam(th, np.zeros_like(th), np.zeros_like(th), g.astype(np.float32), 1, 1e-3)
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    assert np.abs(after - exp)[big].max() < 1e-5
    assert (np.abs(after - th) <= 1e-3 + 1e-6).all()       # Adam moves at most lr per step


def test_training_is_deterministic(ctx):
    b = synth.config4(n_reads=2000, ref_len=500_000, seed=88)
    db = sw.DeviceBatch.from_synth(ctx, b)
    plain = tr.plain_scores(ctx, db)
    feat, y = tr.features_and_labels(ctx, db, plain)
    outs = []
    for _ in range(2):
        m, _ = tr.train(ctx, feat, y, steps=30, batch=1024, seed=3)
        outs.append(sw.sw_mlp_get_params(ctx, m))
        sw.sw_mlp_destroy(ctx, m)
    assert (outs[0] == outs[1]).all()


def test_filter_end_to_end(ctx):
    """Train on one seed, calibrate on a second, filter a third: recall of the
    best hit against plain SW, the decision rule and the compaction."""
    def data(seed, n):
        b = synth.config4(n_reads=n, ref_len=2_000_000, seed=seed)
        db = sw.DeviceBatch.from_synth(ctx, b)
        return b, db, tr.plain_scores(ctx, db)

    b_tr, db_tr, p_tr = data(101, 20_000)
    feat, y = tr.features_and_labels(ctx, db_tr, p_tr)
    mlp, losses = tr.train(ctx, feat, y, steps=400, batch=4096, seed=5, log_every=100)
    assert losses[-1][1] < losses[0][1]
    b_ca, db_ca, p_ca = data(102, 20_000)
    f_ca, _ = tr.features_and_labels(ctx, db_ca, p_ca)
    z = tr.logits_of(ctx, mlp, f_ca).cpu().numpy()
    rid = b_ca.windows["read_id"].astype(np.int64)
    sc = p_ca.hits[:, 0].cpu().numpy()
    best = p_ca.best_score.cpu().numpy()
    lo, hi, rec = tr.calibrate(z, sc, best, rid, target=0.999)
    b_te, db_te, p_te = data(103, 20_000)
    buf = tr.FilterBuffers(b_te.n_pairs, b_te.n_reads)
    kept = tr.filtered_pass(ctx, mlp, db_te, lo, hi, buf)
    torch.cuda.synchronize()
    keep = buf.keep.cpu().numpy().astype(bool)
    zt = buf.logits.cpu().numpy()
    rid_t = b_te.windows["read_id"].astype(np.int64)
    sc_t = p_te.hits[:, 0].cpu().numpy()
    best_t = p_te.best_score.cpu().numpy()
    exp_keep, hit, unsure = tr.filter_outcome(zt, sc_t, best_t, rid_t, lo, hi)
    assert (keep == exp_keep).all()
    n_sel = int(buf.n_sel.item())
    assert n_sel == int(keep.sum())
    assert (buf.sel[:n_sel].cpu().numpy() == np.nonzero(keep)[0]).all()
    w_out = buf.win_out.cpu().numpy().view(synth.WINDOW_DTYPE)[:n_sel]
    assert (w_out == b_te.windows[keep]).all()
    assert int(buf.n_unsure.item()) == int(unsure.sum())
    fbest = buf.best_score.cpu().numpy()
    exp_fbest = np.full(b_te.n_reads, -1)
    np.maximum.at(exp_fbest, rid_t[keep], sc_t[keep])
    assert (fbest == exp_fbest).all()
    recall = float((fbest == best_t).mean())
    assert recall == float(hit.mean())
    assert recall >= 0.995, recall
    assert keep.mean() < 0.5, keep.mean()
    # output-level rule: reads predicted unmapped are not aligned at all
    t_map = 100
    drop, lo2, hi2, _ = tr.calibrate_output(z, sc, best, rid, t_map, target=0.999)
    assert drop <= lo2 <= hi2
    tr.filtered_pass(ctx, mlp, db_te, lo2, hi2, buf, drop=drop)
    torch.cuda.synchronize()
    keep2 = buf.keep.cpu().numpy().astype(bool)
    exp_keep2, hit2, _ = tr.filter_outcome(buf.logits.cpu().numpy(), sc_t, best_t, rid_t, lo2, hi2, drop)
    assert (keep2 == exp_keep2).all()
    assert int(buf.n_sel.item()) == int(keep2.sum())
    fbest2 = buf.best_score.cpu().numpy()
    exp2 = np.full(b_te.n_reads, -1)
    np.maximum.at(exp2, rid_t[keep2], sc_t[keep2])
    assert (fbest2 == exp2).all()          # reads with nothing kept report -1 (unmapped)
    mapped = best_t >= t_map
    rec2 = float((fbest2[mapped] == best_t[mapped]).mean())
    assert rec2 >= 0.995, rec2
    assert (fbest2[~mapped] < t_map).all()
    assert keep2.sum() < keep.sum()
    sw.sw_mlp_destroy(ctx, mlp)


def test_labels_match_host(ctx):
    b = synth.config4(n_reads=3000, ref_len=1_000_000, seed=111)
    db = sw.DeviceBatch.from_synth(ctx, b)
    p = tr.plain_scores(ctx, db)
    sc = p.hits[:, 0].cpu().numpy()
    best = p.best_score.cpu().numpy()
    rid = b.windows["read_id"].astype(np.int64)
    for margin, min_best in ((10, None), (0, None), (10, 200)):
        _, y = tr.features_and_labels(ctx, db, p, margin=margin, min_best=min_best)
        exp = (sc >= 0) & (sc >= best[rid] - margin)
        if min_best is not None:
            exp &= best[rid] >= min_best
        assert (y.cpu().numpy() == exp.astype(np.float32)).all()


def _f3(feat):
    x = feat[:, 3].cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return x.view(np.float32)


def test_network_gains_over_seed_count_rule(ctx):
    """What the trained network gains over the rule without it: on the hard
    workload (repeat families, decoys sharing a 15-mer with the read), the
    network and the seed-count rule (feature 3 in place of the logit, same
    decision structure) are calibrated for the same recall on one set and
    compared on another; the network keeps fewer pairs at that recall."""
    t_map = 200

    def data(seed, n):
        b = synth.config4_hard(n_reads=n, ref_len=2_000_000, seed=seed)
        db = sw.DeviceBatch.from_synth(ctx, b)
        return b, db, tr.plain_scores(ctx, db)

    b_tr, db_tr, p_tr = data(201, 30_000)
    feat, y = tr.features_and_labels(ctx, db_tr, p_tr, min_best=t_map)
    mlp, _ = tr.train(ctx, feat, y, steps=600, batch=4096, seed=7)
    out = {}
    for name, seed in (("cal", 202), ("test", 203)):
        b, db, p = data(seed, 30_000)
        f, _ = tr.features_and_labels(ctx, db, p)
        out[name] = (tr.logits_of(ctx, mlp, f).cpu().numpy(), _f3(f), p.hits[:, 0].cpu().numpy(),
                     p.best_score.cpu().numpy(), b.windows["read_id"].astype(np.int64))
    z, zh, sc, best, rid = out["cal"]
    thr_n = tr.calibrate_output(z, sc, best, rid, t_map, target=0.999)
    thr_h = tr.calibrate_output(zh, sc, best, rid, t_map, target=0.999)
    z, zh, sc, best, rid = out["test"]
    mapped = best >= t_map
    keep_n, hit_n, _ = tr.filter_outcome(z, sc, best, rid, thr_n[1], thr_n[2], thr_n[0])
    keep_h, hit_h, _ = tr.filter_outcome(zh, sc, best, rid, thr_h[1], thr_h[2], thr_h[0])
    rec_n, rec_h = hit_n[mapped].mean(), hit_h[mapped].mean()
    assert rec_n >= 0.997 and rec_h >= 0.997, (rec_n, rec_h)
    assert keep_n.mean() < 0.9 * keep_h.mean(), (keep_n.mean(), keep_h.mean())
    sw.sw_mlp_destroy(ctx, mlp)
