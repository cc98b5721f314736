"""Pins of the CPU oracle against what the mathematics fixes.

Every check here compares the oracle with something other than itself:
closed forms of the recurrences, invariants, special cases that reduce to a
textbook running average, exact rational arithmetic and brute force.  The
paper prints no worked example, so none of the pins are paper values.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import canon
from tests.brute_cog import Brute, kde_weights64

F32 = np.float32


def run_oracle(params, frames, n_train, mode="cog"):
    orc = O.Oracle(params)
    orc.train(frames[:n_train])
    masks, infos = [], []
    for t in range(n_train, len(frames)):
        if mode == "cog":
            m, inf = orc.step(frames[t])
        else:
            m, inf = orc.gmm_step(frames[t]), None
        masks.append(m)
        infos.append(inf)
    st = canon.parse(orc.export())
    orc.close()
    return np.array(masks), infos, st


# ---------------------------------------------------------------- kernel weights

def test_kde_weights_symmetry():
    W = O.kde_weights(8.0).astype(np.int64)
    assert np.array_equal(W, W[::-1, ::-1])


def test_kde_weights_mass_and_shape():
    W = O.kde_weights(8.0).astype(np.int64)
    mass = W.sum(axis=0)
    # interior levels keep the whole unit mass (16 roundings of +-0.5)
    assert np.all(np.abs(mass[40:216] - 65535) <= 8)
    # the edge levels lose the half-kernel that falls outside [0, 255]
    half = 0.5 + 0.5 / math.fsum(math.exp(-(e * e) / 128.0) for e in range(-1024, 1025))
    assert abs(mass[0] - 65535 * half) <= 8
    # unimodal in b for every level, peaked at the level's own bin
    for v in range(256):
        col = W[:, v]
        assert col.argmax() == v // 16
        pk = v // 16
        assert np.all(np.diff(col[:pk + 1]) >= 0) and np.all(np.diff(col[pk:]) <= 0)


def test_kde_weights_vs_float64_fsum():
    W = O.kde_weights(8.0).astype(np.int64)
    Wb = kde_weights64(8.0)
    assert np.abs(W - Wb).max() <= 1
    assert (W != Wb).sum() <= 4


# ---------------------------------------------------------------- prior table

def _params(w, h, C=3, K=3, **kw):
    return O.make_params(w, h, C, K, **kw)


def test_table_constant_training_closed_form():
    N, v = 12, 131
    fr = synth.constant_stream(N + 1, 2, 2, 3, [v, 7, 250])
    _, _, st = run_oracle(_params(2, 2), fr, N)
    W = O.kde_weights(8.0).astype(np.int64)
    for c, val in enumerate([v, 7, 250]):
        acc = N * W[:, val]
        amax = acc.max()
        expect = (255 * acc + amax // 2) // amax
        assert np.array_equal(st["table"][:, c, :], np.broadcast_to(expect, (4, 16)))
        assert st["table"][0, c, val // 16] == 255
    assert np.array_equal(st["cnt"], np.tile([N - 1, 0, 0], (4, 1)))


def test_table_vs_direct_float64_kde():
    """Brute force: direct Parzen sums per bin, max-normalised, within +-1."""
    N = 10
    fr = synth.random_stream(N, 4, 4, 3, seed=11, lo=30, hi=220)
    orc = O.Oracle(_params(4, 4))
    orc.train(fr)
    st = canon.parse(orc.export())
    z = math.fsum(math.exp(-(e * e) / 128.0) for e in range(-1024, 1025))
    phi = {d: math.exp(-(d * d) / 128.0) / z for d in range(-300, 300)}
    for px in range(16):
        for c in range(3):
            xs = fr[:, px // 4, px % 4, c].astype(int)
            dens = [math.fsum(phi[u - x] for x in xs for u in range(16 * b, 16 * b + 16))
                    for b in range(16)]
            dmax = max(dens)
            ref = np.array([255.0 * d / dmax for d in dens])
            assert np.abs(st["table"][px, c].astype(float) - ref).max() <= 1.0


def test_residue_counts_bruteforce_and_special_cases():
    N = 30
    fr = synth.random_stream(N, 3, 5, 3, seed=5)
    orc = O.Oracle(_params(5, 3))
    orc.train(fr)
    st = canon.parse(orc.export())
    d = np.abs(np.diff(fr.astype(int), axis=0)).max(axis=3).reshape(N - 1, 15)
    ref = np.stack([(d < 16).sum(0), ((d >= 16) & (d < 48)).sum(0), (d >= 48).sum(0)], 1)
    assert np.array_equal(st["cnt"].astype(int), ref)
    # pure oscillation of 30 levels -> all in the middle bin; of 100 -> last bin
    for amp, col in ((30, 1), (100, 2)):
        fr = synth.alternating_stream(N, 2, 2, 3, [80, 80, 80], [80 + amp, 80, 80])
        orc = O.Oracle(_params(2, 2))
        orc.train(fr)
        cnt = canon.parse(orc.export())["cnt"]
        expect = np.zeros(3, int)
        expect[col] = N - 1
        assert np.array_equal(cnt[0], expect)


# ---------------------------------------------------------------- mixture step

def _rec(rows):
    return np.array([[w, *mu, var] for (w, mu, var) in rows], dtype=np.float32)


def test_one_step_variance_response_closed_form():
    p = _params(1, 1, K=1)
    v0 = 100.0
    # matched at the floor, x = v0 + 5 on every channel: mu moves by alpha*5,
    # sigma^2 = (1-a) 12 + a * 3 * (5 (1-a))^2
    comp, lab, mp = O.pixel_gmmstep(p, _rec([(1.0, [v0] * 3, 12.0)]), [v0 + 5] * 3, 0.01)
    a = 0.01
    assert lab == 0 and mp == 0
    assert comp[0, 0] == 1.0
    np.testing.assert_allclose(comp[0, 1:4], v0 + a * 5, rtol=1e-6)
    np.testing.assert_allclose(comp[0, 4], (1 - a) * 12 + a * 3 * (5 * (1 - a)) ** 2, rtol=1e-6)
    # x equal to the mean: the variance decays geometrically ...
    comp, _, _ = O.pixel_gmmstep(p, _rec([(1.0, [v0] * 3, 20.0)]), [v0] * 3, 0.01)
    np.testing.assert_allclose(comp[0, 4], 0.99 * 20.0, rtol=1e-6)
    # ... but never below the floor
    comp, _, _ = O.pixel_gmmstep(p, _rec([(1.0, [v0] * 3, 12.0)]), [v0] * 3, 0.01)
    assert comp[0, 4] == F32(12.0)


def test_match_is_first_in_rank_order_not_nearest():
    p = _params(1, 1, K=3)
    rec = _rec([(0.5, [100] * 3, 400.0), (0.3, [103] * 3, 400.0), (0.2, [0] * 3, 675.0)])
    comp, lab, mp = O.pixel_gmmstep(p, rec, [103, 103, 103], 0.01)
    # both slots 0 and 1 match; slot 0 (first in rank order) takes the update
    assert mp == 0 and lab == 0
    assert comp[0, 1] > 100.0 and comp[1, 1] == F32(103.0)
    np.testing.assert_allclose(comp[:, 0], [0.5 * 0.99 + 0.01, 0.3 * 0.99, 0.2 * 0.99], rtol=1e-6)


def test_label_uses_background_set_before_update():
    p = _params(1, 1, K=2)
    # B = 1 (0.72 > T); x matches slot 1 -> foreground, whatever the update does
    rec = _rec([(0.72, [50] * 3, 100.0), (0.28, [150] * 3, 100.0)])
    assert O.pixel_bgset(p, rec) == 1
    _, lab, mp = O.pixel_gmmstep(p, rec, [150] * 3, 0.5)
    assert lab == 1 and mp in (0, 1)
    # B counts strictly above T: 0.7 exactly does not close the set
    rec2 = _rec([(0.7, [50] * 3, 100.0), (0.3, [150] * 3, 100.0)])
    cum = Fraction(float(F32(0.7)))
    assert (cum > Fraction(float(F32(0.7)))) is False
    assert O.pixel_bgset(p, rec2) == 2


def test_no_match_replaces_least_probable_slot_exact():
    p = _params(1, 1, K=3)
    rec = _rec([(0.5, [10] * 3, 50.0), (0.3, [60] * 3, 50.0), (0.2, [110] * 3, 50.0)])
    x = [250, 250, 250]
    comp, lab, mp = O.pixel_gmmstep(p, rec, x, 0.01)
    assert lab == 1 and mp == -1
    a = Fraction(float(F32(0.01)))
    om = Fraction(float(F32(1) - F32(0.01)))
    w = [Fraction(float(F32(0.5))) * om, Fraction(float(F32(0.3))) * om, a]
    S = sum(w)
    exact = [float(wi / S) for wi in w]
    # new slot: (a/S, x, var_init); its key w/sigma is the smallest -> stays last
    np.testing.assert_allclose(comp[:, 0], exact, rtol=4e-7)
    assert np.array_equal(comp[2, 1:4], np.array(x, F32)) and comp[2, 4] == F32(675.0)


@pytest.mark.parametrize("seed", range(6))
def test_sort_and_background_set_exact_rationals(seed):
    rng = np.random.default_rng(seed)
    K = 5
    p = _params(1, 1, K=K)
    for _ in range(200):
        w = rng.dirichlet(np.ones(K)).astype(np.float32)
        if rng.random() < 0.3:
            w[rng.integers(1, K):] = 0
            w = (w / w.sum()).astype(np.float32)
        mus = rng.uniform(0, 255, size=(K, 3))
        var = rng.uniform(12, 900, size=K)
        rec = np.concatenate([w[:, None], mus, var[:, None]], 1).astype(np.float32)
        # background set from exact rationals of the stored values
        cum, B = Fraction(0), K
        near = False
        for b in range(K):
            cum += Fraction(float(rec[b, 0]))
            if abs(cum - Fraction(float(F32(0.7)))) < Fraction(1, 10**6):
                near = True
            if cum > Fraction(float(F32(0.7))):
                B = b + 1
                break
        if not near:
            assert O.pixel_bgset(p, rec) == B
        x = rng.uniform(0, 255, size=3)
        out, lab, mp = O.pixel_gmmstep(p, rec, x, 0.01)
        keys = [Fraction(float(out[k, 0])) ** 2 / Fraction(float(out[k, 4])) for k in range(K)]
        assert all(keys[k] >= keys[k + 1] for k in range(K - 1)), keys
        s = sum(Fraction(float(v)) for v in out[:, 0])
        assert abs(float(s) - 1.0) <= K * 2.0 ** -23
        if mp >= 0:
            # the followed slot still holds the matched component's new mean
            assert np.all(np.abs(out[mp, 1:4] - x) <= np.abs(rec[:, 1:4] - x).max() + 1e-3)


def test_k1_infinite_lambda_is_running_average():
    """K=1 with an unbounded gate: the mixture is the textbook EMA, rho = alpha."""
    n, a = 60, 0.01
    fr = synth.random_stream(n, 2, 3, 3, seed=3, lo=50, hi=200)
    p = _params(3, 2, K=1, lam=1e18, stage_mask=0, kappa_alpha=0.0)
    _, _, st = run_oracle(p, fr, n_train=2, mode="gmm")
    x = fr.reshape(n, 6, 3).astype(np.float64)
    mu = x[0].copy()
    for j in range(1, n):
        mu = (1 - a) * mu + a * x[j]
    np.testing.assert_allclose(st["gmm"][:, 0, 1:4], mu, rtol=1e-5)
    assert np.all(st["gmm"][:, 0, 0] == 1.0)


def test_weights_sum_to_one_and_stay_in_unit_interval():
    spec = synth.preset("surveil-160x120-k3").with_(width=24, height=16, frames=90, n_train=20)
    fr = synth.make_stream(spec)
    orc = O.Oracle(_params(24, 16, K=3))
    orc.train(fr[:20])
    for t in range(20, 90):
        orc.step(fr[t])
        w = canon.parse(orc.export())["gmm"][:, :, 0].astype(np.float64)
        assert np.all(w >= 0) and np.all(w <= 1)
        assert np.abs(w.sum(1) - 1).max() <= 3 * 2.0 ** -23


# ---------------------------------------------------------------- constant input

def test_constant_input_closed_forms():
    N, v = 60, [90, 140, 200]
    fr = synth.constant_stream(N + 40, 3, 3, 3, v)
    p = _params(3, 3, K=3)
    masks, infos, st = run_oracle(p, fr, N)
    a = 0.01
    # training: slot 0 absorbs the pixel, w = 1, mu = v, sigma^2 decays to the floor
    assert np.all(st["gmm"][:, 0, 0] == 1.0) and np.all(st["gmm"][:, 1:, 0] == 0.0)
    np.testing.assert_allclose(st["gmm"][:, 0, 1:4], np.broadcast_to(v, (9, 3)), rtol=1e-6)
    expect_var = max(12.0, 675.0 * (1 - a) ** (N - 1))
    np.testing.assert_allclose(st["gmm"][:, 0, 4], expect_var, rtol=1e-5)
    assert np.all(st["gmm"][:, 0, 4] >= F32(12.0))
    # RGA seeded from the dominant mode
    np.testing.assert_allclose(st["rga"][:, :3], st["gmm"][:, 0, 1:4])
    # every online step is decided by frame differencing, background, no update
    assert all(i["n0"] == 9 and i["n_fg"] == 0 for i in infos)
    assert not masks.any()


def test_constant_input_without_fd_decays_rga_variance():
    N, v = 10, [90, 140, 200]
    steps = 500
    fr = synth.constant_stream(N + steps, 2, 2, 3, v)
    p = _params(2, 2, K=3, stage_mask=O.RGA | O.KDE)
    _, infos, st = run_oracle(p, fr, N)
    assert all(i["n1"] == 4 for i in infos)
    var0 = 675.0 * 0.99 ** (N - 1)
    expect = max(12.0, var0 * 0.99 ** steps)
    np.testing.assert_allclose(st["rga"][:, 3], expect, rtol=1e-5)
    assert np.all(st["rga"][:, 3] >= F32(12.0))
    np.testing.assert_allclose(st["rga"][:, :3], np.broadcast_to(v, (4, 3)), rtol=1e-6)


def test_rga_mean_matches_ema_closed_form():
    N, steps, a = 5, 120, 0.05
    rng = np.random.default_rng(9)
    base = np.array([100, 120, 140])
    fr = np.clip(base + rng.integers(-3, 4, size=(N + steps, 2, 2, 3)), 0, 255).astype(np.uint8)
    p = _params(2, 2, K=2, stage_mask=O.RGA, lambda_rga=1e6, alpha_rga=a)
    orc = O.Oracle(p)
    orc.train(fr[:N])
    mu0 = canon.parse(orc.export())["rga"][:, :3].astype(np.float64)
    for t in range(N, N + steps):
        _, inf = orc.step(fr[t])
        assert inf["n1"] == 4
    mu = canon.parse(orc.export())["rga"][:, :3].astype(np.float64)
    x = fr[N:].reshape(steps, 4, 3).astype(np.float64)
    n = steps
    ref = (1 - a) ** n * mu0 + a * sum((1 - a) ** (n - 1 - j) * x[j] for j in range(n))
    np.testing.assert_allclose(mu, ref, rtol=1e-5)


# ---------------------------------------------------------------- confidence stage

def _trained_const(v, N=20, **kw):
    fr = synth.constant_stream(N, 1, 1, 3, v)
    orc = O.Oracle(_params(1, 1, K=1, var_init=12.0, lam=1e18, **kw))
    orc.train(fr)
    return orc


def test_prior_accepts_value_in_trained_bin():
    # trained on 104: RGA sigma^2 = 12 so 110 fails S1 (108 > 75) but sits in
    # the same prior bin: P = 1, a = 1 -> C = 1 >= 0.5, decided at S2, no update
    orc = _trained_const([104] * 3)
    before = canon.parse(orc.export())
    m, inf = orc.step(np.full(3, 110, np.uint8))
    after = canon.parse(orc.export())
    assert inf["n2"] == 1 and m[0] == 0
    assert np.array_equal(before["gmm"], after["gmm"]) and np.array_equal(before["rga"], after["rga"])


def test_prior_nullified_sends_to_mixture_with_full_rate():
    orc = _trained_const([104] * 3)
    before = canon.parse(orc.export())
    x = np.full(3, 150, np.uint8)
    m, inf = orc.step(x)
    after = canon.parse(orc.export())
    assert inf["n3"] == 1
    # K=1 with an unbounded gate: matched, rho = alpha_e = alpha (C = 0)
    mu0 = before["gmm"][0, 0, 1:4].astype(np.float64)
    np.testing.assert_allclose(after["gmm"][0, 0, 1:4], mu0 + 0.01 * (150 - mu0), rtol=1e-6)


@pytest.mark.parametrize("delta,stage", [(12, 2), (36, 3)])
def test_residue_term_of_confidence(delta, stage):
    """Trained on a 30-level oscillation: b = 1, so C = max(0, 1 - delta/48)."""
    N = 21
    fr = synth.alternating_stream(N, 1, 1, 3, [100, 100, 100], [130, 100, 100])
    # a tiny RGA gate so that S1 never decides
    p = _params(1, 1, K=1, var_init=12.0, lam=1e18, p_null=2.0, lambda_rga=0.01, lambda_m=5.0)
    orc = O.Oracle(p)
    orc.train(fr)
    st = canon.parse(orc.export())
    assert list(st["cnt"][0]) == [0, N - 1, 0]
    xprev = st["prev"][0]
    x = np.array([xprev[0] + delta, xprev[1], xprev[2]], dtype=np.uint8)
    _, inf = orc.step(x)
    assert inf[f"n{stage}"] == 1
    if stage == 3:
        after = canon.parse(orc.export())
        C = 1.0 - delta / 48.0
        ae = 0.01 * (1 - 0.5 * C)
        mu0 = st["gmm"][0, 0, 1:4].astype(np.float64)
        np.testing.assert_allclose(after["gmm"][0, 0, 1:4], mu0 + ae * (x - mu0), rtol=1e-6)


def test_model_distance_term_of_confidence():
    """Trained on a 100-level oscillation: g = 1, so C = max(0, 1 - dr2/(lm^2 var_r))."""
    N = 21
    fr = synth.alternating_stream(N, 1, 1, 3, [60, 60, 60], [160, 60, 60])
    p = _params(1, 1, K=2, p_null=2.0, lambda_rga=1.0, lambda_m=2.0)
    orc = O.Oracle(p)
    orc.train(fr)
    st = canon.parse(orc.export())
    assert list(st["cnt"][0]) == [0, 0, N - 1]
    mu_r = st["rga"][0, :3].astype(np.float64)
    var_r = float(st["rga"][0, 3])
    # pick x so that 1 < dr2/var_r and C = 1 - dr2/(4 var_r) straddles 0.5
    for r, stage in ((1.5, 2), (2.5, 3)):
        o2 = O.Oracle(p)
        o2.train(fr)
        off = math.sqrt(r * var_r)
        x = np.clip(np.rint(mu_r + [off, 0, 0]), 0, 255).astype(np.uint8)
        dr2 = float(((x - mu_r) ** 2).sum())
        C = max(0.0, 1.0 - dr2 / (4.0 * var_r))
        _, inf = o2.step(x)
        assert (inf["n2"] == 1) == (C >= 0.5), (r, C, inf)


# ---------------------------------------------------------------- whole cascade

def test_forced_on_identity_equals_plain_gmm():
    spec = synth.preset("surveil-160x120-k3").with_(width=32, height=24, frames=120, n_train=30)
    fr = synth.make_stream(spec)
    p_cog = _params(32, 24, K=3, stage_mask=0, kappa_alpha=0.0)
    m1, _, s1 = run_oracle(p_cog, fr, 30, mode="cog")
    m2, _, s2 = run_oracle(p_cog, fr, 30, mode="gmm")
    assert np.array_equal(m1, m2)
    assert np.array_equal(s1["gmm"].view(np.uint32), s2["gmm"].view(np.uint32))


def test_illumination_step_flags_only_its_frame():
    N = 12
    fr = synth.step_stream(N + 6, 8, 8, 3, [100] * 3, [160] * 3, N + 2)
    _, infos, _ = run_oracle(_params(8, 8), fr, N)
    flags = [i["illum_flag"] for i in infos]
    assert flags == [0, 0, 1, 0, 0, 0]
    assert infos[2]["n3"] == 64


def test_pixel_permutation_equivariance():
    spec = synth.preset("surveil-160x120-k3").with_(width=20, height=10, frames=70, n_train=20)
    fr = synth.make_stream(spec).reshape(70, 200, 3)
    perm = np.random.default_rng(1).permutation(200)
    p = _params(200, 1)
    m1, i1, s1 = run_oracle(p, fr[:, None], 20)
    m2, i2, s2 = run_oracle(p, fr[:, perm][:, None], 20)
    assert np.array_equal(m1[:, perm], m2)
    assert np.array_equal(s1["gmm"][perm], s2["gmm"]) and np.array_equal(s1["rga"][perm], s2["rga"])
    assert [dict(d, frame=0) for d in i1] == [dict(d, frame=0) for d in i2]


def _mixed_4x4(seed, n):
    rng = np.random.default_rng(seed)
    base = rng.uniform(40, 215, size=(16, 3))
    alt = rng.uniform(0, 255, size=(16, 3))
    fr = np.empty((n, 16, 3))
    for t in range(n):
        v = base + rng.normal(0, 4, size=(16, 3))
        bim = np.arange(16) % 5 == 0
        if t % 2:
            v[bim] = alt[bim] + rng.normal(0, 4, size=(bim.sum(), 3))
        if t > n // 2 and t % 7 < 3:
            v[3:6] = rng.uniform(0, 255, size=3)
        if t % 3 == 0:
            v[10] = fr[t - 1, 10] if t else v[10]
        fr[t] = v
    return np.clip(np.rint(fr), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_4x4_float64_agrees(seed):
    N, steps = 10, 40
    fr = _mixed_4x4(seed, N + steps)
    kw = dict(lambda_rga=2.5, alpha_rga=0.01)
    p = _params(4, 4, K=3, **kw)
    prm = dict(T=0.7, lam=2.5, var_init=675.0, var_min=12.0, alpha=0.01, stage_mask=7,
               tau_fd=0.0, lambda_rga=2.5, alpha_rga=0.01, kde_h=8.0, res_e1=16.0, res_e2=48.0,
               lambda_m=5.0, conf_thr=0.5, p_null=0.1, kappa_alpha=0.5)
    br = Brute(4, 4, 3, 3, prm)
    br.train(fr[:N].astype(int))
    orc = O.Oracle(p)
    orc.train(fr[:N])
    st = canon.parse(orc.export())
    assert np.array_equal(st["table"], np.array(br.table, dtype=np.uint8))
    assert np.array_equal(st["cnt"], np.array(br.cnt))
    stages_seen = set()
    tie = np.zeros(16, bool)
    for t in range(N, N + steps):
        m, _ = orc.step(fr[t])
        bm, bst, marg = br.step(fr[t].astype(int))
        tie |= np.array(marg) < 1e-4
        ok = ~tie
        assert np.array_equal(m[ok], np.array(bm)[ok]), t
        stages_seen |= set(bst)
    st = canon.parse(orc.export())
    ok = ~tie
    assert ok.sum() >= 12
    for px in np.nonzero(ok)[0]:
        bc = br.comp[px]
        ref = np.array([[c[0], *c[1], c[2]] for c in bc])
        np.testing.assert_allclose(st["gmm"][px], ref, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(st["rga"][px], [*br.rga[px][0], br.rga[px][1]], rtol=1e-5)
    assert stages_seen >= {0, 1, 3}


# ---------------------------------------------------------------- further pins

def test_inactive_slots_never_match():
    p = _params(1, 1, K=2)
    # slot 1 is inactive (w = 0) with mean 0; x = 10 would pass its gate
    rec = _rec([(1.0, [200] * 3, 12.0), (0.0, [0] * 3, 675.0)])
    comp, lab, mp = O.pixel_gmmstep(p, rec, [10, 10, 10], 0.01)
    assert lab == 1 and mp == -1
    # the no-match rule fills the last slot with the initial variance
    assert comp[1, 4] == F32(675.0) and np.array_equal(comp[1, 1:4], np.full(3, 10, F32))


@pytest.mark.parametrize("chan_up,nullified", [(1, False), (2, True)])
def test_prior_nullified_drops_only_the_prior_term(chan_up, nullified):
    """Trained on 104: a value one bin up on 1 (2) channels has P ~ 0.23 (0.05).

    Below p_null = 0.1 the prior term is dropped (C = 0, alpha_e = alpha);
    above it C = P and alpha_e = alpha (1 - kappa P); both reach the mixture.
    """
    orc = _trained_const([104] * 3)
    st = canon.parse(orc.export())
    x = np.array([104] * 3, np.uint8)
    x[:chan_up] = 115
    _, inf = orc.step(x)
    assert inf["n3"] == 1
    W = O.kde_weights(8.0).astype(np.int64)
    t_up = (255 * W[7, 104] + W[6, 104] // 2) // W[6, 104]
    ph = float(F32(t_up ** chan_up * 255 ** (3 - chan_up)) / F32(255 ** 3))
    assert (ph < 0.1) == nullified
    C = 0.0 if nullified else ph
    ae = 0.01 * (1 - 0.5 * C)
    after = canon.parse(orc.export())
    mu0 = st["gmm"][0, 0, 1:4].astype(np.float64)
    np.testing.assert_allclose(after["gmm"][0, 0, 1:4], mu0 + ae * (x - mu0), rtol=2e-7)


def test_mixture_background_decision_reseeds_running_average():
    """A value matching the second mode (inside B) is BG at S3; the RGA takes
    that component -- mean and variance -- after its update."""
    seq = [60, 60, 60, 180] * 15
    fr = np.stack([np.full((1, 1, 3), s, np.uint8) for s in seq])
    p = _params(1, 1, K=3, stage_mask=O.FD | O.RGA, T=0.95, alpha=0.2)
    orc = O.Oracle(p)
    orc.train(fr)
    st = canon.parse(orc.export())
    g = st["gmm"][0]
    assert g[0, 1] == F32(60) and g[1, 1] == F32(180) and st["rga"][0, 0] == F32(60)
    x = np.full(3, 184, np.uint8)
    _, inf = orc.step(x)
    assert inf["n3"] == 1 and inf["n3_bg"] == 1
    after = canon.parse(orc.export())
    # the matched component keeps rank 1 and its variance leaves the floor
    assert after["gmm"][0, 1, 1] > 180 and after["gmm"][0, 1, 4] > F32(12.0)
    assert np.array_equal(after["rga"][0, :3], after["gmm"][0, 1, 1:4])
    assert after["rga"][0, 3] == after["gmm"][0, 1, 4]


def test_illumination_counts_only_mixture_level():
    N = 12
    v = 100
    seq = [v] * N + [v + 1, v + 1, v + 61, v + 61]
    fr = np.stack([synth.constant_stream(1, 8, 8, 3, [s] * 3)[0] for s in seq])
    _, infos, _ = run_oracle(_params(8, 8), fr, N)
    assert [i["n1"] for i in infos] == [64, 0, 0, 0]
    assert [i["n0"] for i in infos] == [0, 64, 0, 64]
    assert [i["illum_flag"] for i in infos] == [0, 0, 1, 0]


def test_f32_input_on_level_grid_equals_u8_path():
    """f32 frames holding integer levels, quantised over [0, 256), give the
    u8 results bit for bit (q(v) = v)."""
    spec = synth.preset("surveil-160x120-k3").with_(width=16, height=12, frames=60, n_train=20)
    fr = synth.make_stream(spec)
    pu = _params(16, 12, K=3)
    pf = _params(16, 12, K=3, dtype=O.F32, in_lo=0.0, in_hi=256.0)
    m1, i1, s1 = run_oracle(pu, fr, 20)
    m2, i2, s2 = run_oracle(pf, fr.astype(np.float32), 20)
    assert np.array_equal(m1, m2)
    for k in ("gmm", "rga", "table", "cnt", "label", "prev"):
        assert np.array_equal(s1[k], s2[k]), k
    assert [dict(d, frame=0) for d in i1] == [dict(d, frame=0) for d in i2]


def test_f32_quantisation_clamps_and_scales():
    W = O.kde_weights(8.0).astype(np.int64)
    # range [-1, 1): v maps to floor((v+1)*128); below the range -> level 0,
    # at or above the top -> level 255
    for v, lvl in ((-3.0, 0), (-1.0, 0), (0.0, 128), (0.5, 192), (0.99, 254), (7.0, 255)):
        fr = np.full((6, 1, 1, 1), v, np.float32)
        p = _params(1, 1, C=1, K=1, dtype=O.F32, in_lo=-1.0, in_hi=1.0)
        _, _, st = run_oracle(p, fr, 5)
        acc = 5 * W[:, lvl]
        amax = acc.max()
        assert np.array_equal(st["table"][0, 0], (255 * acc + amax // 2) // amax), v
