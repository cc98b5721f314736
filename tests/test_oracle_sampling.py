"""Pins of the oracle's confidence-based spatio-temporal sampling (§2
"Confidence based temporal sampling", §3.2): closed forms on constant input,
invariants (halted frames change nothing; period 1 is sampling off), the
confidence gate on both sides of its threshold, and a float64 brute-force
model on 4x4 and 16x8 streams."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import canon
from tests.brute_cog import Brute

SAMPLE = O.SAMPLE


def _params(w, h, C=3, K=3, **kw):
    return O.make_params(w, h, C, K, **kw)


def _state_wo_frame(blob):
    """Canonical state with the frame counter zeroed (it always advances)."""
    b = bytearray(blob)
    b[32:40] = bytes(8)
    return bytes(b)


def _expected_skips(n, P, W_frames, N, period, nblk):
    """Closed form for input that is confident on every evaluated frame:
    frames N .. N+W-1 saturate every pixel; from then on block b is skipped
    unless (n + b) % period == 0; the last block may be ragged."""
    if n < N + W_frames:
        return 0
    skip = 0
    for b in range(nblk):
        if (n + b) % period != 0:
            skip += min(64, P - 64 * b)
    return skip


@pytest.mark.parametrize("w,h,W_frames,period", [(16, 12, 5, 4), (10, 7, 3, 3), (8, 8, 1, 2)])
def test_constant_input_skip_counts_closed_form(w, h, W_frames, period):
    N, steps = 6, 30
    P = w * h
    nblk = (P + 63) // 64
    fr = synth.constant_stream(N + steps, h, w, 3, [90, 140, 60])
    o = O.Oracle(_params(w, h, stage_mask=7 | SAMPLE, samp_window=W_frames, samp_period=period))
    o.train(fr[:N])
    for t in range(N, N + steps):
        m, info = o.step(fr[t])
        exp = _expected_skips(t, P, W_frames, N, period, nblk)
        assert info["n_skip"] == exp, (t, info)
        # every evaluated pixel of constant input is decided by frame differencing
        assert info["n0"] == P - exp and info["n1"] == info["n2"] == info["n3"] == 0
        assert (m == 0).all()
    st = canon.parse(o.export())
    assert st["version"] == 3
    # each pixel counted its evaluated frames (all confident)
    evaluated = np.zeros(P, dtype=np.int64)
    for t in range(N, N + steps):
        for b in range(nblk):
            if _expected_skips(t, P, W_frames, N, period, nblk) == 0 or (t + b) % period == 0:
                evaluated[64 * b:64 * b + 64] += 1
    assert np.array_equal(st["sat"].astype(np.int64), evaluated)
    o.close()


def test_halted_frames_change_nothing():
    """One block, period 4: on the frames where the block is halted the
    state stays bitwise as it was and the labels repeat, whatever the input."""
    N, W_frames, period = 8, 4, 4
    fr = synth.constant_stream(N + 60, 8, 8, 3, [100, 100, 100])
    rng = np.random.default_rng(3)
    o = O.Oracle(_params(8, 8, stage_mask=7 | SAMPLE, samp_window=W_frames, samp_period=period))
    o.train(fr[:N])
    halted_seen = 0
    for t in range(N, N + 60):
        before = _state_wo_frame(o.export())
        st0 = canon.parse(o.export())
        sat_full = bool((st0["sat"] >= W_frames).all())
        will_halt = sat_full and (t % period) != 0
        x = rng.integers(0, 256, size=(8, 8, 3), dtype=np.uint8) if will_halt else fr[t]
        m, info = o.step(x)
        if will_halt:
            halted_seen += 1
            assert info["n_skip"] == 64
            assert _state_wo_frame(o.export()) == before
            assert np.array_equal(m, np.where(st0["label"] == 1, 255, 0).astype(np.uint8))
        else:
            assert info["n_skip"] == 0
    assert halted_seen >= 30


def test_period_one_is_sampling_off():
    N, steps = 10, 60
    spec = synth.preset("surveil-160x120-k3").with_(width=24, height=20, frames=N + steps,
                                                    n_train=N)
    fr = synth.make_stream(spec)
    a = O.Oracle(_params(24, 20))
    b = O.Oracle(_params(24, 20, stage_mask=7 | SAMPLE, samp_window=1, samp_period=1))
    a.train(fr[:N])
    b.train(fr[:N])
    for t in range(N, N + steps):
        ma, ia = a.step(fr[t])
        mb, ib = b.step(fr[t])
        assert np.array_equal(ma, mb)
        assert ib["n_skip"] == 0
        assert {k: v for k, v in ia.items()} == {k: v for k, v in ib.items()}
    sa, sb = canon.parse(a.export()), canon.parse(b.export())
    for k in ("gmm", "rga", "table", "cnt", "label", "prev"):
        assert np.array_equal(sa[k], sb[k]), k
    assert (sa["sat"] == 0).all() and (sb["sat"] > 0).any()


@pytest.mark.parametrize("row,col", [(0, 5), (1, 31)])  # inside block 0, and its last pixel
def test_one_unconfident_pixel_resets_its_block(row, col):
    N, W_frames, period = 6, 3, 2
    w, h = 32, 4  # two blocks of 64
    fr = synth.constant_stream(N + 40, h, w, 3, [80, 80, 80])
    fr[N + 12, row, col] = [250, 10, 250]  # far outside every model
    o = O.Oracle(_params(w, h, stage_mask=7 | SAMPLE, samp_window=W_frames, samp_period=period))
    o.train(fr[:N])
    skips = []
    for t in range(N, N + 40):
        _, info = o.step(fr[t])
        skips.append(info["n_skip"])
    # frame N+12 is evaluated for block 0 only if (N+12) % 2 == 0
    assert (N + 12) % period == 0
    t_hit = 12
    # before the hit the two blocks alternate: one of them halted every frame
    assert all(s == 64 for s in skips[W_frames:t_hit])
    # after the hit, block 0 is evaluated for at least W frames (its pixel 5
    # must re-saturate, and the pixel's return to the background breaks the
    # frame difference again), so only block 1 can be halted
    for k in range(t_hit + 1, t_hit + 1 + W_frames):
        block1_halted = (N + k + 1) % period != 0
        assert skips[k] == (64 if block1_halted else 0), (k, skips[k])
    st = canon.parse(o.export())
    assert st["sat"][64:].min() >= W_frames


@pytest.mark.parametrize("delta,confident", [(10, True), (16, True), (18, False), (20, False)])
def test_confidence_gate_at_07_sigma(delta, confident):
    """After training on a constant, sigma_r^2 has the closed form
    max(var_min, var_init (1-alpha)^(N-1)); a step of delta in one channel is
    accepted by S1 (2.5 sigma) and is confident only if delta^2 <= 0.49 sigma_r^2."""
    N, alpha = 20, 0.01
    var0 = max(12.0, 675.0 * (1 - alpha) ** (N - 1))
    assert (delta ** 2 <= 0.49 * var0) == confident and delta ** 2 <= 6.25 * var0
    fr = synth.constant_stream(N + 1, 1, 1, 3, [100, 100, 100])
    fr[N, 0, 0, 1] = 100 + delta
    o = O.Oracle(_params(1, 1, stage_mask=7 | SAMPLE, samp_window=8, samp_period=2,
                         samp_lambda=0.7))
    o.train(fr[:N])
    _, info = o.step(fr[N])
    assert info["n1"] == 1
    st = canon.parse(o.export())
    assert int(st["sat"][0]) == (1 if confident else 0)


def _calm_stream(seed, w, h, n):
    """Mostly static noisy background with a few flickering pixels and a
    short-lived object, so that blocks saturate, break and saturate again."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(40, 200, size=(h, w, 3))
    fr = np.empty((n, h, w, 3))
    for t in range(n):
        f = base + rng.normal(0, 1.0, size=base.shape)
        if 30 <= t < 37:
            f[1:3, 1:3] = [250, 20, 20]
        if t in (22, 45, 58):
            f[h - 1, w - 1] = 255.0 - base[h - 1, w - 1]
        fr[t] = f
    return np.clip(np.rint(fr), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("w,h,seed", [(4, 4, 0), (4, 4, 1), (16, 8, 2)])
def test_brute_force_sampling_agrees(w, h, seed):
    N, steps = 10, 60
    fr = _calm_stream(seed, w, h, N + steps)
    kw = dict(stage_mask=7 | SAMPLE, samp_window=4, samp_period=3, samp_lambda=1.5)
    p = _params(w, h, K=3, lambda_rga=2.5, alpha_rga=0.01, **kw)
    prm = dict(T=0.7, lam=2.5, var_init=675.0, var_min=12.0, alpha=0.01, stage_mask=7 | SAMPLE,
               tau_fd=0.0, lambda_rga=2.5, alpha_rga=0.01, kde_h=8.0, res_e1=16.0, res_e2=48.0,
               lambda_m=5.0, conf_thr=0.5, p_null=0.1, kappa_alpha=0.5,
               samp_window=4, samp_period=3, samp_lambda=1.5)
    P = w * h
    br = Brute(w, h, 3, 3, prm)
    br.train(fr[:N].reshape(N, P, 3).astype(int))
    orc = O.Oracle(p)
    orc.train(fr[:N])
    tie = np.zeros(P, bool)
    halted = 0
    for t in range(N, N + steps):
        m, info = orc.step(fr[t])
        bm, bst, marg = br.step(fr[t].reshape(P, 3).astype(int))
        tie |= np.array(marg) < 1e-4
        assert not tie.any(), "threshold tie in a sampling pin"
        assert np.array_equal(m, np.array(bm, dtype=np.uint8)), t
        assert info["n_skip"] == sum(1 for s in bst if s == -1), t
        halted += info["n_skip"] > 0
    st = canon.parse(orc.export())
    assert np.array_equal(st["sat"], np.array(br.sat, dtype=np.uint16))
    assert halted >= 5, "the stream never halted a block"
    assert (st["sat"] < 4).any() or halted < steps
