"""Edge cases of the HIP path against the oracle, bit for bit: each cascade
stage alone and in pairs, frames smaller than a tile or one pixel wide or
tall, parameter extremes, and a run long enough for mixture weights to decay
into binary32 subnormals (the build keeps IEEE denormals on both sides), and
the shortest and longest training the library accepts."""
import numpy as np
import pytest

import synth
from tests import canon
from tests.gpu_util import (compare_infos, compare_state, gpu_params, orc_params_like, run_gpu,
                            run_orc, say)

pytestmark = pytest.mark.gpu
KEYS = ("gmm", "rga", "table", "cnt", "label", "prev", "sat")


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09339_amd import cog
    return cog


def stream(w, h, frames, n_train, seed_off=0):
    spec = synth.preset("surveil-160x120-k3").with_(width=w, height=h, frames=frames,
                                                    n_train=n_train,
                                                    seed=synth.video.BASE_SEED + 1300 + seed_off)
    return synth.make_stream(spec)


def parity(C, p, fr, n_train, mode="frames"):
    mg, ig, sg = run_gpu(C, p, fr, n_train, mode=mode)
    mo, io, so = run_orc(orc_params_like(p), fr, n_train)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so, keys=KEYS) == 0
    return io


@pytest.mark.parametrize("mode", [6, "step"], ids=["runs-of-6", "per-frame"])
@pytest.mark.parametrize("mask", [1, 2, 4, 3, 5, 6])
def test_stage_subsets(C, mask, mode):
    fr = stream(48, 32, 80, 20, seed_off=mask)
    io = parity(C, gpu_params(C, 48, 32, K=3, stage_mask=mask), fr, 20, mode=mode)
    tot = {k: sum(i[k] for i in io) for k in ("n0", "n1", "n2")}
    if not mask & 1:
        assert tot["n0"] == 0
    if not mask & 2:
        assert tot["n1"] == 0
    if not mask & 4:
        assert tot["n2"] == 0


@pytest.mark.parametrize("w,h", [(1, 1), (1, 7), (7, 1), (64, 1), (65, 1), (1, 65), (3, 43)])
@pytest.mark.parametrize("variant", ["cascade", "cascade-per-frame", "sampling", "gmm"])
def test_tiny_and_thin_frames(C, w, h, variant):
    fr = stream(w, h, 60, 12, seed_off=w * 100 + h)
    kw = {}
    if variant == "sampling":
        kw = dict(stage_mask=15, samp_window=3, samp_period=2)
    if variant == "gmm":
        p = gpu_params(C, w, h, K=3, path=1)
        mg, _, sg = run_gpu(C, p, fr, 12, mode="frames", infos=False)
        mo, _, so = run_orc(orc_params_like(p), fr, 12, mode="gmm")
        assert np.array_equal(mg, mo)
        assert compare_state(sg, so, keys=("gmm", "label", "prev")) == 0
        return
    parity(C, gpu_params(C, w, h, K=4, **kw), fr, 12, mode="step" if variant == "cascade-per-frame" else 5)


@pytest.mark.parametrize("kw", [
    dict(tau_fd=2.0),                      # a tolerant frame difference
    dict(alpha=1.0, alpha_rga=1.0),        # the largest rate
    dict(T=1.0),                           # every component in the background set
    dict(conf_thr=0.0),                    # S2 accepts everything that reaches it
    dict(conf_thr=1.5),                    # S2 accepts nothing
    dict(p_null=0.0, kappa_alpha=1.0),     # prior never nullified, full rate modulation
    dict(lam=100.0, K=1),                  # one component that always matches
    dict(var_min=0.5, var_init=0.5),       # floor equal to the initial variance
])
@pytest.mark.parametrize("mode", [9, "step"], ids=["runs-of-9", "per-frame"])
def test_parameter_extremes(C, kw, mode):
    kw = dict(kw)
    K = kw.pop("K", 3)
    fr = stream(40, 24, 70, 20, seed_off=len(str(kw)))
    say("extreme", kw, mode)
    parity(C, gpu_params(C, 40, 24, K=K, **kw), fr, 20, mode=mode)


def test_subnormal_weights_long_run(C):
    """9 300 frames on a 16x4 frame of a static scene in which a few pixels
    flash once at frame 100: the component each flash creates (weight 0.01)
    then decays by (1 - 0.01) per frame and ends in the binary32 subnormal
    range (about 1e-42 after 9 200 frames, below 2^-126 ~ 1.2e-38); state
    and masks stay bitwise equal."""
    N, T = 20, 9300
    rng = np.random.default_rng(11)
    base = rng.uniform(40, 200, size=(4, 16, 3))
    fr = np.empty((T, 4, 16, 3), dtype=np.uint8)
    for t in range(T):
        f = base.copy()
        if t == 100:
            f[1, 2:9] = 255 - base[1, 2:9]
        fr[t] = np.clip(np.rint(f), 0, 255)
    p = gpu_params(C, 16, 4, K=3, stage_mask=0, kappa_alpha=0.0)  # every pixel through the mixture
    mg, _, sg = run_gpu(C, p, fr, N, mode=1000, infos=False)
    mo, _, so = run_orc(orc_params_like(p), fr, N)
    assert np.array_equal(mg, mo)
    assert compare_state(sg, so, keys=KEYS) == 0
    w = so["gmm"][..., 0]
    sub = (w > 0) & (w < np.finfo(np.float32).tiny)
    assert sub.any(), "no weight reached the subnormal range"


@pytest.mark.parametrize("n_train", [2, 65536], ids=["shortest", "longest"])
def test_training_length_extremes(C, n_train):
    """The shortest and longest training the library accepts (2 and 65 536
    frames) on a 16x8 frame whose channels sit near the centres of prior bins
    0, 1 and 12 with small noise.  At 65 536 frames the bin masses of an even
    and an odd bin pass 2^31, the residue counts reach 65 535, and the u8
    path's paired 32-bit accumulators come closest to their limit; the prior
    table, counts, mixture and every later frame stay bitwise equal."""
    rng = np.random.default_rng(170509347)
    H, W, extra = 8, 16, 8
    T = n_train + extra
    centre = np.array([8, 24, 200], dtype=np.int16)
    fr = np.empty((T, H, W, 3), dtype=np.uint8)
    for t0 in range(0, T, 4096):
        t1 = min(T, t0 + 4096)
        noise = rng.integers(-2, 3, size=(t1 - t0, H, W, 3), dtype=np.int16)
        fr[t0:t1] = np.clip(centre + noise, 0, 255).astype(np.uint8)
    fr[n_train:, 2:5, 3:9] = [250, 10, 90]
    say("training length", n_train)
    p = gpu_params(C, W, H, K=3)
    mg, ig, sg = run_gpu(C, p, fr, n_train, mode="step")
    mo, io, so = run_orc(orc_params_like(p), fr, n_train)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so, keys=KEYS + ("gkey",)) == 0
    assert sum(i["n_fg"] for i in io) > 0
    if n_train == 65536:
        assert int(so["cnt"].max()) == 65535
