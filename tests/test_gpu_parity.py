"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every test feeds the same seeded synthetic frames to both sides and compares
masks, per-frame level statistics and the canonical model state against the
bar: state within 1e-5 relative, masks differing on at most 1e-4 of pixels.
"""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import canon
from tests.gpu_util import (compare_infos, compare_masks, compare_state, gpu_params,
                            orc_params_like, run_gpu, run_orc, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09339_amd import cog
    return cog


def small_stream(w=160, h=120, frames=200, n_train=50, **kw):
    spec = synth.preset("surveil-160x120-k3").with_(width=w, height=h, frames=frames,
                                                    n_train=n_train, **kw)
    return synth.make_stream(spec)


# ------------------------------------------------------------------ training

def test_train_parity_160x120(C):
    fr = small_stream()
    p = gpu_params(C, 160, 120, K=3)
    say("train 160x120 K=3 N=50")
    _, _, sg = run_gpu(C, p, fr[:51], 50, mode="step", infos=False)
    _, _, so = run_orc(orc_params_like(p), fr[:51], 50)
    nb = compare_state(sg, so)
    assert nb == 0, f"{nb} floats differ in their bits"


@pytest.mark.parametrize("h", [2.0, 8.0, 14.0, 24.0, 64.0])
def test_train_parity_kernel_bandwidths(C, h):
    """Kernel bandwidths from narrow (a level's weight in one or two bins) to
    wide (weights over every bin): the prior tables, counts and the whole
    state equal the oracle's."""
    fr = small_stream()
    p = gpu_params(C, 160, 120, K=3, kde_h=h)
    say("train 160x120 K=3 N=50, kde_h", h)
    _, _, sg = run_gpu(C, p, fr[:51], 50, mode="step", infos=False)
    _, _, so = run_orc(orc_params_like(p), fr[:51], 50)
    assert compare_state(sg, so) == 0


# ------------------------------------------------------------------ cascade

def test_cascade_per_frame_parity_160x120(C):
    fr = small_stream()
    p = gpu_params(C, 160, 120, K=3)
    say("cascade per-frame 160x120 K=3, 150 steps")
    mg, ig, sg = run_gpu(C, p, fr, 50, mode="step")
    mo, io, so = run_orc(orc_params_like(p), fr, 50)
    compare_masks(mg, mo)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so) == 0
    # the cascade is exercised: every level decides some pixels
    tot = np.array([[i["n0"], i["n1"], i["n2"], i["n3"]] for i in io]).sum(0)
    assert (tot[1:] > 0).all(), tot


def test_multi_frame_launch_equals_per_frame(C):
    fr = small_stream(frames=140, n_train=40)
    p = gpu_params(C, 160, 120, K=3)
    say("cascade multi-frame vs per-frame 160x120")
    m1, i1, s1 = run_gpu(C, p, fr, 40, mode="step")
    m2, i2, s2 = run_gpu(C, p, fr, 40, mode="frames")
    m3, i3, s3 = run_gpu(C, p, fr, 40, mode=7)
    assert np.array_equal(m1, m2) and np.array_equal(m1, m3)
    compare_infos(i1, i2)
    compare_infos(i1, i3)
    for k in ("gmm", "rga", "label", "prev"):
        assert np.array_equal(s1[k], s2[k]) and np.array_equal(s1[k], s3[k]), k


@pytest.mark.parametrize("tile", [64, 128, 256, 512, 1024])
def test_tile_size_invariance(C, tile):
    fr = small_stream(w=97, h=61, frames=90, n_train=30)
    p = gpu_params(C, 97, 61, K=3, tile_px=tile)
    say("tile", tile)
    mg, ig, sg = run_gpu(C, p, fr, 30, mode="frames")
    mo, io, so = run_orc(orc_params_like(p), fr, 30)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so) == 0


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_K(C, K):
    fr = small_stream(w=40, h=27, frames=80, n_train=20)
    p = gpu_params(C, 40, 27, K=K)
    say("K", K)
    mg, ig, sg = run_gpu(C, p, fr, 20, mode="frames")
    mo, io, so = run_orc(orc_params_like(p), fr, 20)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so) == 0


@pytest.mark.parametrize("shape", [(37, 23, 3, 4), (50, 31, 1, 2), (1, 1, 3, 3), (63, 1, 3, 5),
                                   (65, 1, 1, 3)])
def test_ragged_shapes_and_single_channel(C, shape):
    w, h, c, K = shape
    fr = small_stream(w=max(w, 16), h=max(h, 16), frames=60, n_train=15)
    fr = fr[:, :h, :w, :c].copy()
    p = gpu_params(C, w, h, c=c, K=K)
    say("shape", shape)
    mg, ig, sg = run_gpu(C, p, fr, 15, mode="step")
    mo, io, so = run_orc(orc_params_like(p), fr, 15)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so) == 0


def test_f32_latent_input(C):
    """64-channel latent maps flattened to independent C=1 pixels (§3.3)."""
    rng = np.random.default_rng(170509343)
    T, N, H, W = 60, 20, 30 * 8, 40
    base = rng.normal(0, 1, size=(H, W, 1)).astype(np.float32)
    drift = rng.normal(0, 0.02, size=(H, W, 1)).astype(np.float32)
    fr = np.stack([base + drift * t + rng.normal(0, 0.1, size=(H, W, 1)).astype(np.float32)
                   for t in range(T)])
    fr[40:, 100:140, 10:20] += 3.0
    p = gpu_params(C, W, H, c=1, K=3, dtype=C.COG_F32, in_lo=-4.0, in_hi=4.0,
                   var_init=0.25, var_min=0.0025, res_e1=0.2, res_e2=0.6, tau_fd=0.0)
    say("f32 latent", fr.shape)
    mo, io, so = run_orc(orc_params_like(p), fr, N)
    for mode in ("frames", "step"):
        mg, ig, sg = run_gpu(C, p, fr, N, mode=mode)
        assert np.array_equal(mg, mo), mode
        compare_infos(ig, io)
        assert compare_state(sg, so) == 0, mode


# ------------------------------------------------------------------ baseline and identity

def test_plain_gmm_path_parity(C):
    fr = small_stream(frames=120, n_train=30)
    p = gpu_params(C, 160, 120, K=3, path=C.COG_PATH_GMM)
    say("plain GMM path 160x120")
    mg, ig, sg = run_gpu(C, p, fr, 30, mode="frames")
    mo, _, so = run_orc(orc_params_like(p), fr, 30, mode="gmm")
    assert np.array_equal(mg, mo)
    assert compare_state(sg, so, keys=("gmm", "label", "prev")) == 0
    for i, m in zip(ig, mg):
        assert i["n3"] == 19200 and i["n_fg"] == int((m == 255).sum())


def test_plain_gmm_path_parity_640x480_full_frame(C):
    """The baseline mixture kernel (its own 64-pixel field-major layout) on a
    full 640x480 stream, every pixel against the oracle, in one launch and
    frame by frame."""
    spec = synth.preset("surveil-640x480-k5")
    N = spec.n_train
    fr = synth.make_stream(spec, 0, N + 60, threads=16)
    p = gpu_params(C, 640, 480, K=5, path=C.COG_PATH_GMM)
    say("plain GMM path 640x480, 60 steps")
    mo, _, so = run_orc(orc_params_like(p), fr, N, mode="gmm")
    for mode in ("frames", "step"):
        mg, ig, sg = run_gpu(C, p, fr, N, mode=mode, infos=mode == "frames")
        assert np.array_equal(mg, mo), mode
        assert compare_state(sg, so, keys=("gmm", "label", "prev")) == 0
        if mode == "frames":
            for i, m in zip(ig, mg):
                assert i["n3"] == 640 * 480 and i["n_fg"] == int((m == 255).sum())


def test_forced_on_identity_cascade_equals_plain_gmm(C):
    fr = small_stream(frames=120, n_train=30)
    p1 = gpu_params(C, 160, 120, K=3, stage_mask=0, kappa_alpha=0.0)
    p2 = gpu_params(C, 160, 120, K=3, path=C.COG_PATH_GMM)
    say("forced-on identity")
    m1, _, s1 = run_gpu(C, p1, fr, 30, mode="step")
    m2, _, s2 = run_gpu(C, p2, fr, 30, mode="step")
    assert np.array_equal(m1, m2)
    assert np.array_equal(s1["gmm"].view(np.uint32), s2["gmm"].view(np.uint32))


def test_illumination_flag(C):
    N = 12
    seq = [100] * N + [101, 101, 161, 161]
    fr = np.stack([np.full((8, 8, 3), s, np.uint8) for s in seq])
    p = gpu_params(C, 8, 8, K=3)
    say("illumination")
    _, ig, _ = run_gpu(C, p, fr, N, mode="step")
    assert [i["illum_flag"] for i in ig] == [0, 0, 1, 0]
    assert [i["n0"] for i in ig] == [0, 64, 0, 64]


# ------------------------------------------------------------------ full sizes, sampled

def _sample_pixels(H, W, seed):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(H * W, size=4000, replace=False).tolist())
    # plus two dense 64x8 blocks (several tiles, foreground-rich rows)
    for (y0, x0) in ((H // 3, W // 4), (2 * H // 3, W // 2)):
        for y in range(y0, y0 + 8):
            idx.update(range(y * W + x0, y * W + x0 + 64))
    return np.array(sorted(idx))


@pytest.mark.parametrize("name,n_steps", [("surveil-640x480-k5", 60),
                                          ("surveil-1920x1080-k5-occ01", 100),
                                          ("surveil-1920x1080-k5-occ05", 120),
                                          ("surveil-1920x1080-k5-occ10", 100),
                                          ("surveil-1920x1080-k5-occ30", 100)])
def test_full_size_sampled_parity(C, name, n_steps):
    """The full-size streams through one multi-frame launch (the regime the
    benchmark times) against the oracle on sampled pixels' time series."""
    spec = synth.preset(name)
    N = spec.n_train
    fr = synth.make_stream(spec, 0, N + n_steps, threads=16)
    p = gpu_params(C, spec.width, spec.height, K=spec.K)
    say("full size", name, "steps", n_steps)
    mg, ig, sg = run_gpu(C, p, fr, N, mode="frames")
    P = spec.pixels
    # whole-frame properties
    w = sg["gmm"][:, :, 0].astype(np.float64)
    assert np.abs(w.sum(1) - 1).max() <= spec.K * 2.0 ** -23
    assert (sg["gmm"][:, :, -1] >= np.float32(12.0)).all() and (sg["rga"][:, -1] >= 12.0).all()
    assert set(np.unique(mg)) <= {0, 255}
    for i, m in zip(ig, mg):
        assert i["n0"] + i["n1"] + i["n2"] + i["n3"] == P
        assert i["n_fg"] == int((m == 255).sum())
    # sampled pixels against the oracle on the same pixels' time series
    pix = _sample_pixels(spec.height, spec.width, spec.seed)
    sub = fr.reshape(len(fr), P, 3)[:, pix][:, None]
    po = orc_params_like(p)
    po.width, po.height = len(pix), 1
    mo, _, so = run_orc(po, sub, N)
    compare_masks(mg[:, pix], mo)
    assert np.array_equal(mg[:, pix], mo)
    assert compare_state(sg, so, pix=pix) == 0


@pytest.mark.parametrize("name,n_steps", [("surveil-1920x1080-k5-occ05", 30),
                                          ("surveil-1920x1080-k5-occ30", 30)])
def test_full_size_per_frame_sampled_parity(C, name, n_steps):
    """The live-camera regime at 1920x1080: one cog_step per frame (the
    per-frame kernel with compacted survivors), the per-frame statistics
    checked on the whole frame and the sampled pixels against the oracle."""
    spec = synth.preset(name)
    N = spec.n_train
    fr = synth.make_stream(spec, 0, N + n_steps, threads=16)
    p = gpu_params(C, spec.width, spec.height, K=spec.K)
    say("full size per frame", name, "steps", n_steps)
    mg, ig, sg = run_gpu(C, p, fr, N, mode="step")
    P = spec.pixels
    for i, m in zip(ig, mg):
        assert i["n0"] + i["n1"] + i["n2"] + i["n3"] == P
        assert i["n_fg"] == int((m == 255).sum())
    pix = _sample_pixels(spec.height, spec.width, spec.seed)
    sub = fr.reshape(len(fr), P, 3)[:, pix][:, None]
    po = orc_params_like(p)
    po.width, po.height = len(pix), 1
    mo, _, so = run_orc(po, sub, N)
    assert np.array_equal(mg[:, pix], mo)
    assert compare_state(sg, so, pix=pix) == 0
    # the same frames through one multi-frame launch give the same result
    mf, i_f, sf = run_gpu(C, p, fr, N, mode="frames")
    assert np.array_equal(mf, mg)
    compare_infos(i_f, ig)
    for k in ("gmm", "rga", "label", "prev"):
        assert np.array_equal(sf[k], sg[k]), k


# ------------------------------------------------------------------ boundary behaviour

def test_export_import_resume_is_bitwise(C):
    import torch
    fr = small_stream(frames=130, n_train=30)
    p = gpu_params(C, 160, 120, K=3)
    say("export/import resume")
    m_full, i_full, s_full = run_gpu(C, p, fr, 30, mode="step")
    dev = torch.from_numpy(fr).cuda()
    a = C.CogStream(p, stream=torch.cuda.current_stream())
    a.train_prior(dev[:30])
    a.step_frames(dev[30:80])
    blob = a.export_state()
    a.close()
    b = C.CogStream(p, stream=torch.cuda.current_stream())
    b.import_state(blob)
    masks = torch.zeros((50, 19200), dtype=torch.uint8, device="cuda")
    infos = b.step_frames(dev[80:130], masks, want_info=True)
    st = canon.parse(b.export_state())
    b.close()
    assert np.array_equal(masks.cpu().numpy(), m_full[50:])
    compare_infos(infos, i_full[50:])
    for k in ("gmm", "rga", "table", "cnt", "label", "prev"):
        assert np.array_equal(st[k], s_full[k]), k
    assert st["frame"] == 130


def test_host_pointers_equal_device_pointers(C):
    fr = small_stream(w=64, h=40, frames=70, n_train=20)
    p = gpu_params(C, 64, 40, K=3)
    say("host pointers")
    mg, ig, sg = run_gpu(C, p, fr, 20, mode="frames")
    s = C.CogStream(p)
    s.train_prior(fr[:20])
    masks = np.zeros((50, 64 * 40), np.uint8)
    infos = s.step_frames(fr[20:], masks, want_info=True)
    st = canon.parse(s.export_state())
    s.close()
    assert np.array_equal(masks, mg)
    compare_infos(infos, ig)
    assert np.array_equal(st["gmm"], sg["gmm"])


def test_call_order_and_buffer_errors(C):
    import torch
    p = gpu_params(C, 32, 32, K=3)
    fr = torch.from_numpy(small_stream(w=32, h=32, frames=12, n_train=10)).cuda()
    s = C.CogStream(p, stream=torch.cuda.current_stream())
    with pytest.raises(C.CogError) as ei:
        s.step(fr[0])
    assert ei.value.status == C.COG_E_STATE
    with pytest.raises(C.CogError) as ei:
        C.cog_train_prior(s.h, fr[:1])
    assert ei.value.status == C.COG_E_INVALID
    s.train_prior(fr[:10])
    with pytest.raises(C.CogError) as ei:
        s.train_prior(fr[:10])
    assert ei.value.status == C.COG_E_STATE
    s.step(fr[10])
    s.reset()
    with pytest.raises(C.CogError):
        s.step(fr[11])
    s.close()
    need = C.cog_state_bytes(p)
    small = torch.zeros(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(C.CogError) as ei:
        C.cog_create(p, device_state=small)
    assert ei.value.status == C.COG_E_OOM


def test_caller_owned_state_buffer(C):
    import torch
    fr = small_stream(w=48, h=30, frames=60, n_train=20)
    p = gpu_params(C, 48, 30, K=3)
    say("caller-owned state")
    buf = torch.zeros(C.cog_state_bytes(p), dtype=torch.uint8, device="cuda")
    s = C.CogStream(p, stream=torch.cuda.current_stream(), device_state=buf)
    dev = torch.from_numpy(fr).cuda()
    s.train_prior(dev[:20])
    masks = torch.zeros((40, 48 * 30), dtype=torch.uint8, device="cuda")
    s.step_frames(dev[20:], masks)
    st = canon.parse(s.export_state())
    s.close()
    mo, _, so = run_orc(orc_params_like(p), fr, 20)
    assert np.array_equal(masks.cpu().numpy(), mo)
    assert compare_state(st, so) == 0
