"""Parity of the sampling variant (confidence-based spatio-temporal sampling,
COG_STAGE_SAMPLE) of the HIP cascade with the oracle, through the C ABI:
masks, per-frame statistics (with the halted-pixel count) and the canonical
state including the saturation counters, bit for bit."""
import numpy as np
import pytest

import synth
from tests import canon
from tests.gpu_util import (compare_infos, compare_masks, compare_state, gpu_params,
                            orc_params_like, run_gpu, run_orc, say)

pytestmark = pytest.mark.gpu

SAMP = 8
KEYS = ("gmm", "rga", "table", "cnt", "label", "prev", "sat")


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09339_amd import cog
    return cog


def stream(w, h, frames, n_train, seed_off=0, **kw):
    spec = synth.preset("surveil-160x120-k3").with_(width=w, height=h, frames=frames,
                                                    n_train=n_train,
                                                    seed=synth.video.BASE_SEED + 900 + seed_off, **kw)
    return synth.make_stream(spec)


def sampled(C, w, h, c=3, K=3, **kw):
    base = dict(stage_mask=7 | SAMP, samp_window=8, samp_period=4)
    base.update(kw)
    return gpu_params(C, w, h, c=c, K=K, **base)


@pytest.mark.parametrize("mode", ["step", "frames", 7])
def test_sampling_parity_160x120(C, mode):
    fr = stream(160, 120, 200, 50)
    p = sampled(C, 160, 120)
    say("sampling 160x120 mode", mode)
    mg, ig, sg = run_gpu(C, p, fr, 50, mode=mode)
    mo, io, so = run_orc(orc_params_like(p), fr, 50)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so, keys=KEYS) == 0
    skipped = sum(i["n_skip"] for i in io)
    assert skipped > 0.2 * 160 * 120 * 150, "sampling halted too little to test"


@pytest.mark.parametrize("w,h,c,K,window,period,lam", [
    (37, 23, 3, 5, 4, 3, 2.5),   # ragged last block
    (50, 21, 1, 2, 6, 2, 1.0),   # single channel, tighter confidence gate
    (9, 5, 3, 4, 3, 5, 0.7),     # less than one block, the paper's 0.7 sigma
])
def test_sampling_parity_ragged(C, w, h, c, K, window, period, lam):
    fr = stream(w, h, 120, 20, seed_off=w)
    if c == 1:
        fr = np.ascontiguousarray(fr[..., :1])
    p = sampled(C, w, h, c=c, K=K, samp_window=window, samp_period=period, samp_lambda=lam)
    mg, ig, sg = run_gpu(C, p, fr, 20, mode=5)
    mo, io, so = run_orc(orc_params_like(p), fr, 20)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so, keys=KEYS) == 0


def test_sampling_parity_f32_latent(C):
    lat = synth.latent_stream(90, channels=8, h=12, w=10, seed=synth.video.BASE_SEED + 950)
    fr = lat.reshape(90, 960, 1)
    p = sampled(C, 960, 1, c=1, K=3, dtype=1, in_lo=-5.0, in_hi=5.0, samp_window=5,
                samp_period=3, samp_lambda=2.0)
    mg, ig, sg = run_gpu(C, p, fr, 20, mode="frames")
    mo, io, so = run_orc(orc_params_like(p), fr, 20)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so, keys=KEYS) == 0


def test_sampling_parity_640x480_full(C):
    spec = synth.preset("surveil-640x480-k5")
    fr = synth.make_stream(spec, 0, 200)
    p = sampled(C, 640, 480, K=5, samp_window=16, samp_period=4)
    say("sampling 640x480, 100 steps after 100 training frames")
    mg, ig, sg = run_gpu(C, p, fr, 100, mode="frames")
    mo, io, so = run_orc(orc_params_like(p), fr, 100)
    compare_masks(mg, mo)
    assert np.array_equal(mg, mo)
    compare_infos(ig, io)
    assert compare_state(sg, so, keys=KEYS) == 0


def test_sampling_resume_through_export(C):
    import torch
    fr = stream(64, 40, 140, 20, seed_off=3)
    p = sampled(C, 64, 40, samp_window=6, samp_period=3)
    dev = torch.from_numpy(fr).cuda()
    torch.cuda.synchronize()
    a = C.CogStream(p, stream=torch.cuda.current_stream())
    a.train_prior(dev[:20])
    a.step_frames(dev[20:80])
    blob = a.export_state()
    st = canon.parse(blob)
    assert st["version"] == 3 and (st["sat"] > 0).any()
    b = C.CogStream(p, stream=torch.cuda.current_stream())
    b.import_state(blob)
    ma = torch.zeros((60, 64 * 40), dtype=torch.uint8, device="cuda")
    mb = torch.zeros_like(ma)
    ia = a.step_frames(dev[80:], ma, want_info=True)
    ib = b.step_frames(dev[80:], mb, want_info=True)
    torch.cuda.synchronize()
    assert torch.equal(ma, mb) and ia == ib
    assert a.export_state() == b.export_state()
    a.close()
    b.close()


def test_sampling_needs_64_pixel_tiles(C):
    p = sampled(C, 64, 40, tile_px=256)
    with pytest.raises(C.CogError) as e:
        C.CogStream(p)
    assert e.value.status == C.COG_E_UNSUPPORTED


def test_sampling_in_batched_ticks(C):
    """Sampled and unsampled streams of one class (and another class) ticked
    together equal each stream alone."""
    import torch
    S = torch.cuda.Stream()
    specs = [
        (sampled(C, 48, 40, K=5, samp_window=5, samp_period=3), stream(48, 40, 100, 20, 11)),
        (gpu_params(C, 48, 40, K=5), stream(48, 40, 100, 20, 12)),
        (sampled(C, 33, 17, K=3, samp_window=4, samp_period=2), stream(33, 17, 100, 20, 13)),
    ]
    ticks = [1, 4, 8, 2, 9, 3, 7, 16, 1, 5, 13, 11]
    with torch.cuda.stream(S):
        devs = [torch.from_numpy(fr).cuda() for _, fr in specs]
        alone, batched, ctxs = [], [], []
        for (p, fr), d in zip(specs, devs):
            m = torch.zeros((80, p.width * p.height), dtype=torch.uint8, device="cuda")
            s = C.CogStream(p, stream=S)
            s.train_prior(d[:20])
            s.step_frames(d[20:], m)
            S.synchronize()
            alone.append((m.cpu().numpy(), s.export_state()))
            s.close()
        b = C.CogBatch(S, max_items=4)
        masks = []
        for (p, fr), d in zip(specs, devs):
            s = C.CogStream(p, stream=S)
            s.train_prior(d[:20])
            ctxs.append(s)
            masks.append(torch.zeros((80, p.width * p.height), dtype=torch.uint8, device="cuda"))
        off = 0
        for n in ticks:
            b.tick([(c.h, d[20 + off:20 + off + n], m[off:off + n], n, False)
                    for c, d, m in zip(ctxs, devs, masks)])
            off += n
        assert off == 80
        S.synchronize()
        for i, c in enumerate(ctxs):
            assert np.array_equal(masks[i].cpu().numpy(), alone[i][0]), i
            assert c.export_state() == alone[i][1], i
            c.close()
        b.close()
