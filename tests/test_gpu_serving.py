"""Serving loop (cog_server_*): continuous batching of many streams.

Frames of several streams arrive at seeded Poisson times from a submitting
thread while the scheduler batches whatever is queued; streams open while
others run.  Every stream's masks and final state must equal, bit for bit,
the same frames run alone through cog_step_frames; every submission must
complete exactly once, in order within its stream.  Admission by the HBM
budget, reuse of closed streams' buffers and the error paths are checked
too.
"""
import threading
import time

import numpy as np
import pytest

import synth
from tests import canon
from tests.gpu_util import compare_masks, compare_state, gpu_params, orc_params_like, run_orc, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09339_amd import cog
    return cog


def _synth(w, h, frames, seed_off):
    spec = synth.preset("surveil-160x120-k3").with_(width=w, height=h, frames=frames, n_train=20,
                                                    seed=synth.video.BASE_SEED + 700 + seed_off)
    return synth.make_stream(spec)


def stream_set(C):
    """(name, params, frames [T, ...]); the first 20 frames train."""
    lat = synth.latent_stream(70, channels=4, h=8, w=6, seed=synth.video.BASE_SEED + 790)
    return [
        ("u8c3k5-48x32", gpu_params(C, 48, 32, c=3, K=5), _synth(48, 32, 70, 1)),
        ("u8c3k3-40x24", gpu_params(C, 40, 24, c=3, K=3), _synth(40, 24, 60, 2)),
        ("u8c3k5-21x13", gpu_params(C, 21, 13, c=3, K=5), _synth(21, 13, 66, 3)),
        ("u8c1k2-30x20", gpu_params(C, 30, 20, c=1, K=2),
         np.ascontiguousarray(_synth(30, 20, 55, 4)[..., :1])),
        ("f32c1k3-latent", gpu_params(C, 192, 1, c=1, K=3, dtype=1, in_lo=-5.0, in_hi=5.0),
         lat.reshape(70, 192, 1)),
    ]


def alone(C, p, dev, n_train):
    import torch
    T = dev.shape[0] - n_train
    masks = torch.zeros((T, p.width * p.height), dtype=torch.uint8, device="cuda")
    s = C.CogStream(p, stream=torch.cuda.current_stream())
    s.train_prior(dev[:n_train])
    s.step_frames(dev[n_train:], masks)
    torch.cuda.synchronize()
    st = s.export_state()
    s.close()
    return masks.cpu().numpy(), st


def test_serving_mix_equals_alone(C):
    import torch
    streams = stream_set(C)
    devs = [torch.from_numpy(np.ascontiguousarray(fr)).cuda() for _, _, fr in streams]
    torch.cuda.synchronize()
    ref = [alone(C, p, d, 20) for (_, p, _), d in zip(streams, devs)]
    masks = [torch.zeros((d.shape[0] - 20, p.width * p.height), dtype=torch.uint8, device="cuda")
             for (_, p, _), d in zip(streams, devs)]
    torch.cuda.synchronize()
    srv = C.CogServer(hbm_budget=1 << 30, max_streams=8, depth=2)
    rng = np.random.default_rng(7)
    # submissions: (arrival time s, stream, first frame, n frames); streams 3
    # and 4 open only after the others have run for a while
    subs = []
    for i, (_, p, fr) in enumerate(streams):
        t = 0.0 if i < 3 else 0.004
        f = 0
        T = len(fr) - 20
        while f < T:
            n = int(min(T - f, rng.choice([1, 1, 1, 2, 3])))
            t += float(rng.exponential(0.0001))
            subs.append((t, i, f, n))
            f += n
    subs.sort()
    ids = {}
    tags = {}
    say("serving: %d submissions over %d streams" % (len(subs), len(streams)))
    t_start = time.perf_counter()
    for t, i, f, n in subs:
        while time.perf_counter() - t_start < t:
            pass
        if i not in ids:
            ids[i] = srv.open(streams[i][1], devs[i][:20])
        tag = len(tags)
        tags[tag] = (i, f, n)
        srv.submit(ids[i], devs[i][20 + f:20 + f + n], masks[i][f:f + n], tag=tag, nframes=n)
    srv.drain()
    comps = srv.poll(max_n=len(subs) + 10)
    assert len(comps) == len(subs)
    assert all(c["status"] == 0 for c in comps)
    assert sorted(c["tag"] for c in comps) == list(range(len(subs)))
    for i in range(len(streams)):
        mine = [c["tag"] for c in comps if c["stream_id"] == ids[i]]
        assert mine == sorted(mine), "completions out of order within a stream"
        assert all(c["t_done_us"] >= c["t_submit_us"] for c in comps)
    st = srv.stats()
    say("serving stats", st)
    assert st["frames"] == sum(len(fr) - 20 for _, _, fr in streams)
    assert st["ticks"] < len(subs), "no batching happened"
    states = {i: srv.export_state(ids[i]) for i in ids}
    for i in ids:
        srv.close_stream(ids[i])
    srv.close()
    for i, (name, p, fr) in enumerate(streams):
        mg = masks[i].cpu().numpy()
        assert np.array_equal(mg, ref[i][0]), (name, int((mg != ref[i][0]).sum()))
        assert states[i] == ref[i][1], (name, "state differs")
        # and each served stream against the oracle directly
        mo, _, so = run_orc(orc_params_like(p), fr, 20)
        compare_masks(mg, mo)
        assert np.array_equal(mg, mo), (name, int((mg != mo).sum()))
        assert compare_state(canon.parse(states[i]), so) == 0, name


def test_admission_by_budget_and_pool_reuse(C):
    import torch
    fr = torch.from_numpy(_synth(32, 32, 24, 5)).cuda()
    small_fr = fr[:20, :8, :8].contiguous()
    torch.cuda.synchronize()  # the server reads them on its own stream
    p = gpu_params(C, 32, 32, c=3, K=5)
    nb = C.cog_state_bytes(p)
    srv = C.CogServer(hbm_budget=int(nb * 2.5), max_streams=3, depth=2)
    a = srv.open(p, fr[:20])
    b = srv.open(p, fr[:20])
    with pytest.raises(C.CogError) as e:
        srv.open(p, fr[:20])
    assert e.value.status == C.COG_E_OOM
    st = srv.stats()
    assert st["streams_open"] == 2 and st["streams_rejected"] == 1
    assert st["bytes_in_use"] == 2 * nb and st["bytes_allocated"] >= int(nb * 2.5)
    assert st["bytes_largest_free"] < nb
    srv.close_stream(a)
    assert srv.stats()["bytes_largest_free"] == nb  # a's range, not merged across b
    c = srv.open(p, fr[:20])  # reuses a's range
    st = srv.stats()
    assert st["bytes_in_use"] == 2 * nb and st["streams_open"] == 2
    # a smaller stream fits beside them
    small = gpu_params(C, 8, 8, c=3, K=3)
    d = srv.open(small, small_fr)
    with pytest.raises(C.CogError) as e:  # max_streams reached
        srv.open(small, small_fr)
    assert e.value.status == C.COG_E_OOM
    for sid in (b, c, d):
        srv.close_stream(sid)
    st = srv.stats()
    assert st["streams_open"] == 0 and st["bytes_in_use"] == 0
    assert st["bytes_largest_free"] == st["bytes_allocated"]  # every range merged back
    srv.close()


def test_close_before_training_then_destroy(C):
    """Streams closed right after admission, before the scheduler has issued
    their training slices, leave stale entries in the training queue; the
    server must still shut down.  Each round opens a stream needing several
    slices and one needing one, closes both at once, checks that nothing
    remains open and destroys the server."""
    import torch
    big = torch.zeros((20, 600, 1024, 3), dtype=torch.uint8, device="cuda")  # 3 slices
    small = torch.from_numpy(_synth(16, 8, 20, 9)).cuda()
    torch.cuda.synchronize()
    pb = gpu_params(C, 1024, 600, c=3, K=3)
    ps = gpu_params(C, 16, 8, c=3, K=3)
    for r in range(8):
        say("close before training, round", r)
        srv = C.CogServer(hbm_budget=2 * C.cog_state_bytes(pb), max_streams=4)
        a = srv.open(pb, big)
        b = srv.open(ps, small)
        srv.close_stream(b)
        srv.close_stream(a)
        st = srv.stats()
        assert st["streams_open"] == 0 and st["bytes_in_use"] == 0
        srv.close()


def test_close_with_pending_frames_and_errors(C):
    import torch
    fr = torch.from_numpy(_synth(24, 16, 40, 6)).cuda()
    masks = torch.zeros((20, 24 * 16), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()  # the server reads them on its own stream
    p = gpu_params(C, 24, 16, c=3, K=3)
    srv = C.CogServer(hbm_budget=1 << 28, max_streams=4)
    sid = srv.open(p, fr[:20])
    for k in range(20):
        srv.submit(sid, fr[20 + k:21 + k], masks[k:k + 1], tag=k)
    srv.close_stream(sid)  # queued frames still complete
    srv.drain()
    comps = srv.poll()
    assert [c["tag"] for c in comps] == list(range(20))
    assert srv.stats()["streams_open"] == 0
    with pytest.raises(C.CogError) as e:
        srv.submit(sid, fr[20:21], None, tag=99)
    assert e.value.status == C.COG_E_INVALID
    with pytest.raises(C.CogError):
        srv.export_state(sid)
    sid2 = srv.open(p, fr[:20])
    for bad in (0, 65):
        with pytest.raises(C.CogError) as e:
            srv.submit(sid2, fr[20:21], None, tag=0, nframes=bad)
        assert e.value.status == C.COG_E_INVALID
    with pytest.raises(C.CogError) as e:
        srv.open(gpu_params(C, 24, 16, c=3, K=3, path=1), fr[:20])
    assert e.value.status == C.COG_E_UNSUPPORTED
    with pytest.raises(C.CogError) as e:
        srv.open(gpu_params(C, 24, 16, c=3, K=3, tile_px=128), fr[:20])
    assert e.value.status == C.COG_E_UNSUPPORTED
    # the stream after the failures still serves
    srv.submit(sid2, fr[20:22], masks[:2], tag=5, nframes=2)
    srv.drain(sid2)
    assert [c["tag"] for c in srv.poll(wait_us=1000)] == [5]
    srv.close()


def test_concurrent_submitters_and_poller(C):
    """Two submitting threads and a polling thread on one server."""
    import torch
    streams = stream_set(C)[:2]
    devs = [torch.from_numpy(np.ascontiguousarray(fr)).cuda() for _, _, fr in streams]
    torch.cuda.synchronize()
    ref = [alone(C, p, d, 20) for (_, p, _), d in zip(streams, devs)]
    masks = [torch.zeros((d.shape[0] - 20, p.width * p.height), dtype=torch.uint8, device="cuda")
             for (_, p, _), d in zip(streams, devs)]
    torch.cuda.synchronize()
    srv = C.CogServer(hbm_budget=1 << 28, max_streams=4, depth=3)
    ids = [srv.open(p, d[:20]) for (_, p, _), d in zip(streams, devs)]
    got = []
    stop = threading.Event()

    def poller():
        while not stop.is_set():
            got.extend(srv.poll(wait_us=2000))

    def submitter(i):
        T = devs[i].shape[0] - 20
        for f in range(T):
            srv.submit(ids[i], devs[i][20 + f:21 + f], masks[i][f:f + 1], tag=i * 1000 + f)

    th = [threading.Thread(target=poller)] + [threading.Thread(target=submitter, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th[1:]:
        t.join()
    srv.drain()
    stop.set()
    th[0].join()
    got.extend(srv.poll())
    assert len(got) == sum(d.shape[0] - 20 for d in devs)
    states = [srv.export_state(s) for s in ids]
    srv.close()
    for i in range(2):
        assert np.array_equal(masks[i].cpu().numpy(), ref[i][0])
        assert states[i] == ref[i][1]


def test_serving_full_size_streams_equal_alone(C):
    """A 1920x1080 and a 640x480 stream (K=5) served together, one frame per
    submission, the second admitted while the first runs: masks and state
    equal each stream alone, bit for bit."""
    import torch
    specs = [(1920, 1080, 32, 21), (640, 480, 40, 22)]
    streams = [(gpu_params(C, w, h, c=3, K=5), _synth(w, h, n, s)) for w, h, n, s in specs]
    devs = [torch.from_numpy(np.ascontiguousarray(fr)).cuda() for _, fr in streams]
    torch.cuda.synchronize()
    ref = [alone(C, p, d, 20) for (p, _), d in zip(streams, devs)]
    masks = [torch.zeros((d.shape[0] - 20, p.width * p.height), dtype=torch.uint8, device="cuda")
             for (p, _), d in zip(streams, devs)]
    torch.cuda.synchronize()
    srv = C.CogServer(hbm_budget=4 << 30, max_streams=4, depth=2)
    ids = {0: srv.open(streams[0][0], devs[0][:20])}
    nxt = {0: 0}  # next frame of each stream (after its training frames)
    tag = 0
    for step in range(max(d.shape[0] for d in devs) - 20 + 3):
        if step == 3:
            ids[1] = srv.open(streams[1][0], devs[1][:20])
            nxt[1] = 0
        for i in ids:
            f = nxt[i]
            if f < devs[i].shape[0] - 20:
                srv.submit(ids[i], devs[i][20 + f:21 + f], masks[i][f:f + 1], tag=tag, nframes=1)
                nxt[i] = f + 1
                tag += 1
    srv.drain()
    comps = srv.poll(max_n=tag + 8)
    assert len(comps) == tag and all(c["status"] == 0 for c in comps)
    states = {i: srv.export_state(ids[i]) for i in ids}
    for i in ids:
        srv.close_stream(ids[i])
    srv.close()
    for i in range(2):
        mg = masks[i].cpu().numpy()
        assert np.array_equal(mg, ref[i][0]), i
        assert states[i] == ref[i][1], i
        p, fr = streams[i]
        say("served full-size stream against the oracle", p.width, p.height)
        mo, _, so = run_orc(orc_params_like(p), fr, 20)
        compare_masks(mg, mo)
        assert np.array_equal(mg, mo), (i, int((mg != mo).sum()))
        assert compare_state(canon.parse(states[i]), so) == 0, i


def _sample_pixels(H, W, seed, n=3000):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(H * W, size=n, replace=False).tolist())
    for (y0, x0) in ((H // 3, W // 4), (2 * H // 3, W // 2)):
        for y in range(y0, y0 + 4):
            idx.update(range(y * W + x0, y * W + x0 + 128))
    return np.array(sorted(idx))


def test_serving_4k_stream_sampled_against_oracle(C):
    """A 3840x2160 stream served one frame per submission beside a 640x480
    stream admitted while it runs: the 4K stream's masks and state on sampled
    pixels, and the small stream in full, against the oracle."""
    import torch
    spec4 = synth.preset("surveil-1920x1080-k5-occ05").with_(width=3840, height=2160, frames=36,
                                                             n_train=20)
    fr4 = synth.make_stream(spec4, threads=16)
    p4 = gpu_params(C, 3840, 2160, c=3, K=5)
    fr1 = _synth(640, 480, 40, 31)
    p1 = gpu_params(C, 640, 480, c=3, K=5)
    devs = [torch.from_numpy(fr4).cuda(), torch.from_numpy(fr1).cuda()]
    masks = [torch.zeros((d.shape[0] - 20, d.shape[1] * d.shape[2]), dtype=torch.uint8, device="cuda")
             for d in devs]
    torch.cuda.synchronize()
    srv = C.CogServer(hbm_budget=8 << 30, max_streams=4, depth=2)
    ids = {0: srv.open(p4, devs[0][:20])}
    nxt = {0: 0}
    tag = 0
    for step in range(24):
        if step == 2:
            ids[1] = srv.open(p1, devs[1][:20])
            nxt[1] = 0
        for i in ids:
            f = nxt[i]
            if f < devs[i].shape[0] - 20:
                srv.submit(ids[i], devs[i][20 + f:21 + f], masks[i][f:f + 1], tag=tag, nframes=1)
                nxt[i] = f + 1
                tag += 1
    srv.drain()
    comps = srv.poll(max_n=tag + 8)
    assert len(comps) == tag and all(c["status"] == 0 for c in comps)
    states = {i: srv.export_state(ids[i]) for i in ids}
    for i in ids:
        srv.close_stream(ids[i])
    srv.close()
    m4 = masks[0].cpu().numpy()
    P = 3840 * 2160
    pix = _sample_pixels(2160, 3840, spec4.seed)
    sub = fr4.reshape(len(fr4), P, 3)[:, pix][:, None]
    po = orc_params_like(p4)
    po.width, po.height = len(pix), 1
    say("4K served stream against the oracle on", len(pix), "pixels")
    mo, _, so = run_orc(po, sub, 20)
    assert np.array_equal(m4[:, pix], mo), int((m4[:, pix] != mo).sum())
    assert compare_state(canon.parse(states[0]), so, pix=pix) == 0
    assert set(np.unique(m4)) <= {0, 255}
    del m4, states[0]
    m1 = masks[1].cpu().numpy()
    mo, _, so = run_orc(orc_params_like(p1), fr1, 20)
    assert np.array_equal(m1, mo), int((m1 != mo).sum())
    assert compare_state(canon.parse(states[1]), so) == 0


def test_drain_waits_for_training(C):
    """A stream with nothing submitted: cog_server_drain returns after its
    training, so the training frames may be overwritten then; its results still
    equal the alone run's.  A stream closed while it may still train gives its
    range back only after the training."""
    import torch
    fr = torch.from_numpy(_synth(64, 48, 40, 8)).cuda()
    p = gpu_params(C, 64, 48, c=3, K=5)
    ref_masks, ref_state = alone(C, p, fr, 20)
    train = fr[:20].clone()
    torch.cuda.synchronize()
    srv = C.CogServer(hbm_budget=int(C.cog_state_bytes(p) * 1.5), max_streams=4)
    gone = srv.open(p, train)
    srv.close_stream(gone)          # its range returns after its training
    sid = srv.open(p, train)        # and is reused here
    srv.drain(sid)
    train.zero_()                   # the training has read its frames
    torch.cuda.synchronize()
    masks = torch.zeros((20, 64 * 48), dtype=torch.uint8, device="cuda")
    for k in range(20):
        srv.submit(sid, fr[20 + k:21 + k], masks[k:k + 1], tag=k)
    srv.drain(sid)
    assert [c["tag"] for c in srv.poll()] == list(range(20))
    assert np.array_equal(masks.cpu().numpy(), ref_masks)
    assert srv.export_state(sid) == ref_state
    srv.close()
