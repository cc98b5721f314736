"""Batched tick (cog_batch_*): every stream's result in a batch is the same as
alone.

Streams of several classes (RGB u8 with K=5 and K=3, single-channel u8,
f32 latent maps), ragged sizes, uneven lengths, late joins and per-tick
frame counts from 1 to 12 are advanced together, and each stream's masks,
per-frame statistics and exported state must equal, bit for bit, the same
stream run alone through cog_step_frames with the same frame runs (which the
parity tests tie to the oracle).  One stream is also checked against the
oracle directly.
"""
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


@pytest.fixture(scope="module")
def S():
    import torch
    return torch.cuda.Stream()


def _synth(w, h, frames, n_train, seed_off):
    spec = synth.preset("surveil-160x120-k3").with_(width=w, height=h, frames=frames,
                                                    n_train=n_train,
                                                    seed=synth.video.BASE_SEED + 500 + seed_off)
    return synth.make_stream(spec)


def stream_set(C):
    """(name, params, frames [T, ...], n_train, join_tick)."""
    out = []
    fr = _synth(40, 30, 80, 20, 1)
    out.append(("u8c3k5-40x30", gpu_params(C, 40, 30, c=3, K=5), fr, 20, 0))
    fr = _synth(64, 48, 70, 20, 2)
    out.append(("u8c3k3-64x48", gpu_params(C, 64, 48, c=3, K=3), fr, 20, 0))
    fr = _synth(33, 17, 60, 20, 3)
    out.append(("u8c3k5-33x17", gpu_params(C, 33, 17, c=3, K=5), fr, 20, 2))
    fr = np.ascontiguousarray(_synth(50, 20, 75, 20, 4)[..., :1])
    out.append(("u8c1k2-50x20", gpu_params(C, 50, 20, c=1, K=2), fr, 20, 1))
    lat = synth.latent_stream(85, channels=8, h=6, w=5, seed=synth.video.BASE_SEED + 504)
    out.append(("f32c1k3-latent", gpu_params(C, 240, 1, c=1, K=3, dtype=1, in_lo=-5.0, in_hi=5.0),
                lat.reshape(85, 240, 1), 20, 0))
    fr = _synth(7, 3, 40, 20, 5)  # fewer pixels than one tile
    out.append(("u8c3k5-7x3", gpu_params(C, 7, 3, c=3, K=5), fr, 20, 3))
    return out


TICK_FRAMES = [1, 3, 8, 1, 12, 2, 9, 1, 5, 10, 4, 11, 1, 6, 7, 3, 8, 2, 12, 1, 9, 4, 2, 8, 1]
INFO_TICKS = {1, 4, 9}


def tick_plan(streams):
    """Per tick, per stream: (first frame offset after training, nframes)."""
    pos = [0] * len(streams)
    plan = []
    for t, f in enumerate(TICK_FRAMES):
        row = []
        for i, (_, _, fr, n_train, join) in enumerate(streams):
            left = len(fr) - n_train - pos[i]
            k = 0 if t < join else min(f, left)
            row.append((pos[i], k))
            pos[i] += k
        plan.append(row)
    return plan, pos


def run_alone(C, S, streams, plan):
    import torch
    res = []
    with torch.cuda.stream(S):
        for i, (name, p, fr, n_train, _) in enumerate(streams):
            dev = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
            T = len(fr) - n_train
            masks = torch.zeros((max(T, 1), p.width * p.height), dtype=torch.uint8, device="cuda")
            s = C.CogStream(p, stream=S)
            s.train_prior(dev[:n_train])
            infos = {}
            for t, row in enumerate(plan):
                off, k = row[i]
                if k == 0:
                    continue
                r = s.step_frames(dev[n_train + off:n_train + off + k], masks[off:off + k],
                                  want_info=t in INFO_TICKS)
                if r is not None:
                    infos[t] = r
            S.synchronize()
            res.append((masks.cpu().numpy(), infos, s.export_state()))
            s.close()
    return res


def run_batched(C, S, streams, plan, schedules=None, autotune_at=None, max_items=16):
    import torch
    out = []
    with torch.cuda.stream(S):
        devs, masks, ctxs = [], [], []
        for name, p, fr, n_train, _ in streams:
            dev = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
            T = len(fr) - n_train
            m = torch.zeros((max(T, 1), p.width * p.height), dtype=torch.uint8, device="cuda")
            s = C.CogStream(p, stream=S)
            s.train_prior(dev[:n_train])
            devs.append(dev)
            masks.append(m)
            ctxs.append(s)
        b = C.CogBatch(S, max_items=max_items)
        for key, sch in (schedules or {}).items():
            b.set_schedule(*key, **sch)
        infos = [dict() for _ in streams]
        for t, row in enumerate(plan):
            entries, idx = [], []
            for i, (off, k) in enumerate(row):
                n_train = streams[i][3]
                entries.append((ctxs[i].h, devs[i][n_train + off:n_train + off + max(k, 1)],
                                masks[i][off:off + max(k, 1)], k, t in INFO_TICKS))
                idx.append(i)
            if autotune_at is not None and t == autotune_at:
                before = [c.export_state() for c in ctxs]
                best = b.autotune(entries, reps=1)
                say("autotune picked", best)
                after = [c.export_state() for c in ctxs]
                assert before == after, "autotune changed a stream's state"
            r = b.tick(entries)
            for i, inf in zip(idx, r):
                if inf is not None and row[i][1] > 0:
                    infos[i][t] = inf[:row[i][1]]
        S.synchronize()
        for i in range(len(streams)):
            out.append((masks[i].cpu().numpy(), infos[i], ctxs[i].export_state()))
        b.close()
        for c in ctxs:
            c.close()
    return out


def assert_same(streams, a, b):
    for (name, *_), (ma, ia, sa), (mb, ib, sb) in zip(streams, a, b):
        assert np.array_equal(ma, mb), (name, int((ma != mb).sum()))
        assert ia.keys() == ib.keys(), name
        for t in ia:
            assert ia[t] == ib[t], (name, t)
        assert sa == sb, (name, "state differs")


@pytest.fixture(scope="module")
def reference(C, S):
    streams = stream_set(C)
    plan, used = tick_plan(streams)
    say("batch reference: streams", [s[0] for s in streams], "frames used", used)
    return streams, plan, run_alone(C, S, streams, plan)


@pytest.fixture(scope="module")
def batched_default(C, S, reference):
    streams, plan, _ = reference
    say("batched, default schedule")
    return run_batched(C, S, streams, plan)


def test_batch_equals_alone_default_schedule(C, S, reference, batched_default):
    streams, plan, alone = reference
    assert_same(streams, alone, batched_default)


def assert_matches_oracle(streams, plan, got, used):
    """Every stream's batched masks, the per-frame statistics of the ticks
    that asked for them, and its final state against the oracle run over the
    same frames."""
    for i, ((name, p, fr, n_train, _), (mg, infos, blob)) in enumerate(zip(streams, got)):
        n = used[i]
        say("oracle check", name, "frames", n)
        mo, io, so = run_orc(orc_params_like(p), fr[:n_train + n], n_train)
        compare_masks(mg[:n], mo)
        assert np.array_equal(mg[:n], mo), (name, int((mg[:n] != mo).sum()))
        for t, inf in infos.items():
            off, k = plan[t][i]
            assert len(inf) == k, (name, t)
            for a, b in zip(inf, io[off:off + k]):
                assert dict(a) == dict(b), (name, t, a, b)
        assert compare_state(canon.parse(blob), so) == 0, name


def test_batched_streams_match_oracle(C, reference, batched_default):
    """Every stream of the batch -- RGB K=5 and K=3, a ragged 33x17 and a
    sub-tile 7x3 stream, single-channel u8 with K=2 and the f32 latent map --
    against the oracle directly."""
    streams, plan, _ = reference
    used = [sum(row[i][1] for row in plan) for i in range(len(streams))]
    assert_matches_oracle(streams, plan, batched_default, used)


def test_alone_run_matches_oracle(C, reference):
    """Ties the reference itself to the oracle for one stream."""
    streams, plan, alone = reference
    name, p, fr, n_train, _ = streams[0]
    used = sum(row[0][1] for row in plan)
    mo, _, so = run_orc(orc_params_like(p), fr[:n_train + used], n_train)
    mg = alone[0][0][:used]
    compare_masks(mg, mo)
    assert np.array_equal(mg, mo)
    sg = canon.parse(alone[0][2])
    assert compare_state(sg, so) == 0


SCHEDULES = [
    dict(blocks_per_cu=-1, dynamic=0, group=1, use_graph=1, compact=1),
    dict(blocks_per_cu=-1, dynamic=0, group=4, use_graph=0, compact=0),
    dict(blocks_per_cu=0, dynamic=0, group=1, use_graph=0, compact=1),
    dict(blocks_per_cu=0, dynamic=1, group=1, use_graph=1, compact=0),
    dict(blocks_per_cu=0, dynamic=1, group=16, use_graph=1, compact=1),
    dict(blocks_per_cu=1, dynamic=0, group=3, use_graph=1, compact=0),
    dict(blocks_per_cu=1, dynamic=1, group=2, use_graph=0, compact=1),
    dict(blocks_per_cu=-1, dynamic=0, group=4, use_graph=1, compact=0),
]


@pytest.mark.parametrize("sch", SCHEDULES, ids=lambda s: "bpc{blocks_per_cu}-d{dynamic}-g{group}-gr{use_graph}-c{compact}".format(**s))
def test_batch_equals_alone_every_schedule(C, S, reference, sch):
    streams, plan, alone = reference
    classes = {(p.channels, p.K, p.dtype) for _, p, *_ in streams}
    say("batched, schedule", sch)
    got = run_batched(C, S, streams, plan, schedules={k: sch for k in classes})
    assert_same(streams, alone, got)


def test_autotune_keeps_results(C, S, reference):
    streams, plan, alone = reference
    say("batched with autotune at tick 5")
    assert_same(streams, alone, run_batched(C, S, streams, plan, autotune_at=5))


def test_tick_without_work_and_zero_frames(C, S):
    import torch
    with torch.cuda.stream(S):
        b = C.CogBatch(S, max_items=4)
        assert b.tick([]) == []
        p = gpu_params(C, 16, 8, c=3, K=3)
        fr = torch.from_numpy(_synth(16, 8, 30, 20, 9)).cuda()
        s = C.CogStream(p, stream=S)
        s.train_prior(fr[:20])
        before = s.export_state()
        b.tick([(s.h, fr[20:21], None, 0, False)])
        assert s.export_state() == before
        b.close()
        s.close()


def test_batch_errors(C, S):
    import torch
    with torch.cuda.stream(S):
        fr = torch.from_numpy(_synth(16, 8, 30, 20, 8)).cuda()
        S.synchronize()  # the frames are read on another stream below
        p = gpu_params(C, 16, 8, c=3, K=3)
        b = C.CogBatch(S, max_items=4)
        a = C.CogStream(p, stream=S)
        # untrained
        with pytest.raises(C.CogError) as e:
            b.tick([(a.h, fr[20:21], None, 1, False)])
        assert e.value.status == C.COG_E_STATE
        a.train_prior(fr[:20])
        # duplicate context
        with pytest.raises(C.CogError) as e:
            b.tick([(a.h, fr[20:21], None, 1, False), (a.h, fr[21:22], None, 1, False)])
        assert e.value.status == C.COG_E_INVALID
        # more items than the batch holds
        with pytest.raises(C.CogError) as e:
            b.tick([(a.h, fr[20:21], None, 1, False)] * 5)
        assert e.value.status == C.COG_E_INVALID
        # context on another stream
        other = torch.cuda.Stream()
        o = C.CogStream(p, stream=other)
        o.train_prior(fr[:20])
        other.synchronize()
        with pytest.raises(C.CogError) as e:
            b.tick([(o.h, fr[20:21], None, 1, False)])
        assert e.value.status == C.COG_E_INVALID
        # baseline path and other tile sizes
        g = C.CogStream(gpu_params(C, 16, 8, c=3, K=3, path=1), stream=S)
        g.train_prior(fr[:20])
        with pytest.raises(C.CogError) as e:
            b.tick([(g.h, fr[20:21], None, 1, False)])
        assert e.value.status == C.COG_E_UNSUPPORTED
        t = C.CogStream(gpu_params(C, 16, 8, c=3, K=3, tile_px=256), stream=S)
        t.train_prior(fr[:20])
        with pytest.raises(C.CogError) as e:
            b.tick([(t.h, fr[20:21], None, 1, False)])
        assert e.value.status == C.COG_E_UNSUPPORTED
        # statistics for more frames than the stream's statistics chunk (64 here)
        big = torch.zeros((70, 16 * 8 * 3), dtype=torch.uint8, device="cuda")
        with pytest.raises(C.CogError) as e:
            b.tick([(a.h, big, None, 70, True)])
        assert e.value.status == C.COG_E_INVALID
        # a failed tick leaves the stream as it was
        before = a.export_state()
        with pytest.raises(C.CogError):
            b.tick([(a.h, fr[20:21], None, 1, False), (g.h, fr[20:21], None, 1, False)])
        assert a.export_state() == before
        # schedules are validated
        with pytest.raises(C.CogError):
            b.set_schedule(3, 3, 0, group=0)
        with pytest.raises(C.CogError):
            b.set_schedule(3, 9, 0)
        with pytest.raises(C.CogError):
            b.set_schedule(3, 3, 0, compact=2)
        b.set_schedule(3, 3, 0, blocks_per_cu=2, dynamic=1, group=8, use_graph=0, compact=0)
        assert b.get_schedule(3, 3, 0) == dict(blocks_per_cu=2, dynamic=1, group=8, use_graph=0,
                                               compact=0)
        S.synchronize()
        for c in (a, o, g, t):
            c.close()
        b.close()


def test_more_than_eight_classes_rejected(C, S):
    import torch
    with torch.cuda.stream(S):
        fr = torch.from_numpy(_synth(8, 8, 22, 20, 7)).cuda()
        b = C.CogBatch(S, max_items=16)
        ctxs = []
        for K in range(1, 10):
            c, k = (3, K) if K <= 8 else (1, 1)
            f = fr if c == 3 else fr[..., :1].contiguous()
            s = C.CogStream(gpu_params(C, 8, 8, c=c, K=k), stream=S)
            s.train_prior(f[:20])
            ctxs.append((s, f))
        ents = [(s.h, f[20:21], None, 1, False) for s, f in ctxs]
        with pytest.raises(C.CogError) as e:
            b.tick(ents)
        assert e.value.status == C.COG_E_INVALID
        b.tick(ents[:8])
        S.synchronize()
        for s, _ in ctxs:
            s.close()
        b.close()


def test_batch_equals_alone_full_size_streams(C, S):
    """Full-size streams (1280x720 and 640x480 at K=5, 320x240 at K=3, one
    joining late) through the same tick plan: launch shapes like the
    64-stream workload's, with multi-frame ticks staging the prior in LDS and
    graphs captured once a launch set repeats; every stream equals its alone
    run bit for bit."""
    streams = [
        ("u8c3k5-1280x720", gpu_params(C, 1280, 720, c=3, K=5), _synth(1280, 720, 50, 20, 11), 20, 0),
        ("u8c3k5-640x480", gpu_params(C, 640, 480, c=3, K=5), _synth(640, 480, 60, 20, 12), 20, 2),
        ("u8c3k3-320x240", gpu_params(C, 320, 240, c=3, K=3), _synth(320, 240, 70, 20, 13), 20, 0),
    ]
    plan, used = tick_plan(streams)
    say("full-size batch: frames used", used)
    alone = run_alone(C, S, streams, plan)
    batched = run_batched(C, S, streams, plan)
    assert_same(streams, alone, batched)
    assert_matches_oracle(streams, plan, batched, used)
