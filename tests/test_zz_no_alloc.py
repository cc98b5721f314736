"""cog_group_background_noalloc: the grouping on the library's static device
scratch gives the same map and statistics as cog_group_background, call after
call on one GPU (the second call on a smaller stream, so stale scratch
contents of the first are present), with device and host map buffers; a
stream beyond the scratch's size is refused."""
import numpy as np
import pytest

import synth
from tests.gpu_util import gpu_params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09339_amd import cog
    return cog


def trained(C, w, h, seed_off, K=5, frames=40):
    import torch
    spec = synth.preset("surveil-640x480-k5").with_(width=w, height=h, frames=frames, n_train=frames,
                                                    seed=synth.video.BASE_SEED + 900 + seed_off)
    fr = torch.from_numpy(synth.make_stream(spec, threads=8)).cuda()
    s = C.CogStream(gpu_params(C, w, h, c=3, K=K), stream=torch.cuda.current_stream())
    s.train_prior(fr)
    torch.cuda.synchronize()
    return s


def both(C, s, P, host):
    import torch
    if host:
        ma = np.zeros(P, np.uint8)
        mb = np.full(P, 7, np.uint8)
    else:
        ma = torch.zeros(P, dtype=torch.uint8, device="cuda")
        mb = torch.full((P,), 7, dtype=torch.uint8, device="cuda")
    ia = C.cog_group_background(s.h, ma)
    ib = C.cog_group_background_noalloc(s.h, mb)
    torch.cuda.synchronize()
    if not host:
        ma, mb = ma.cpu().numpy(), mb.cpu().numpy()
    return ma, ia, mb, ib


@pytest.mark.parametrize("host", [False, True], ids=["device-map", "host-map"])
def test_noalloc_grouping_equals_allocating_call(C, host):
    big = trained(C, 640, 480, 1)
    small = trained(C, 97, 61, 2, K=3)
    for name, s, P in (("640x480", big, 640 * 480), ("97x61 after 640x480", small, 97 * 61)):
        say("no-alloc grouping", name, "host map" if host else "device map")
        ma, ia, mb, ib = both(C, s, P, host)
        assert np.array_equal(ma, mb), (name, int((ma != mb).sum()))
        assert ia == ib, (name, ia, ib)
        assert ia["iterations"] >= 1
        assert sum(g["count"] for g in ia["groups"]) == P
        assert set(np.unique(mb)) <= {0, 1, 2, 255}
    # and the large stream again, after the small one
    ma, ia, mb, ib = both(C, big, 640 * 480, host)
    assert np.array_equal(ma, mb) and ia == ib
    # no map, info only
    assert C.cog_group_background_noalloc(small.h) == C.cog_group_background(small.h)
    big.close()
    small.close()


def test_noalloc_grouping_rejects_streams_beyond_the_scratch(C):
    import torch
    w, h = 4097, 2048  # one column more than the 2^23-pixel limit allows
    assert w * h > C.COG_NOALLOC_MAX_PIXELS
    s = C.CogStream(gpu_params(C, w, h, c=3, K=1), stream=torch.cuda.current_stream())
    with pytest.raises(C.CogError) as e:
        C.cog_group_background_noalloc(s.h)
    assert e.value.status == C.COG_E_STATE  # untrained first
    s.train_prior(torch.zeros((2, h, w, 3), dtype=torch.uint8, device="cuda"))
    with pytest.raises(C.CogError) as e:
        C.cog_group_background_noalloc(s.h)
    assert e.value.status == C.COG_E_INVALID
    s.close()
