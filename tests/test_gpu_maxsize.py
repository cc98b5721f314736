"""The cascade at the library's largest frame, 16384 x 16384 = 2^28 pixels
(45 GB of state at K=3): one launch of 9 frames in the configuration the
bench times (prior staged in LDS, a full 8-frame block whose mask window is
2^31 bytes, then a 1-frame block), then a single-frame step with statistics.
Checked against the oracle on sampled pixels (their time series run through
the oracle as a small frame) and by whole-frame properties.  The frames are
drawn on the device (synth.device); the oracle receives the same bytes."""
import numpy as np
import pytest

from tests.gpu_util import gpu_params, orc_params_like, run_orc, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09339_amd import cog
    return cog


def test_maximum_frame_size(C):
    import torch
    from synth.device import DeviceScene
    W = H = 16384
    P = W * H
    N, T = 2, 12
    p = gpu_params(C, W, H, c=3, K=3)
    say("max size: drawing", T, "frames of", W, "x", H)
    fr = DeviceScene(W, H, 170509339 + 77, fg_occ=0.05, n_rects=16).frames(0, T)
    masks = torch.zeros((T - N, P), dtype=torch.uint8, device="cuda")
    s = C.CogStream(p, stream=torch.cuda.current_stream())
    try:
        s.train_prior(fr[:N])
        say("max size: 9-frame launch")
        s.step_frames(fr[N:T - 1], masks[:T - N - 1])
        say("max size: last frame with statistics")
        info = s.step(fr[T - 1], masks[T - N - 1], want_info=True)
        torch.cuda.synchronize()
    finally:
        s.close()
    assert info["n0"] + info["n1"] + info["n2"] + info["n3"] == P
    assert info["n_fg"] == int((masks[T - N - 1] == 255).sum().item())
    # sampled pixels: the first and last 64-pixel runs, runs across a row end,
    # and random pixels
    rng = np.random.default_rng(5)
    pix = set(range(64)) | set(range(P - 64, P)) | set(range(W - 32, W + 32))
    pix |= set(range(P // 2 - 32, P // 2 + 32))
    pix |= set(rng.choice(P, size=3000, replace=False).tolist())
    pix = np.array(sorted(pix))
    idx = torch.from_numpy(pix).cuda()
    sub = fr.view(T, P, 3).index_select(1, idx).cpu().numpy()[:, None]
    mg = masks.index_select(1, idx).cpu().numpy()
    po = orc_params_like(p)
    po.width, po.height = len(pix), 1
    mo, _, _ = run_orc(po, sub, N)
    assert set(np.unique(mg)) <= {0, 255}
    assert np.array_equal(mg, mo)
