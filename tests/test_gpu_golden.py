"""The HIP path against the stored oracle digests (tests/golden): masks,
every canonical state section and the per-frame level counts of six small
streams (u8 C=3/C=1, K=2..5, the sampling variant, the plain-mixture mode
of the cascade ABI, f32 latent input), bit for bit, without running the
oracle."""
import json
import os

import numpy as np
import pytest

from tests.golden import make_golden as G
from tests.gpu_util import gpu_params, run_gpu, say

pytestmark = pytest.mark.gpu
FIX = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09339_amd import cog
    return cog


@pytest.mark.parametrize("i", range(len(G.CASES)))
def test_hip_matches_oracle_digests(C, i):
    with open(FIX) as f:
        stored = json.load(f)["cases"][i]
    name, w, h, c, K, dtype, frames, n_train, kw = G.CASES[i]
    assert stored["name"] == name
    fr = G.frames_for(name, w, h, c, dtype, frames, i)
    p = gpu_params(C, w, h, c=c, K=K, dtype=dtype, **kw)
    say("golden", name)
    mg, ig, sg = run_gpu(C, p, fr, n_train, mode="frames")
    assert G.digest(mg) == stored["masks_sha256"], name
    for k in G.SECTIONS:
        assert G.digest(sg[k]) == stored["state_sha256"][k], (name, k)
    got = [[r[k] for k in ("n0", "n1", "n2", "n3", "n3_bg", "n_fg", "illum_flag", "n_skip")]
           for r in ig]
    assert got == stored["infos"], name
