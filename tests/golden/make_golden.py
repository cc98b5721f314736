"""Writes oracle_digests.json: the oracle's outputs on small seeded streams,
as SHA-256 digests of the masks and of each canonical state section, plus
the per-frame level counts.  The paper prints no worked example with
numbers, so these fixtures come from the oracle (this script calls nothing
else but the seeded input generators); they freeze its behaviour, so that an
unintended change to it is caught, and give the GPU tests a second, stored
reference.  Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json")
SECTIONS = ("gmm", "rga", "table", "cnt", "label", "prev", "sat", "gkey")

# (name, width, height, channels, K, dtype, frames, n_train, parameters shared by
# the oracle's and the library's parameter blocks)
CASES = [
    ("cascade-u8c3k3-48x32", 48, 32, 3, 3, 0, 60, 20, {}),
    ("cascade-u8c1k2-37x23", 37, 23, 1, 2, 0, 50, 16, {}),
    ("cascade-u8c3k5-70x9", 70, 9, 3, 5, 0, 48, 12, {}),
    ("sampling-u8c3k4-64x8", 64, 8, 3, 4, 0, 70, 20,
     {"stage_mask": 15, "samp_window": 4, "samp_period": 3}),
    ("plain-gmm-u8c3k3-40x24", 40, 24, 3, 3, 0, 50, 20,
     {"stage_mask": 0, "kappa_alpha": 0.0}),
    ("cascade-f32c1k3-latent-480x1", 480, 1, 1, 3, 1, 45, 15, {"in_lo": -5.0, "in_hi": 5.0}),
]


def frames_for(name, w, h, c, dtype, frames, seed_off):
    if dtype == 1:
        lat = synth.latent_stream(frames, channels=8, h=6, w=10, seed=synth.video.BASE_SEED + 2000)
        return np.ascontiguousarray(lat.reshape(frames, w * h, 1))
    spec = synth.preset("surveil-160x120-k3").with_(width=w, height=h, frames=frames, n_train=1,
                                                    seed=synth.video.BASE_SEED + 2000 + seed_off)
    fr = synth.make_stream(spec)
    return np.ascontiguousarray(fr[..., :c])


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def run_case(i, case):
    from tests import canon
    name, w, h, c, K, dtype, frames, n_train, kw = case
    fr = frames_for(name, w, h, c, dtype, frames, i)
    o = O.Oracle(O.make_params(w, h, c, K, dtype=dtype, **kw))
    o.train(fr[:n_train])
    masks, infos = [], []
    for t in range(n_train, frames):
        m, inf = o.step(fr[t])
        masks.append(m)
        infos.append([inf[k] for k in ("n0", "n1", "n2", "n3", "n3_bg", "n_fg", "illum_flag",
                                       "n_skip")])
    st = canon.parse(o.export())
    o.close()
    return {"name": name, "width": w, "height": h, "channels": c, "K": K, "dtype": dtype,
            "frames": frames, "n_train": n_train, "params": kw, "seed_index": i,
            "masks_sha256": digest(np.stack(masks)),
            "state_sha256": {k: digest(st[k]) for k in SECTIONS},
            "infos": infos}


def generate():
    return [run_case(i, c) for i, c in enumerate(CASES)]


if __name__ == "__main__":
    res = generate()
    with open(OUT, "w") as f:
        json.dump({"note": "oracle digests; written by tests/golden/make_golden.py", "cases": res},
                  f, indent=1)
    print("wrote", OUT, len(res), "cases")
