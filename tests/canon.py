"""Parser of the canonical state layout shared by the oracle and the library.

Layout: a 64-byte header {u32 magic 'COG1', u32 version, i32 width, height,
channels, K, dtype, n_train, i64 frame}, then sections each padded to 64 bytes:
gmm f32[P][K][C+2] (w, mu[C], var in rank order), rga f32[P][C+1],
table u8[P][C][16], cnt u16[P][3], label u8[P], prev f32[P][C], and from
version 2 on sat u16[P] (the sampling saturation counters) and gkey u32[P][2]
(the grouping keys of the training warm-up), and from version 3 on shared u8[P]
(1 where the pixel takes its group's shared running-average variance).
"""
import numpy as np

MAGIC = 0x31474F43


def _pad(n):
    return (n + 63) // 64 * 64


def parse(blob: bytes) -> dict:
    b = np.frombuffer(blob, dtype=np.uint8)
    hdr32 = b[:8].view(np.uint32)
    assert hdr32[0] == MAGIC, hex(int(hdr32[0]))
    version = int(hdr32[1])
    assert version in (1, 2, 3), version
    W, H, C, K, dtype, n_train = (int(v) for v in b[8:32].view(np.int32))
    frame = int(b[32:40].view(np.int64)[0])
    P = W * H
    out = dict(width=W, height=H, channels=C, K=K, dtype=dtype, n_train=n_train, frame=frame,
               version=version)
    off = 64
    sections = [
        ("gmm", np.float32, (P, K, C + 2)),
        ("rga", np.float32, (P, C + 1)),
        ("table", np.uint8, (P, C, 16)),
        ("cnt", np.uint16, (P, 3)),
        ("label", np.uint8, (P,)),
        ("prev", np.float32, (P, C)),
    ]
    if version >= 2:
        sections.append(("sat", np.uint16, (P,)))
        sections.append(("gkey", np.uint32, (P, 2)))
    if version >= 3:
        sections.append(("shared", np.uint8, (P,)))
    for name, dt, shape in sections:
        nbytes = int(np.prod(shape)) * np.dtype(dt).itemsize
        out[name] = b[off:off + nbytes].copy().view(dt).reshape(shape)
        off += _pad(nbytes)
    assert off <= len(b)
    return out
