"""Helpers for the GPU parity tests: run the HIP library and the oracle on
the same seeded frames and compare their outputs."""
import sys

import numpy as np

from oracle import oracle as O
from tests import canon

# parity bar: model state within 1e-5 relative, masks differing on at most
# 1e-4 of the pixels (threshold ties)
STATE_RTOL = 1e-5
MASK_FRAC = 1e-4

ORC_KEYS = {"lam": "lam"}


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def gpu_params(C, w, h, c=3, K=3, dtype=0, **kw):
    p = C.cog_default_params(w, h, c, dtype, K)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def orc_params_like(p):
    """Oracle parameters equal to a library parameter block."""
    return O.make_params(
        p.width, p.height, p.channels, p.K, dtype=p.dtype, in_lo=p.in_lo, in_hi=p.in_hi,
        alpha=p.alpha, T=p.T, lam=p.lam, var_init=p.var_init, var_min=p.var_min,
        stage_mask=p.stage_mask, tau_fd=p.tau_fd, lambda_rga=p.lambda_rga,
        alpha_rga=p.alpha_rga, kde_h=p.kde_h, res_e1=p.res_e1, res_e2=p.res_e2,
        lambda_m=p.lambda_m, conf_thr=p.conf_thr, p_null=p.p_null,
        kappa_alpha=p.kappa_alpha, illum_frac=p.illum_frac, samp_window=p.samp_window,
        samp_period=p.samp_period, samp_lambda=p.samp_lambda)


def run_gpu(C, p, frames, n_train, mode="step", infos=True, stream=None):
    """frames: numpy [T, ..., C].  Returns (masks [T-N, P] u8, infos, canonical state)."""
    import torch
    T = len(frames)
    P = p.width * p.height
    dev = torch.from_numpy(np.ascontiguousarray(frames)).cuda()
    masks = torch.zeros((T - n_train, P), dtype=torch.uint8, device="cuda")
    s = C.CogStream(p, stream=stream if stream is not None else torch.cuda.current_stream())
    try:
        s.train_prior(dev[:n_train])
        inf = []
        if mode == "step":
            for t in range(n_train, T):
                r = s.step(dev[t], masks[t - n_train], want_info=infos)
                inf.append(r)
        elif mode == "frames":
            inf = s.step_frames(dev[n_train:], masks, want_info=infos)
        elif isinstance(mode, int):
            for t0 in range(n_train, T, mode):
                t1 = min(T, t0 + mode)
                r = s.step_frames(dev[t0:t1], masks[t0 - n_train:t1 - n_train], want_info=infos)
                if r:
                    inf.extend(r)
        torch.cuda.synchronize()
        st = canon.parse(s.export_state())
    finally:
        s.close()
    return masks.cpu().numpy(), inf, st


def run_orc(p_orc, frames, n_train, mode="cog"):
    orc = O.Oracle(p_orc)
    orc.train(frames[:n_train])
    masks, infos = [], []
    for t in range(n_train, len(frames)):
        if mode == "cog":
            m, i = orc.step(frames[t])
        else:
            m, i = orc.gmm_step(frames[t]), None
        masks.append(m)
        infos.append(i)
    st = canon.parse(orc.export())
    orc.close()
    return np.array(masks), infos, st


def compare_state(sg, so, keys=("gmm", "rga", "table", "cnt", "label", "prev"), pix=None):
    """Asserts the parity bar; returns the number of bitwise-different floats."""
    nbits = 0
    for k in keys:
        a, b = sg[k], so[k]
        if pix is not None:
            a = a[pix]
        assert a.shape == b.shape, (k, a.shape, b.shape)
        if a.dtype.kind == "f":
            diff = np.abs(a.astype(np.float64) - b.astype(np.float64))
            tol = STATE_RTOL * np.maximum(np.abs(a), np.abs(b)).astype(np.float64) + 1e-30
            bad = diff > tol
            assert not bad.any(), (k, int(bad.sum()), np.argwhere(bad)[:5])
            nbits += int((a.view(np.uint32) != b.view(np.uint32)).sum())
        else:
            assert np.array_equal(a, b), (k, int((a != b).sum()))
    return nbits


def compare_masks(mg, mo):
    diff = (mg != mo).sum()
    assert diff <= MASK_FRAC * mg.size, (int(diff), mg.size)
    return int(diff)


def compare_infos(ig, io):
    for a, b in zip(ig, io):
        a = dict(a)
        b = dict(b)
        assert a == b, (a, b)
