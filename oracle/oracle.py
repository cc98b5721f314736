"""ctypes front end of the C oracle (cog_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the HIP library or its
binding.  ``build()`` compiles the C source with gcc; the library is loaded
from this directory.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cog_oracle.c")
LIB = os.path.join(HERE, "libcog_oracle.so")

FD, RGA, KDE, SAMPLE = 1, 2, 4, 8
U8, F32 = 0, 1

# Defaults of the readings taken where the paper gives no number (K, alpha,
# T and lambda are the Stauffer-Grimson values of the workloads).
DEFAULTS = dict(
    dtype=U8, in_lo=0.0, in_hi=256.0,
    alpha=0.01, T=0.7, lam=2.5, var_init=None, var_min=None,
    stage_mask=FD | RGA | KDE,
    tau_fd=0.0, lambda_rga=2.5, alpha_rga=None,
    kde_h=8.0, res_e1=16.0, res_e2=48.0,
    lambda_m=None, conf_thr=0.5, p_null=0.1, kappa_alpha=0.5,
    illum_frac=0.7,
    samp_window=32, samp_period=4, samp_lambda=None,
)


class OrcParams(ct.Structure):
    _fields_ = [
        ("width", ct.c_int32), ("height", ct.c_int32), ("channels", ct.c_int32), ("K", ct.c_int32),
        ("dtype", ct.c_int32), ("in_lo", ct.c_float), ("in_hi", ct.c_float),
        ("alpha", ct.c_float), ("T", ct.c_float), ("lam", ct.c_float),
        ("var_init", ct.c_float), ("var_min", ct.c_float),
        ("stage_mask", ct.c_uint32),
        ("tau_fd", ct.c_float), ("lambda_rga", ct.c_float), ("alpha_rga", ct.c_float),
        ("kde_h", ct.c_float), ("res_e1", ct.c_float), ("res_e2", ct.c_float),
        ("lambda_m", ct.c_float), ("conf_thr", ct.c_float), ("p_null", ct.c_float),
        ("kappa_alpha", ct.c_float),
        ("illum_frac", ct.c_float),
        ("samp_window", ct.c_int32), ("samp_period", ct.c_int32), ("samp_lambda", ct.c_float),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (scalar, -O2, no contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ct.CDLL(LIB)
        P = ct.POINTER
        L.orc_kde_weights.argtypes = [ct.c_double, P(ct.c_uint16)]
        L.orc_create.argtypes = [P(OrcParams)]
        L.orc_create.restype = ct.c_void_p
        L.orc_destroy.argtypes = [ct.c_void_p]
        L.orc_train.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int]
        L.orc_step.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, P(ct.c_int64)]
        L.orc_gmm_step.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.orc_pixel_gmmstep.argtypes = [P(OrcParams), P(ct.c_float), P(ct.c_float), ct.c_float,
                                        P(ct.c_int), P(ct.c_int)]
        L.orc_pixel_bgset.argtypes = [P(OrcParams), P(ct.c_float)]
        L.orc_group_keys.argtypes = [ct.c_void_p, P(ct.c_uint32)]
        L.orc_group.argtypes = [ct.c_void_p, P(ct.c_uint8), P(ct.c_double)]
        L.orc_group_run.argtypes = [P(ct.c_uint32), ct.c_int64, P(ct.c_uint8), P(ct.c_double)]
        L.orc_group_share.argtypes = [ct.c_void_p, P(ct.c_uint8), P(ct.c_float)]
        L.orc_group_set.argtypes = [ct.c_void_p, P(ct.c_uint8), P(ct.c_float)]
        L.orc_canonical_bytes.argtypes = [P(OrcParams)]
        L.orc_canonical_bytes.restype = ct.c_size_t
        L.orc_export.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t]
        _lib = L
    return _lib


def make_params(width: int, height: int, channels: int = 3, K: int = 3, **kw) -> OrcParams:
    d = dict(DEFAULTS)
    d.update(kw)
    if d["var_init"] is None:
        d["var_init"] = channels * 225.0
    if d["var_min"] is None:
        d["var_min"] = channels * 4.0
    if d["alpha_rga"] is None:
        d["alpha_rga"] = d["alpha"]
    if d["lambda_m"] is None:
        d["lambda_m"] = 2.0 * d["lambda_rga"]
    if d["samp_lambda"] is None:
        d["samp_lambda"] = d["lambda_rga"]
    p = OrcParams()
    p.width, p.height, p.channels, p.K = width, height, channels, K
    for k, v in d.items():
        setattr(p, k, v)
    return p


def kde_weights(h: float = 8.0) -> np.ndarray:
    out = np.zeros((16, 256), dtype=np.uint16)
    rc = lib().orc_kde_weights(h, out.ctypes.data_as(ct.POINTER(ct.c_uint16)))
    if rc != 0:
        raise ValueError("bad bandwidth")
    return out


def pixel_gmmstep(params: OrcParams, comp: np.ndarray, x, alpha_e: float):
    """One mixture step on a single K x (C+2) record; returns (comp', label, m_post)."""
    comp = np.ascontiguousarray(comp, dtype=np.float32).copy()
    xv = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    lab = ct.c_int(-1)
    mp = ct.c_int(-9)
    lib().orc_pixel_gmmstep(ct.byref(params), comp.ctypes.data_as(ct.POINTER(ct.c_float)),
                            xv.ctypes.data_as(ct.POINTER(ct.c_float)), float(alpha_e),
                            ct.byref(lab), ct.byref(mp))
    return comp, lab.value, mp.value


def _group_info(info) -> dict:
    groups = []
    for g in range(3):
        o = info[1 + 8 * g:9 + 8 * g]
        groups.append(dict(count=int(o[0]), center=(int(o[1]), int(o[2])), mean=(o[3], o[5]),
                           sd=(o[4], o[6]), grouped=int(o[7])))
    return dict(iterations=int(info[0]), groups=groups)


def group_run(keys) -> tuple:
    """The grouping's clustering and band on given keys [P, 2] (u32)."""
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    m = np.zeros(len(k), dtype=np.uint8)
    info = np.zeros(1 + 8 * 3, dtype=np.float64)
    if lib().orc_group_run(k.ctypes.data_as(ct.POINTER(ct.c_uint32)), len(k),
                           m.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                           info.ctypes.data_as(ct.POINTER(ct.c_double))) != 0:
        raise ValueError("orc_group_run failed")
    return m, _group_info(info)


def pixel_bgset(params: OrcParams, comp: np.ndarray) -> int:
    comp = np.ascontiguousarray(comp, dtype=np.float32)
    return lib().orc_pixel_bgset(ct.byref(params), comp.ctypes.data_as(ct.POINTER(ct.c_float)))


class Oracle:
    """One stream's oracle state; frames are numpy arrays [.., P or H,W, C]."""

    def __init__(self, params: OrcParams):
        self.params = params
        self._h = lib().orc_create(ct.byref(params))
        if not self._h:
            raise ValueError("invalid oracle parameters")
        self.npix = params.width * params.height
        self.C = params.channels
        self._dt = np.uint8 if params.dtype == U8 else np.float32

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _frames(self, a, n=None):
        a = np.ascontiguousarray(a, dtype=self._dt)
        per = self.npix * self.C
        if n is None:
            if a.size != per:
                raise ValueError("frame size mismatch")
        elif a.size != per * n:
            raise ValueError("frames size mismatch")
        return a

    def train(self, frames) -> None:
        n = len(frames)
        a = self._frames(frames, n)
        if lib().orc_train(self._h, a.ctypes.data, n) != 0:
            raise RuntimeError("orc_train failed")

    def step(self, frame):
        a = self._frames(frame)
        mask = np.empty(self.npix, dtype=np.uint8)
        info = (ct.c_int64 * 9)()
        if lib().orc_step(self._h, a.ctypes.data, mask.ctypes.data, info) != 0:
            raise RuntimeError("orc_step failed")
        keys = ("frame", "n0", "n1", "n2", "n3", "n3_bg", "n_fg", "illum_flag", "n_skip")
        return mask, dict(zip(keys, list(info)))

    def gmm_step(self, frame):
        a = self._frames(frame)
        mask = np.empty(self.npix, dtype=np.uint8)
        if lib().orc_gmm_step(self._h, a.ctypes.data, mask.ctypes.data) != 0:
            raise RuntimeError("orc_gmm_step failed")
        return mask

    def group_keys(self) -> np.ndarray:
        """Per-pixel grouping keys [P, 2] (u32) from the training warm-up."""
        out = np.zeros((self.npix, 2), dtype=np.uint32)
        if lib().orc_group_keys(self._h, out.ctypes.data_as(ct.POINTER(ct.c_uint32))) != 0:
            raise RuntimeError("orc_group_keys failed (train first)")
        return out

    def group(self):
        """(map [P] u8 with 255 = ungrouped, info dict) of the spatio-temporal grouping."""
        m = np.zeros(self.npix, dtype=np.uint8)
        info = np.zeros(1 + 8 * 3, dtype=np.float64)
        if lib().orc_group(self._h, m.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                           info.ctypes.data_as(ct.POINTER(ct.c_double))) != 0:
            raise RuntimeError("orc_group failed (train first)")
        return m, _group_info(info)

    def group_share(self, group_map) -> np.ndarray:
        """Shared S1 variance per group for the pixels of group_map ([P] u8, 0..2 or 255;
        None ungroups every pixel); returns the 3 shared variances."""
        gv = np.zeros(3, dtype=np.float32)
        if group_map is None:
            mp = ct.POINTER(ct.c_uint8)()
        else:
            m = np.ascontiguousarray(group_map, dtype=np.uint8).reshape(-1)
            if m.size != self.npix:
                raise ValueError("group map must hold one byte per pixel")
            mp = m.ctypes.data_as(ct.POINTER(ct.c_uint8))
        if lib().orc_group_share(self._h, mp, gv.ctypes.data_as(ct.POINTER(ct.c_float))) != 0:
            raise RuntimeError("orc_group_share failed (train first; groups 0..2 or 255)")
        return gv

    def group_set(self, group_map, gvar) -> None:
        """The members of group g take the shared variance gvar[g] (no fitting)."""
        m = np.ascontiguousarray(group_map, dtype=np.uint8).reshape(-1)
        g = np.ascontiguousarray(gvar, dtype=np.float32).reshape(3)
        if m.size != self.npix:
            raise ValueError("group map must hold one byte per pixel")
        if lib().orc_group_set(self._h, m.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                               g.ctypes.data_as(ct.POINTER(ct.c_float))) != 0:
            raise RuntimeError("orc_group_set failed")

    def export(self) -> bytes:
        nb = lib().orc_canonical_bytes(ct.byref(self.params))
        buf = np.zeros(nb, dtype=np.uint8)
        if lib().orc_export(self._h, buf.ctypes.data, nb) != 0:
            raise RuntimeError("orc_export failed")
        return buf.tobytes()
