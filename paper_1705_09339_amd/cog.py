"""ctypes binding of libcog.so (include/cog.h), argument marshalling only.

Every step of the method runs in the HIP library; this module only turns
Python objects into pointers and sizes.  Frames and masks may be numpy arrays
(host memory) or torch tensors (host or HIP device memory); torch is used only
for device memory and streams.  There is no fallback: if the library is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcog.so")

COG_OK, COG_E_INVALID, COG_E_OOM, COG_E_STATE, COG_E_DEVICE, COG_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
COG_U8, COG_F32 = 0, 1
COG_STAGE_FD, COG_STAGE_RGA, COG_STAGE_KDE, COG_STAGE_ALL, COG_STAGE_SAMPLE = 1, 2, 4, 7, 8
COG_PATH_CASCADE, COG_PATH_GMM = 0, 1

STATUS_NAMES = {0: "COG_OK", -1: "COG_E_INVALID", -2: "COG_E_OOM", -3: "COG_E_STATE",
                -4: "COG_E_DEVICE", -5: "COG_E_UNSUPPORTED"}


class cog_params(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_uint32),
        ("width", ct.c_int32), ("height", ct.c_int32), ("channels", ct.c_int32),
        ("dtype", ct.c_int32), ("in_lo", ct.c_float), ("in_hi", ct.c_float),
        ("K", ct.c_int32),
        ("alpha", ct.c_float), ("T", ct.c_float), ("lam", ct.c_float),
        ("var_init", ct.c_float), ("var_min", ct.c_float),
        ("stage_mask", ct.c_uint32),
        ("tau_fd", ct.c_float), ("lambda_rga", ct.c_float), ("alpha_rga", ct.c_float),
        ("kde_bins", ct.c_int32), ("kde_h", ct.c_float), ("res_e1", ct.c_float), ("res_e2", ct.c_float),
        ("lambda_m", ct.c_float), ("conf_thr", ct.c_float), ("p_null", ct.c_float),
        ("kappa_alpha", ct.c_float), ("illum_frac", ct.c_float),
        ("path", ct.c_int32), ("tile_px", ct.c_int32),
        ("samp_window", ct.c_int32), ("samp_period", ct.c_int32), ("samp_lambda", ct.c_float),
    ]


class cog_step_info(ct.Structure):
    _fields_ = [
        ("frame", ct.c_int64), ("n_stage", ct.c_int64 * 4), ("n3_bg", ct.c_int64),
        ("n_fg", ct.c_int64), ("illum_flag", ct.c_int32), ("n_skip", ct.c_int32),
    ]

    def as_dict(self) -> dict:
        return dict(frame=self.frame, n0=self.n_stage[0], n1=self.n_stage[1], n2=self.n_stage[2],
                    n3=self.n_stage[3], n3_bg=self.n3_bg, n_fg=self.n_fg, illum_flag=self.illum_flag,
                    n_skip=self.n_skip)


class cog_tick_item(ct.Structure):
    _fields_ = [
        ("ctx", ct.c_void_p), ("frames", ct.c_void_p), ("masks", ct.c_void_p),
        ("nframes", ct.c_int32), ("reserved", ct.c_int32), ("infos", ct.c_void_p),
    ]


class cog_schedule(ct.Structure):
    _fields_ = [
        ("blocks_per_cu", ct.c_int32), ("dynamic", ct.c_int32), ("group", ct.c_int32),
        ("use_graph", ct.c_int32), ("compact", ct.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class cog_completion(ct.Structure):
    _fields_ = [
        ("stream_id", ct.c_int32), ("nframes", ct.c_int32), ("tag", ct.c_int64),
        ("t_submit_us", ct.c_double), ("t_done_us", ct.c_double), ("status", ct.c_int32),
        ("reserved", ct.c_int32),
    ]


class cog_server_stats(ct.Structure):
    _fields_ = [(f, ct.c_int64) for f in (
        "ticks", "frames", "pixel_frames", "streams_open", "streams_admitted", "streams_rejected",
        "bytes_budget", "bytes_allocated", "bytes_in_use", "bytes_largest_free", "pending",
        "in_flight")]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class cog_group_stats(ct.Structure):
    _fields_ = [("count", ct.c_int64), ("grouped", ct.c_int64), ("center", ct.c_int64 * 2),
                ("mean", ct.c_double * 2), ("sd", ct.c_double * 2)]


class cog_group_info(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("reserved", ct.c_int32),
                ("group", cog_group_stats * 3)]

    def as_dict(self) -> dict:
        return dict(iterations=self.iterations, groups=[
            dict(count=g.count, center=(g.center[0], g.center[1]), mean=(g.mean[0], g.mean[1]),
                 sd=(g.sd[0], g.sd[1]), grouped=g.grouped) for g in self.group])


class CogError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libcog.so is not built ({path}); run paper_1705_09339_amd/build.py")
    L = ct.CDLL(path)
    P, V = ct.POINTER, ct.c_void_p
    sig = {
        "cog_default_params": ([P(cog_params), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32], ct.c_int),
        "cog_state_bytes": ([P(cog_params), P(ct.c_size_t)], ct.c_int),
        "cog_canonical_bytes": ([P(cog_params), P(ct.c_size_t)], ct.c_int),
        "cog_create": ([P(cog_params), V, V, ct.c_size_t, P(V)], ct.c_int),
        "cog_train_prior": ([V, V, ct.c_int32, ct.c_int32], ct.c_int),
        "cog_step": ([V, V, ct.c_int32, V, ct.c_int32, P(cog_step_info)], ct.c_int),
        "cog_step_frames": ([V, V, ct.c_int32, ct.c_int32, V, ct.c_int32, P(cog_step_info)], ct.c_int),
        "cog_reset": ([V], ct.c_int),
        "cog_destroy": ([V], None),
        "cog_export_state": ([V, V, ct.c_size_t], ct.c_int),
        "cog_import_state": ([V, V, ct.c_size_t], ct.c_int),
        "cog_kde_weights": ([ct.c_float, P(ct.c_uint16)], ct.c_int),
        "cog_last_error": ([V], ct.c_char_p),
        "cog_group_background": ([V, V, ct.c_int32, P(cog_group_info)], ct.c_int),
        "cog_group_background_noalloc": ([V, V, ct.c_int32, P(cog_group_info)], ct.c_int),
        "cog_group_share": ([V, V, ct.c_int32, P(ct.c_float)], ct.c_int),
        "cog_batch_create": ([V, ct.c_int32, P(V)], ct.c_int),
        "cog_batch_tick": ([V, P(cog_tick_item), ct.c_int32], ct.c_int),
        "cog_batch_autotune": ([V, P(cog_tick_item), ct.c_int32, ct.c_int32, P(cog_schedule)], ct.c_int),
        "cog_batch_set_schedule": ([V, ct.c_int32, ct.c_int32, ct.c_int32, P(cog_schedule)], ct.c_int),
        "cog_batch_get_schedule": ([V, ct.c_int32, ct.c_int32, ct.c_int32, P(cog_schedule)], ct.c_int),
        "cog_batch_destroy": ([V], None),
        "cog_server_create": ([V, ct.c_size_t, ct.c_int32, ct.c_int32, P(V)], ct.c_int),
        "cog_server_open": ([V, P(cog_params), V, ct.c_int32, P(ct.c_int32)], ct.c_int),
        "cog_server_submit": ([V, ct.c_int32, V, ct.c_int32, V, ct.c_int64], ct.c_int),
        "cog_server_close": ([V, ct.c_int32], ct.c_int),
        "cog_server_poll": ([V, P(cog_completion), ct.c_int32, P(ct.c_int32), ct.c_int64], ct.c_int),
        "cog_server_drain": ([V, ct.c_int32], ct.c_int),
        "cog_server_export": ([V, ct.c_int32, V, ct.c_size_t], ct.c_int),
        "cog_server_stats_get": ([V, P(cog_server_stats)], ct.c_int),
        "cog_server_destroy": ([V], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()

EXPORTED = ("cog_default_params", "cog_state_bytes", "cog_canonical_bytes", "cog_create",
            "cog_train_prior", "cog_step", "cog_step_frames", "cog_reset", "cog_destroy",
            "cog_export_state", "cog_import_state", "cog_kde_weights", "cog_last_error",
            "cog_group_background", "cog_group_background_noalloc", "cog_group_share",
            "cog_batch_create", "cog_batch_tick", "cog_batch_autotune", "cog_batch_set_schedule",
            "cog_batch_get_schedule", "cog_batch_destroy",
            "cog_server_create", "cog_server_open", "cog_server_submit", "cog_server_close",
            "cog_server_poll", "cog_server_drain", "cog_server_export", "cog_server_stats_get",
            "cog_server_destroy")


def _check(rc: int, h=None):
    if rc != COG_OK:
        msg = lib.cog_last_error(h)
        raise CogError(rc, msg.decode() if msg else "")


def _ptr(a):
    """(address, on_device, keepalive) of a numpy array or torch tensor."""
    if a is None:
        return None, 0, None
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a)
        return a.ctypes.data, 0, a
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), 1 if a.is_cuda else 0, a
    raise TypeError(f"unsupported buffer type {type(a)}")


# ---- functions with the C names ------------------------------------------------

def cog_default_params(width: int, height: int, channels: int = 3, dtype: int = COG_U8,
                       K: int = 3, **overrides) -> cog_params:
    p = cog_params()
    _check(lib.cog_default_params(ct.byref(p), width, height, channels, dtype, K))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def cog_state_bytes(p: cog_params) -> int:
    n = ct.c_size_t(0)
    _check(lib.cog_state_bytes(ct.byref(p), ct.byref(n)))
    return n.value


def cog_canonical_bytes(p: cog_params) -> int:
    n = ct.c_size_t(0)
    _check(lib.cog_canonical_bytes(ct.byref(p), ct.byref(n)))
    return n.value


def cog_create(p: cog_params, stream=None, device_state=None) -> int:
    """stream: a torch.cuda.Stream, a raw hipStream_t int, or None (default).
    device_state: optional torch uint8 tensor on the device."""
    h = ct.c_void_p(0)
    sptr = None
    if stream is not None:
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    dptr, nbytes = None, 0
    if device_state is not None:
        dptr, on_dev, _ = _ptr(device_state)
        if not on_dev:
            raise ValueError("device_state must be device memory")
        nbytes = device_state.numel() * device_state.element_size()
    _check(lib.cog_create(ct.byref(p), sptr, dptr, nbytes, ct.byref(h)))
    return h.value


def cog_train_prior(h: int, frames) -> None:
    ptr, dev, keep = _ptr(frames)
    _check(lib.cog_train_prior(h, ptr, len(frames), dev), h)
    del keep


def cog_step(h: int, frame, mask_out=None, want_info: bool = False) -> Optional[dict]:
    fp, fdev, k1 = _ptr(frame)
    mp, mdev, k2 = _ptr(mask_out)
    info = cog_step_info() if want_info else None
    _check(lib.cog_step(h, fp, fdev, mp, mdev, ct.byref(info) if info is not None else None), h)
    del k1, k2
    return info.as_dict() if info is not None else None


def cog_step_frames(h: int, frames, masks_out=None, want_info: bool = False):
    n = len(frames)
    fp, fdev, k1 = _ptr(frames)
    mp, mdev, k2 = _ptr(masks_out)
    infos = (cog_step_info * n)() if want_info else None
    _check(lib.cog_step_frames(h, fp, n, fdev, mp, mdev, infos), h)
    del k1, k2
    return [i.as_dict() for i in infos] if infos is not None else None


def cog_reset(h: int) -> None:
    _check(lib.cog_reset(h), h)


def cog_destroy(h: int) -> None:
    lib.cog_destroy(h)


def cog_export_state(h: int, p: cog_params) -> bytes:
    n = cog_canonical_bytes(p)
    buf = np.zeros(n, dtype=np.uint8)
    _check(lib.cog_export_state(h, buf.ctypes.data, n), h)
    return buf.tobytes()


def cog_import_state(h: int, blob: bytes) -> None:
    a = np.frombuffer(blob, dtype=np.uint8)
    _check(lib.cog_import_state(h, a.ctypes.data, a.size), h)


def cog_kde_weights(hw: float = 8.0) -> np.ndarray:
    out = np.zeros((16, 256), dtype=np.uint16)
    _check(lib.cog_kde_weights(hw, out.ctypes.data_as(ct.POINTER(ct.c_uint16))))
    return out


def cog_group_background(h: int, map_out=None) -> dict:
    """Spatio-temporal grouping after training; fills map_out (P bytes, numpy
    or torch, 255 = ungrouped) if given and returns the info as a dict."""
    mp, mdev, keep = _ptr(map_out)
    info = cog_group_info()
    _check(lib.cog_group_background(h, mp, mdev, ct.byref(info)), h)
    del keep
    return info.as_dict()


def cog_group_background_noalloc(h: int, map_out=None) -> dict:
    """cog_group_background on the library's static device scratch (no
    device allocation; streams of at most COG_NOALLOC_MAX_PIXELS pixels)."""
    mp, mdev, keep = _ptr(map_out)
    info = cog_group_info()
    _check(lib.cog_group_background_noalloc(h, mp, mdev, ct.byref(info)), h)
    del keep
    return info.as_dict()


COG_NOALLOC_MAX_PIXELS = 1 << 23


def cog_group_share(h: int, group_map=None) -> np.ndarray:
    """One shared running-average variance per group for the pixels of
    group_map (P bytes, numpy or torch; 0..2, 255 = outside every group);
    None ungroups every pixel.  Returns the 3 shared variances."""
    gv = np.zeros(3, dtype=np.float32)
    mp, mdev, keep = _ptr(group_map)
    _check(lib.cog_group_share(h, mp, mdev, gv.ctypes.data_as(ct.POINTER(ct.c_float))), h)
    del keep
    return gv


def cog_last_error(h: Optional[int] = None) -> str:
    m = lib.cog_last_error(h)
    return m.decode() if m else ""


class CogStream:
    """One stream's context: owns the handle, forwards to the C calls."""

    def __init__(self, params: cog_params, stream=None, device_state=None):
        self.params = params
        self.h = cog_create(params, stream, device_state)

    def train_prior(self, frames):
        cog_train_prior(self.h, frames)

    def step(self, frame, mask_out=None, want_info=False):
        return cog_step(self.h, frame, mask_out, want_info)

    def step_frames(self, frames, masks_out=None, want_info=False):
        return cog_step_frames(self.h, frames, masks_out, want_info)

    def reset(self):
        cog_reset(self.h)

    def group(self, map_out=None) -> dict:
        return cog_group_background(self.h, map_out)

    def share(self, group_map=None):
        return cog_group_share(self.h, group_map)

    def export_state(self) -> bytes:
        return cog_export_state(self.h, self.params)

    def import_state(self, blob: bytes):
        cog_import_state(self.h, blob)

    def close(self):
        if self.h:
            cog_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---- batched tick ----------------------------------------------------------------

def _stream_ptr(stream):
    if stream is None:
        return None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def cog_batch_create(stream=None, max_items: int = 256) -> int:
    b = ct.c_void_p(0)
    _check(lib.cog_batch_create(_stream_ptr(stream), max_items, ct.byref(b)))
    return b.value


def _items(entries):
    """entries: (ctx handle, frames, masks or None, nframes or None, want_info)."""
    n = len(entries)
    arr = (cog_tick_item * max(n, 1))()
    keep, infos = [], []
    for i, (h, frames, masks, nframes, want_info) in enumerate(entries):
        fp, fdev, k1 = _ptr(frames)
        mp, mdev, k2 = _ptr(masks)
        if frames is not None and not fdev:
            raise ValueError("batched ticks take device frames")
        if masks is not None and not mdev:
            raise ValueError("batched ticks take device masks")
        nf = len(frames) if nframes is None else int(nframes)
        inf = (cog_step_info * max(nf, 1))() if want_info else None
        arr[i].ctx = h
        arr[i].frames = fp
        arr[i].masks = mp
        arr[i].nframes = nf
        arr[i].reserved = 0
        arr[i].infos = ct.cast(inf, ct.c_void_p) if inf is not None else None
        keep += [k1, k2, inf]
        infos.append((inf, nf))
    return arr, n, keep, infos


def cog_batch_tick(b: int, entries):
    """Advance each entry's stream; returns per entry a list of info dicts (or None)."""
    arr, n, keep, infos = _items(entries)
    _check(lib.cog_batch_tick(b, arr, n))
    del keep
    return [[inf[i].as_dict() for i in range(nf)] if inf is not None else None
            for inf, nf in infos]


def cog_batch_autotune(b: int, entries, reps: int = 3) -> dict:
    arr, n, keep, _ = _items(entries)
    best = cog_schedule()
    _check(lib.cog_batch_autotune(b, arr, n, reps, ct.byref(best)))
    del keep
    return best.as_dict()


def cog_batch_set_schedule(b: int, channels: int, K: int, dtype: int, **kw) -> None:
    s = cog_schedule(blocks_per_cu=kw.get("blocks_per_cu", -1), dynamic=kw.get("dynamic", 0),
                     group=kw.get("group", 4), use_graph=kw.get("use_graph", 1),
                     compact=kw.get("compact", 1))
    _check(lib.cog_batch_set_schedule(b, channels, K, dtype, ct.byref(s)))


def cog_batch_get_schedule(b: int, channels: int, K: int, dtype: int) -> dict:
    s = cog_schedule()
    _check(lib.cog_batch_get_schedule(b, channels, K, dtype, ct.byref(s)))
    return s.as_dict()


def cog_batch_destroy(b: int) -> None:
    lib.cog_batch_destroy(b)


class CogBatch:
    """A batch executor on one HIP stream; forwards to the C calls."""

    def __init__(self, stream=None, max_items: int = 256):
        self.b = cog_batch_create(stream, max_items)

    def tick(self, entries):
        return cog_batch_tick(self.b, entries)

    def autotune(self, entries, reps: int = 3) -> dict:
        return cog_batch_autotune(self.b, entries, reps)

    def set_schedule(self, channels, K, dtype, **kw):
        cog_batch_set_schedule(self.b, channels, K, dtype, **kw)

    def get_schedule(self, channels, K, dtype) -> dict:
        return cog_batch_get_schedule(self.b, channels, K, dtype)

    def close(self):
        if self.b:
            cog_batch_destroy(self.b)
            self.b = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class TickTable:
    """A reusable cog_tick_item array for tight tick loops: the fields are
    exposed as numpy columns (ctx, frames, masks, nframes), so a caller
    updates pointers and counts without building Python objects per tick."""

    _dtype = np.dtype([("ctx", np.uint64), ("frames", np.uint64), ("masks", np.uint64),
                       ("nframes", np.int32), ("reserved", np.int32), ("infos", np.uint64)])

    def __init__(self, n: int):
        assert self._dtype.itemsize == ct.sizeof(cog_tick_item)
        self.n = n
        self._arr = (cog_tick_item * max(n, 1))()
        self.view = np.frombuffer(self._arr, dtype=self._dtype, count=n)

    def tick(self, b: int, n: Optional[int] = None) -> None:
        _check(lib.cog_batch_tick(b, self._arr, self.n if n is None else n))

    def autotune(self, b: int, reps: int = 3) -> dict:
        best = cog_schedule()
        _check(lib.cog_batch_autotune(b, self._arr, self.n, reps, ct.byref(best)))
        return best.as_dict()


# ---- serving loop ------------------------------------------------------------------

class CogServer:
    """A serving loop (cog_server_*): streams are opened within an HBM budget,
    frames submitted as they arrive, completions polled."""

    def __init__(self, hbm_budget: int, max_streams: int = 256, depth: int = 2, stream=None):
        s = ct.c_void_p(0)
        _check(lib.cog_server_create(_stream_ptr(stream), int(hbm_budget), max_streams, depth,
                                     ct.byref(s)))
        self.s = s.value
        self.params = {}

    def open(self, params: cog_params, train_frames) -> int:
        fp, fdev, keep = _ptr(train_frames)
        if not fdev:
            raise ValueError("training frames must be device memory")
        sid = ct.c_int32(-1)
        _check(lib.cog_server_open(self.s, ct.byref(params), fp, len(train_frames), ct.byref(sid)))
        del keep
        self.params[sid.value] = params
        return sid.value

    def submit(self, sid: int, frames, masks=None, tag: int = 0, nframes: Optional[int] = None):
        fp, fdev, _ = _ptr(frames)
        mp, mdev, _ = _ptr(masks)
        if not fdev or (masks is not None and not mdev):
            raise ValueError("frames and masks must be device memory")
        n = 1 if nframes is None else nframes
        _check(lib.cog_server_submit(self.s, sid, fp, n, mp, tag))

    def submit_ptr(self, sid: int, frames_ptr: int, masks_ptr: int, tag: int, nframes: int = 1):
        _check(lib.cog_server_submit(self.s, sid, frames_ptr, nframes, masks_ptr, tag))

    def close_stream(self, sid: int):
        _check(lib.cog_server_close(self.s, sid))

    def poll(self, max_n: int = 1024, wait_us: int = 0):
        buf = (cog_completion * max_n)()
        n = ct.c_int32(0)
        _check(lib.cog_server_poll(self.s, buf, max_n, ct.byref(n), wait_us))
        return [dict(stream_id=c.stream_id, nframes=c.nframes, tag=c.tag, t_submit_us=c.t_submit_us,
                     t_done_us=c.t_done_us, status=c.status) for c in buf[:n.value]]

    def drain(self, sid: int = -1):
        _check(lib.cog_server_drain(self.s, sid))

    def export_state(self, sid: int) -> bytes:
        nb = cog_canonical_bytes(self.params[sid])
        buf = np.zeros(nb, dtype=np.uint8)
        _check(lib.cog_server_export(self.s, sid, buf.ctypes.data, nb))
        return buf.tobytes()

    def stats(self) -> dict:
        st = cog_server_stats()
        _check(lib.cog_server_stats_get(self.s, ct.byref(st)))
        return st.as_dict()

    def close(self):
        if self.s:
            lib.cog_server_destroy(self.s)
            self.s = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
