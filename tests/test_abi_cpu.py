"""The C-ABI library loads, exports what include/cog.h declares, and its
host-only logic behaves; no GPU is touched here."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def C():
    from paper_1705_09339_amd import cog
    return cog


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cog.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cog_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(C):
    names = declared_functions()
    assert len(names) >= 13
    lib = ct.CDLL(C.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(C.EXPORTED)


def test_header_has_no_torch_types():
    src = open(os.path.join(ROOT, "include", "cog.h")).read()
    assert "torch" not in src.lower().replace("torch-", "")
    assert 'extern "C"' in src


def test_struct_layouts_match_header(C, tmp_path):
    """Compile a C probe against include/cog.h and compare every field offset."""
    import subprocess
    fields_p = [f for f, _ in C.cog_params._fields_]
    cfields = {f: ("lambda" if f == "lam" else f) for f in fields_p}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cog.h"', "int main(void){",
             'printf("%zu\\n", sizeof(cog_params));',
             'printf("%zu\\n", sizeof(cog_step_info));']
    for f in fields_p:
        lines.append(f'printf("%zu\\n", offsetof(cog_params, {cfields[f]}));')
    for f, _ in C.cog_step_info._fields_:
        lines.append(f'printf("%zu\\n", offsetof(cog_step_info, {f}));')
    for st in (C.cog_tick_item, C.cog_schedule, C.cog_completion, C.cog_server_stats,
               C.cog_group_stats, C.cog_group_info):
        lines.append(f'printf("%zu\\n", sizeof({st.__name__}));')
        for f, _ in st._fields_:
            lines.append(f'printf("%zu\\n", offsetof({st.__name__}, {f}));')
    lines.append("return 0;}")
    (tmp_path / "probe.c").write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(tmp_path / "probe.c")], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == ct.sizeof(C.cog_params) and vals[1] == ct.sizeof(C.cog_step_info)
    offs = vals[2:]
    exp = [getattr(C.cog_params, f).offset for f in fields_p] + \
          [getattr(C.cog_step_info, f).offset for f, _ in C.cog_step_info._fields_]
    for st in (C.cog_tick_item, C.cog_schedule, C.cog_completion, C.cog_server_stats,
               C.cog_group_stats, C.cog_group_info):
        exp += [ct.sizeof(st)] + [getattr(st, f).offset for f, _ in st._fields_]
    assert offs == exp


def test_default_params(C):
    p = C.cog_default_params(640, 480, 3, C.COG_U8, 5)
    assert p.struct_size == ct.sizeof(C.cog_params)
    assert (p.K, p.alpha, p.T, p.lam, p.var_init, p.var_min) == (5, np.float32(0.01), np.float32(0.7),
                                                                 2.5, 675.0, 12.0)
    assert p.stage_mask == 7 and p.kde_bins == 16 and p.lambda_m == 5.0
    assert (p.res_e1, p.res_e2, p.conf_thr, p.p_null, p.kappa_alpha) == (16, 48, 0.5, np.float32(0.1), 0.5)
    assert p.illum_frac == np.float32(0.7) and p.path == C.COG_PATH_CASCADE
    assert (p.samp_window, p.samp_period, p.samp_lambda) == (32, 4, 2.5)


@pytest.mark.parametrize("bad", [
    dict(K=0), dict(K=9), dict(channels=2), dict(width=0), dict(var_min=0.0),
    dict(var_init=1.0), dict(kde_bins=8), dict(stage_mask=16), dict(tile_px=384),
    dict(stage_mask=15, samp_window=0), dict(stage_mask=15, samp_period=0),
    dict(stage_mask=15, samp_lambda=-1.0), dict(stage_mask=8, path=1),
    dict(path=2), dict(alpha=0.0), dict(res_e1=60.0), dict(dtype=1, in_lo=1.0, in_hi=1.0),
    dict(struct_size=4),
])
def test_invalid_params_rejected_without_device(C, bad):
    p = C.cog_default_params(64, 48, 3, C.COG_U8, 3)
    for k, v in bad.items():
        setattr(p, k, v)
    with pytest.raises(C.CogError) as ei:
        C.cog_state_bytes(p)
    assert ei.value.status == C.COG_E_INVALID
    with pytest.raises(C.CogError) as ei:
        C.cog_create(p)
    assert ei.value.status == C.COG_E_INVALID
    assert C.cog_last_error(None)


def test_state_bytes_cover_the_model(C):
    for (w, h, K) in ((160, 120, 3), (640, 480, 5), (1920, 1080, 5)):
        p = C.cog_default_params(w, h, 3, C.COG_U8, K)
        n = C.cog_state_bytes(p)
        P = w * h
        R = ((K * 5) + 3) // 4 * 4
        assert n >= P * (R * 4 + 16 + 64 + 3) + P // 8
        assert n < P * (R * 4 + 16 + 64 + 3) * 1.2 + 2**22
        g = C.cog_default_params(w, h, 3, C.COG_U8, K, path=C.COG_PATH_GMM)
        assert C.cog_state_bytes(g) < n


def test_canonical_bytes_agree_with_oracle(C):
    for (w, h, c, K) in ((160, 120, 3, 3), (37, 23, 1, 5), (1, 1, 3, 8)):
        p = C.cog_default_params(w, h, c, C.COG_U8, K)
        op = O.make_params(w, h, c, K)
        assert C.cog_canonical_bytes(p) == O.lib().orc_canonical_bytes(ct.byref(op))


@pytest.mark.parametrize("h", [8.0, 3.0, 17.5])
def test_kde_weights_equal_oracle_table(C, h):
    assert np.array_equal(C.cog_kde_weights(h), O.kde_weights(h))


def test_create_without_device_reports_device_error(C):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = C.cog_default_params(16, 16, 3, C.COG_U8, 3)
    with pytest.raises(C.CogError) as ei:
        C.cog_create(p)
    assert ei.value.status == C.COG_E_DEVICE


def test_null_context_calls_are_invalid(C):
    assert C.lib.cog_reset(None) == C.COG_E_INVALID
    assert C.lib.cog_step(None, None, 0, None, 0, None) == C.COG_E_INVALID
    assert C.lib.cog_train_prior(None, None, 10, 0) == C.COG_E_INVALID
    assert C.lib.cog_group_background(None, None, 0, None) == C.COG_E_INVALID
    assert C.lib.cog_group_background_noalloc(None, None, 0, None) == C.COG_E_INVALID
    C.lib.cog_destroy(None)


def test_batch_create_without_device_reports_device_error(C):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(C.CogError) as ei:
        C.cog_batch_create(None, 8)
    assert ei.value.status == C.COG_E_DEVICE


def test_null_batch_calls_are_invalid(C):
    s = C.cog_schedule(0, 0, 1, 1)
    assert C.lib.cog_batch_tick(None, None, 0) == C.COG_E_INVALID
    assert C.lib.cog_batch_set_schedule(None, 3, 5, 0, ct.byref(s)) == C.COG_E_INVALID
    assert C.lib.cog_batch_get_schedule(None, 3, 5, 0, ct.byref(s)) == C.COG_E_INVALID
    assert C.lib.cog_batch_autotune(None, None, 0, 1, None) == C.COG_E_INVALID
    out = ct.c_void_p(0)
    assert C.lib.cog_batch_create(None, 0, ct.byref(out)) == C.COG_E_INVALID
    assert C.lib.cog_batch_create(None, 5000, ct.byref(out)) == C.COG_E_INVALID
    C.lib.cog_batch_destroy(None)


def test_server_create_without_device_reports_device_error(C):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(C.CogError) as ei:
        C.CogServer(1 << 30)
    assert ei.value.status == C.COG_E_DEVICE


def test_null_server_calls_are_invalid(C):
    n = ct.c_int32(0)
    assert C.lib.cog_server_submit(None, 0, None, 1, None, 0) == C.COG_E_INVALID
    assert C.lib.cog_server_close(None, 0) == C.COG_E_INVALID
    assert C.lib.cog_server_poll(None, None, 0, ct.byref(n), 0) == C.COG_E_INVALID
    assert C.lib.cog_server_drain(None, -1) == C.COG_E_INVALID
    out = ct.c_void_p(0)
    assert C.lib.cog_server_create(None, 1 << 30, 0, 2, ct.byref(out)) == C.COG_E_INVALID
    assert C.lib.cog_server_create(None, 1 << 30, 8, 9, ct.byref(out)) == C.COG_E_INVALID
    assert C.lib.cog_server_create(None, 0, 8, 2, ct.byref(out)) == C.COG_E_INVALID
    C.lib.cog_server_destroy(None)
