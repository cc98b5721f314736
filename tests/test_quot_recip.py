"""The cascade kernels replace three divisions per survivor by a quotient from
a correctly rounded reciprocal and two fused residual corrections (the scene
prior's normalisation, the frame-difference similarity and the renormalised
mixture weights).  Results stay bit-identical to binary32 division only if
that algorithm is exact on every operand the kernels feed it; this checks
the algorithm on the CPU, exhaustively where the dividends are the 255^C + 1
prior integers and widely elsewhere, and that the check itself rejects the
uncorrected estimate."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _build(tmp_path, src):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "chk")
    subprocess.run([cc, "-O2", "-ffp-contract=off", "-o", exe, src, "-lm"], check=True)
    return exe


def _run(exe, scale=1):
    out = subprocess.run([exe, str(scale)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.strip().splitlines())}


def test_quotient_matches_division(tmp_path):
    res = _run(_build(tmp_path, os.path.join(HERE, "quot_recip_check.c")))
    assert res == {"prior": 0, "difference": 0, "general": 0, "weights": 0}


def test_check_rejects_uncorrected_quotient(tmp_path):
    """Without corrections (q = a y) the same groups must show differences,
    or the check would prove nothing."""
    src = open(os.path.join(HERE, "quot_recip_check.c")).read()
    a = "  return fmaf(fmaf(-d, q1, a), y, q1);"
    assert a in src
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(a, "  (void)q1;\n  return q0;"))
    res = _run(_build(tmp_path, str(mut)))
    assert all(v > 0 for v in res.values()), res
