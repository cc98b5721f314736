"""Pins of the oracle's shared parameter set per group (§2 "Clustering Similar
Background - Spatio-Temporal Grouping": the last item of its list and eq. 3):
the pixels of a group take one variance for their running Gaussian average,
the mean of the members' variances, and stop adapting it.

The pins do not restate the formula.  They check what the mathematics fixes:
the mean of identical values on the 2^-16 grid is that value, the mean lies
within the grid's rounding of the float64 mean of the members, it is never
below var_min even where the grid rounds the members below it, an empty map
changes nothing, pixels outside the groups evolve exactly as without
grouping (pixels are independent), a shared variance never moves while the
means still adapt, and ungrouping lets the variance adapt again."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import canon


def _trained(spec_name="surveil-160x120-k3", n_train=None, frames=80):
    spec = synth.preset(spec_name)
    fr = synth.make_stream(spec, 0, frames)
    nt = spec.n_train if n_train is None else n_train
    o = O.Oracle(O.make_params(spec.width, spec.height, 3, spec.K))
    o.train(fr[:nt])
    return o, fr, nt, spec


def _var(o):
    return canon.parse(o.export())["rga"][:, -1].copy()


def test_identical_members_share_their_own_value():
    """Constant input: every pixel ends training with the same variance, which is
    above 128 (so a multiple of 2^-16): the shared value is exactly it."""
    N = 30
    fr = synth.constant_stream(N, 3, 4, 3, [90, 100, 110])
    o = O.Oracle(O.make_params(4, 3, 3, 3))
    o.train(fr)
    v0 = _var(o)
    assert (v0 == v0[0]).all() and v0[0] >= 128.0
    gv = o.group_share(np.zeros(12, dtype=np.uint8))
    assert gv[0] == v0[0] and gv[1] == 0.0 and gv[2] == 0.0
    assert (_var(o) == v0[0]).all()
    st = canon.parse(o.export())
    assert st["version"] == 3 and (st["shared"] == 1).all()


def test_shared_value_is_held_at_var_min():
    """var_min off the 2^-16 grid (12 + 2^-20): constant input holds every
    variance at var_min, whose grid value is 12, below var_min; the shared
    value is var_min itself, never less."""
    vm = 12.0 + 2.0 ** -20
    assert float(np.float32(vm)) == vm and np.rint(vm * 65536.0) / 65536.0 == 12.0
    fr = synth.constant_stream(30, 3, 4, 3, [90, 100, 110])
    o = O.Oracle(O.make_params(4, 3, 3, 3, var_min=vm, var_init=vm))
    o.train(fr)
    assert (_var(o) == np.float32(vm)).all()
    gv = o.group_share(np.zeros(12, dtype=np.uint8))
    assert gv[0] == np.float32(vm)
    assert (_var(o) == np.float32(vm)).all()


def test_shared_value_is_the_members_mean():
    """On a surveillance stream with the grouping's own map: each shared value is
    within the grid rounding (2^-17) plus one binary32 rounding of the float64
    mean of its members' variances, at least var_min; members hold it,
    everyone else keeps their variance."""
    o, fr, nt, spec = _trained()
    v0 = _var(o)
    m, info = o.group()
    gv = o.group_share(m)
    v1 = _var(o)
    var_min = o.params.var_min
    for g in range(3):
        sel = m == g
        assert sel.sum() == info["groups"][g]["grouped"]
        if not sel.any():
            assert gv[g] == 0.0
            continue
        mean64 = float(np.mean(v0[sel].astype(np.float64)))
        tol = 2.0 ** -17 + float(np.spacing(np.float32(mean64)))
        assert abs(float(gv[g]) - max(mean64, var_min)) <= tol, (g, gv[g], mean64)
        assert gv[g] >= var_min
        assert (v1[sel] == gv[g]).all()
    assert (v1[m == 255] == v0[m == 255]).all()
    st = canon.parse(o.export())
    assert (st["shared"] == (m != 255)).all()


def test_wrong_group_sum_is_caught():
    """The bound above is tight enough to see one member moved to another group."""
    o, fr, nt, spec = _trained()
    v0 = _var(o)
    m, _ = o.group()
    g = int(np.bincount(m[m != 255], minlength=3).argmax())
    members = np.flatnonzero(m == g)
    far = members[np.argmax(np.abs(v0[members] - np.median(v0[members])))]
    mean_all = float(np.mean(v0[members].astype(np.float64)))
    mean_less = float(np.mean(v0[members[members != far]].astype(np.float64)))
    assert abs(mean_all - mean_less) > 2.0 ** -17 + float(np.spacing(np.float32(mean_all)))


def test_empty_map_changes_nothing():
    o1, fr, nt, spec = _trained()
    o2, _, _, _ = _trained()
    o2.group_share(np.full(o2.npix, 255, dtype=np.uint8))
    assert o1.export() == o2.export()
    for t in range(nt, nt + 10):
        m1, i1 = o1.step(fr[t])
        m2, i2 = o2.step(fr[t])
        assert (m1 == m2).all() and i1 == i2
    assert o1.export() == o2.export()


def test_outside_pixels_evolve_as_without_grouping():
    """Pixels are independent: after sharing, the pixels outside every group
    follow exactly the run without grouping (masks and state rows), while the
    members keep their shared variance on every frame and their means adapt."""
    o1, fr, nt, spec = _trained()
    o2, _, _, _ = _trained()
    m, _ = o2.group()
    gv = o2.group_share(m)
    out, ins = m == 255, m != 255
    assert out.any() and ins.any()
    mu_before = canon.parse(o2.export())["rga"][ins, :-1].copy()
    for t in range(nt, min(len(fr), nt + 20)):
        m1, _ = o1.step(fr[t])
        m2, _ = o2.step(fr[t])
        assert (m1[out] == m2[out]).all()
        rga2 = canon.parse(o2.export())["rga"]
        assert (rga2[ins, -1] == gv[m[ins]]).all()
    s1, s2 = canon.parse(o1.export()), canon.parse(o2.export())
    for key in ("gmm", "rga", "label", "prev"):
        assert (s1[key][out] == s2[key][out]).all(), key
    assert (s2["rga"][ins, :-1] != mu_before).any()


def test_singleton_on_grid_keeps_decisions_until_the_variance_would_move():
    """A pixel alone in its group with a variance on the 2^-16 grid shares its
    own value: on the next frame its label, level counts and mean equal the
    ungrouped run's; only the variance, which the ungrouped run adapts on an S1
    acceptance, stays."""
    o1, fr, nt, spec = _trained(n_train=4)
    o2, _, _, _ = _trained(n_train=4)
    v0 = _var(o1)
    cand = np.flatnonzero(v0 >= 128.0)
    assert cand.size
    m = np.full(o2.npix, 255, dtype=np.uint8)
    m[cand] = np.arange(cand.size) % 3
    # singletons: one pixel per group
    m[cand[3:]] = 255
    gv = o2.group_share(m)
    for j, px in enumerate(cand[:3]):
        assert gv[j] == v0[px]
    m1, _ = o1.step(fr[nt])
    m2, _ = o2.step(fr[nt])
    assert (m1 == m2).all()
    r1, r2 = canon.parse(o1.export())["rga"], canon.parse(o2.export())["rga"]
    assert (r1[:, :-1] == r2[:, :-1]).all()
    assert (r2[cand[:3], -1] == v0[cand[:3]]).all()
    outside = np.ones(o2.npix, dtype=bool)
    outside[cand[:3]] = False
    assert (r1[outside, -1] == r2[outside, -1]).all()


def test_ungrouping_lets_the_variance_adapt_again():
    o, fr, nt, spec = _trained()
    m, _ = o.group()
    gv = o.group_share(m)
    o.group_share(None)
    st = canon.parse(o.export())
    assert (st["shared"] == 0).all()
    v_after = st["rga"][:, -1].copy()
    ins = m != 255
    assert (v_after[ins] == gv[m[ins]]).all()
    for t in range(nt, nt + 5):
        o.step(fr[t])
    assert (canon.parse(o.export())["rga"][ins, -1] != v_after[ins]).any()


def test_invalid_group_id_is_rejected():
    o, fr, nt, spec = _trained()
    v0 = _var(o)
    m = np.full(o.npix, 255, dtype=np.uint8)
    m[0] = 3
    with pytest.raises(RuntimeError):
        o.group_share(m)
    assert (_var(o) == v0).all()
