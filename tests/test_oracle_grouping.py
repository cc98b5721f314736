"""Pins of the oracle's spatio-temporal grouping (§2 "Clustering Similar
Background - Spatio-Temporal Grouping"): closed-form features on constant
input, exact separation of a static and a bimodal region, the converged
k-means fixed point checked by brute force, the degenerate single-cluster
case, and invariance under a permutation of the pixels."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


def _oracle(fr, n_train, w, h, C=3, K=3):
    o = O.Oracle(O.make_params(w, h, C, K))
    o.train(fr[:n_train])
    return o


def _key(var):
    """Grouping key: the binary32 pattern of a non-negative variance >> 16."""
    v = np.float32(max(var, 0.0))
    return int(np.array([v], dtype=np.float32).view(np.uint32)[0]) >> 16


def test_constant_input_keys_closed_form():
    """Constant input: the dominant weight stays 1 (variance 0, key 0), and its
    variance follows var_j = (1 - alpha) var_{j-1} from var_init down to the
    floor; the key of the sequence's temporal variance agrees with a float64
    evaluation to within one key unit (binary32 sums)."""
    N, alpha, var_init, var_min = 40, 0.01, 675.0, 12.0
    fr = synth.constant_stream(N, 3, 2, 3, [90, 100, 110])
    o = _oracle(fr, N, 2, 3)
    keys = o.group_keys()
    assert (keys[:, 1] == 0).all()
    seq, v = [], var_init
    for _ in range(N - 1):
        v = max(var_min, (1 - alpha) * v)
        seq.append(v)
    seq = np.array(seq)
    var64 = float(np.mean(seq ** 2) - np.mean(seq) ** 2)
    assert np.all(np.abs(keys[:, 0].astype(np.int64) - _key(var64)) <= 1), (keys[:, 0], _key(var64))
    m, info = o.group()
    # identical pixels: one cluster, everything grouped (sd 0, closed interval)
    assert info["groups"][0]["count"] == 6 and info["groups"][0]["grouped"] == 6
    assert (m == 0).all() and info["iterations"] == 2


def test_static_and_bimodal_regions_separate():
    """Left half constant, right half alternating between two colours: the
    dominant weight of the right half varies, so its weight key is non-zero,
    and the two halves land in different groups."""
    N, h, w = 60, 6, 16
    fr = np.empty((N, h, w, 3), dtype=np.uint8)
    fr[:, :, : w // 2] = [120, 120, 120]
    fr[0::2, :, w // 2:] = [40, 200, 60]
    fr[1::2, :, w // 2:] = [200, 40, 180]
    o = _oracle(fr, N, w, h)
    keys = o.group_keys().reshape(h, w, 2)
    assert (keys[:, : w // 2, 1] == 0).all() and (keys[:, w // 2:, 1] > 0).all()
    m, info = o.group()
    m = m.reshape(h, w)
    left, right = np.unique(m[:, : w // 2]), np.unique(m[:, w // 2:])
    assert len(left) == 1 and len(right) == 1 and left[0] != right[0] and 255 not in (left[0], right[0])


def _lloyd_fixed_point(keys, info):
    centers = np.array([g["center"] for g in info["groups"]], dtype=np.int64)
    d = ((keys[:, None, :].astype(np.int64) - centers[None]) ** 2).sum(-1)
    asg = d.argmin(1)  # first minimum = lowest index on ties
    return centers, asg


@pytest.mark.parametrize("name,frames", [("surveil-160x120-k3", 60)])
def test_kmeans_fixed_point_and_threshold(name, frames):
    spec = synth.preset(name)
    fr = synth.make_stream(spec, 0, frames)
    o = _oracle(fr, spec.n_train, spec.width, spec.height, K=spec.K)
    keys = o.group_keys()
    m, info = o.group()
    assert info["iterations"] < 32, "did not converge"
    centers, asg = _lloyd_fixed_point(keys, info)
    for g in range(3):
        mem = keys[asg == g].astype(np.int64)
        assert info["groups"][g]["count"] == len(mem)
        if len(mem):
            # converged: each centre is the floor of its members' mean
            assert tuple(mem.sum(0) // len(mem)) == tuple(centers[g])
            np.testing.assert_allclose(info["groups"][g]["mean"], mem.mean(0), rtol=1e-12)
            np.testing.assert_allclose(info["groups"][g]["sd"], mem.std(0), rtol=1e-9, atol=1e-9)
    # eq. 3: grouped iff both keys within one standard deviation of the mean
    mean = np.array([g["mean"] for g in info["groups"]])[asg]
    sd = np.array([g["sd"] for g in info["groups"]])[asg]
    inside = (np.abs(keys - mean) <= sd).all(1)
    assert np.array_equal(m == 255, ~inside)
    assert np.array_equal(m[inside], asg[inside])
    assert sum(g["grouped"] for g in info["groups"]) == int(inside.sum())
    # the bimodal square and the background both form groups
    assert len([g for g in info["groups"] if g["grouped"] > 0]) >= 2


def test_grouping_is_pixel_permutation_invariant():
    spec = synth.preset("surveil-160x120-k3").with_(width=32, height=24, frames=60, n_train=50)
    fr = synth.make_stream(spec)
    perm = np.random.default_rng(5).permutation(32 * 24)
    flat = fr.reshape(60, -1, 3)
    a = _oracle(fr, 50, 32, 24)
    b = _oracle(np.ascontiguousarray(flat[:, perm]).reshape(60, 24, 32, 3), 50, 32, 24)
    ma, ia = a.group()
    mb, ib = b.group()
    assert np.array_equal(ma[perm], mb)
    assert ia == ib


# ---- the clustering on hand-made keys ----------------------------------------------

def test_kmeans_initial_centres_and_ties():
    """Two pixels with keys (0,0) and (1,0): the centres start at the minimum
    (0,0), the floor of the mean (0,0) and the maximum (1,0); pixel 0 is
    equally near centres 0 and 1 and takes 0 (lowest index); pixel 1 takes 2."""
    m, info = O.group_run([[0, 0], [1, 0]])
    assert [g["count"] for g in info["groups"]] == [1, 0, 1]
    assert info["groups"][0]["center"] == (0, 0) and info["groups"][2]["center"] == (1, 0)
    assert list(m) == [0, 2] and info["iterations"] == 2


def test_kmeans_three_obvious_clusters():
    """Three separated clouds placed at the minimum, the mean and the maximum
    of the keys end in three clusters whose centres are the floors of the
    cloud means; eq. 3's closed one-sigma band keeps a and b whole and only
    the centre point of c (hand-checked: c's standard deviation is 0.894)."""
    a = [[0, 0], [2, 0], [0, 2], [2, 2]]                      # mean (1, 1), sd (1, 1)
    b = [[500, 500], [502, 500]]                              # mean (501, 500), sd (1, 0)
    c = [[1000, 1000], [1002, 1000], [1000, 1002], [1002, 1002], [1001, 1001]]
    m, info = O.group_run(a + b + c)
    g = info["groups"]
    assert info["iterations"] == 2
    assert [x["count"] for x in g] == [4, 2, 5]
    assert [x["center"] for x in g] == [(1, 1), (501, 500), (1001, 1001)]
    assert list(m) == [0, 0, 0, 0, 1, 1, 255, 255, 255, 255, 2]
    assert [x["grouped"] for x in g] == [4, 2, 1]
