"""The seeded input generator: the thread-pool path draws the same frames and
ground truth as the sequential one (both parity sides and the benchmark rely
on it), for every kind of scene object."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("name,stop", [("surveil-160x120-k3", 30), ("surveil-640x480-k5", 12)])
def test_threaded_generation_equals_sequential(name, stop):
    spec = synth.preset(name)
    a, ga = synth.make_stream(spec, 3, stop, with_gt=True)
    b, gb = synth.make_stream(spec, 3, stop, with_gt=True, threads=4)
    assert np.array_equal(a, b) and np.array_equal(ga, gb)


def test_threaded_generation_with_ellipses():
    spec = synth.preset("surveil-1920x1080-k5-occ30").with_(width=320, height=180, frames=20)
    a, ga = synth.make_stream(spec, with_gt=True)
    b, gb = synth.make_stream(spec, with_gt=True, threads=4)
    assert np.array_equal(a, b) and np.array_equal(ga, gb)
    assert ga.mean() > 0.1  # the ellipses are drawn
