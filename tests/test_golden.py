"""The oracle against its stored digests (tests/golden/oracle_digests.json,
written by tests/golden/make_golden.py from the oracle alone): any change to
the oracle's arithmetic shows up here and has to be justified and the
fixture rewritten.  Also checks the fixture's own consistency: per frame the
level counts sum to the pixel count."""
import json
import os

import pytest

from tests.golden import make_golden as G

FIX = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")


def _stored():
    with open(FIX) as f:
        return json.load(f)["cases"]


def test_fixture_is_consistent():
    for c in _stored():
        P = c["width"] * c["height"]
        for inf in c["infos"]:
            n0, n1, n2, n3, n3bg, nfg, _illum, nskip = inf
            assert n0 + n1 + n2 + n3 + nskip == P, c["name"]
            assert 0 <= n3bg <= n3 and 0 <= nfg <= P


@pytest.mark.parametrize("i", range(len(G.CASES)))
def test_oracle_matches_stored_digests(i):
    stored = _stored()[i]
    live = G.run_case(i, G.CASES[i])
    assert live == stored, stored["name"]
