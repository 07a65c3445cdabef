"""Philox4x32-10 against its published known-answer vectors, and the
noise-bank selection rule."""
import json
import os

import numpy as np

from oracle import philox

KAT = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")))


def test_known_answers():
    for v in KAT["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert list(philox.philox4x32_10(ctr, key)) == [int(x, 16) for x in v["out"]]


def test_bank_lookup_rule():
    rng = np.random.default_rng(0)
    S = 16
    bank = rng.standard_normal((3, S, S))
    coords = np.array([(i, j) for i in range(5) for j in range(5)])
    V = philox.bank_noise(bank, coords, 4, seed=123456789012, instance=2, frame=7)
    for mem in range(4):
        s, oy, ox, o = philox.member_draw(123456789012, 2, 7, mem, 3, S)
        for (i, j), v in zip(coords, V[:, mem]):
            u, w = (j, i) if o & 1 else (i, j)
            u = -u if o & 2 else u
            w = -w if o & 4 else w
            assert v == bank[s, (oy + u) % S, (ox + w) % S]
    # distinct frames and members draw differently; same inputs repeat exactly
    V2 = philox.bank_noise(bank, coords, 4, seed=123456789012, instance=2, frame=7)
    assert np.array_equal(V, V2)
    V3 = philox.bank_noise(bank, coords, 4, seed=123456789012, instance=2, frame=8)
    assert not np.array_equal(V, V3)
