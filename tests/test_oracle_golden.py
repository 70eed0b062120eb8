"""FP64 oracle vs stored exact-rational images (tests/golden/*.json).

The fixtures were written by ``tests/golden/make_golden.py``, which calls only
the exact-rational brute force; they freeze the definition's value on three
tiny cases (whole volume with and without ERT, two sub-volumes with local ERT).
"""
import glob
import json
import os

import numpy as np
import pytest

GOLD = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.json")))


@pytest.mark.parametrize("path", GOLD, ids=[os.path.basename(p) for p in GOLD])
def test_oracle_matches_golden(orc, path):
    g = json.load(open(path))
    n1, n2, n3 = g["dims"]
    vol = np.array(g["vol"], np.float32).reshape(n3, n2, n1)
    tf = np.array(g["tf"], np.float32).reshape(-1, 4)
    bricks = None
    if g["boxes"]:
        bricks = [(tuple(b[0]), tuple(b[1]), tuple(b[2])) for b in g["boxes"]]
    res = orc.render(vol, tf, [np.array(g["R"])], g["W"], g["H"], g["vmin"], g["vmax"],
                     step=g["step"], tau=g["tau"], extent=g["extent"], bricks=bricks)
    want = np.array(g["image"])
    np.testing.assert_allclose(res["image"][0], want, rtol=0, atol=1e-12)
    assert (want[..., 3] > 0).sum() > 4


def test_golden_present():
    assert len(GOLD) >= 3
