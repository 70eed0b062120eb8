"""Write the exact-rational reference images under tests/golden/.

Calls only ``oracle.exact`` (the brute-force rational renderer); inputs are
stored alongside the outputs so the fixture does not depend on any generator.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


def rot(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
            [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
            [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]]


def case(name, seed, dims, M, W, H, extent, tau, boxes=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    n1, n2, n3 = dims
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    tf = rng.uniform(0, 1, (M, 4)).astype(np.float32)
    tf[:, 3] *= 0.3
    R = rot(rng.normal(0, 1, 4))
    vmin, vmax = float(vol.min()), float(vol.max())
    img = exact.render(vol.tolist(), tf.tolist(), R, W, H, extent, vmin, vmax, 0.5, tau, boxes=boxes)
    out = {
        "name": name,
        "what": "exact-rational image of the ray-casting definition (paper Sec. 2, 2.4, 2.5)",
        "dims": list(dims), "W": W, "H": H, "extent": extent, "tau": tau, "step": 0.5,
        "vmin": vmin, "vmax": vmax, "R": R,
        "vol": [float(v) for v in vol.ravel()], "tf": [float(v) for v in tf.ravel()],
        "boxes": boxes,
        "image": [[list(map(float, px)) for px in row] for row in img],
    }
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    case("tiny_whole_ert", 101, (5, 4, 6), 8, 6, 5, 6.0, 0.7)
    case("tiny_whole_noert", 102, (4, 6, 5), 6, 5, 5, 6.5, 2.0)
    boxes = [((0, 0, 0), (3, 4, 6), (0, 1, 1)), ((3, 0, 0), (5, 4, 6), (1, 1, 1))]
    case("tiny_bricked_local_ert", 103, (6, 5, 7), 8, 6, 6, 8.0, 0.6, boxes=boxes)
