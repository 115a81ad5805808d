"""Reader for the small cited fixtures under tests/golden/."""
import glob
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(path):
    expect = {}
    n = None
    pairs = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "expect":
                expect[parts[1]] = int(parts[2])
            elif parts[0] == "n":
                n = int(parts[1])
            else:
                pairs.append((int(parts[0]), int(parts[1])))
    p = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
    return n, p[:, 0].copy(), p[:, 1].copy(), expect


def all_fixtures():
    return sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))
