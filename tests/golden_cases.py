"""Reader for the hand-derived fixtures in ``tests/golden/tiny_cases.txt``."""
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_cases.txt")


def load():
    cases, cur = [], None
    for line in open(PATH):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        f = line.split()
        if f[0] == "case":
            cur = {"name": f[1], "n_modules": int(f[2]), "cut": int(f[3]), "d": [], "k": []}
            cases.append(cur)
        elif f[0] == "d":
            cur["d"].append([int(x) for x in f[1:]])
        elif f[0] == "k":
            cur["k"].append([int(x) for x in f[1:]])
    out = []
    for c in cases:
        d = np.array(c["d"], dtype=np.int64).reshape(-1, 5)
        ev = {"module": d[:, 0].astype(np.uint16), "row": d[:, 1].astype(np.uint16),
              "col": d[:, 2].astype(np.uint16), "adc": d[:, 3].astype(np.uint16),
              "n_modules": c["n_modules"]}
        k = np.array(c["k"], dtype=np.int64).reshape(-1, 3)
        out.append((c["name"], ev, c["cut"], d[:, 4], k))
    return out
