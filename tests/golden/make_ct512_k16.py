"""Writes ct512_k16_seed0.json: sampled exact moments (eq. 2) of the 512^3 uint16 CT-like
volume synth.ct_phantom(seed=0), up to order 16, computed one by one by the oracle.

    python tests/golden/make_ct512_k16.py

Only oracle/ and the seeded input generator are used; nothing here touches the HIP path.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

K = 16
SHAPE = (512, 512, 512)
SEED = 0


def sample(K, seed=1):
    """Every moment of order <= 2, the axis extremes and a seeded sample of the rest."""
    allm = oracle.moment_list(K)
    pick = [m for m in allm if sum(m) <= 2]
    pick += [(16, 0, 0), (0, 16, 0), (0, 0, 16), (8, 0, 8), (0, 8, 8), (8, 8, 0), (5, 6, 5), (1, 14, 1),
             (3, 3, 3), (2, 1, 1), (1, 2, 1), (1, 1, 2), (4, 0, 0), (2, 2, 0)]
    rest = [m for m in allm if sum(m) >= 3 and m not in pick]
    rng = np.random.default_rng(seed)
    pick += [rest[i] for i in sorted(rng.choice(len(rest), size=24, replace=False))]
    return sorted(set(pick), key=lambda m: oracle.moment_index(*m))


def main():
    t0 = time.time()
    V = synth.ct_phantom(SHAPE, seed=SEED)
    out = []
    for (p, q, r) in sample(K):
        out.append([p, q, r, str(oracle.moment_single(V, p, q, r))])
        print(p, q, r, f"{time.time() - t0:.0f}s", flush=True)
    doc = {"what": "exact raw moments M_pqr = sum V x^p y^q z^r (eq. 2), sampled",
           "volume": {"generator": "synth.ct_phantom", "shape_zyx": list(SHAPE), "seed": SEED},
           "max_order": K, "moments": out}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "ct512_k16_seed0.json"), "w") as fh:
        json.dump(doc, fh, indent=0)


if __name__ == "__main__":
    main()
