"""Writes ct512_k16_seed0.json: every exact moment (eq. 2) of order <= 16 (969 values) of
the 512^3 uint16 CT-like volume synth.ct_phantom(seed=0), computed by the oracle.

    python tests/golden/make_ct512_k16.py

Only oracle/ and the seeded input generator are used; nothing here touches the HIP path.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

K = 16
SHAPE = (512, 512, 512)
SEED = 0


def main():
    t0 = time.time()
    V = synth.ct_phantom(SHAPE, seed=SEED)
    allm = oracle.moment_list(K)
    vals = oracle.moments_exact(V, K)
    print(f"{len(vals)} moments in {time.time() - t0:.0f}s", flush=True)
    out = [[p, q, r, str(v)] for (p, q, r), v in zip(allm, vals)]
    doc = {"what": "exact raw moments M_pqr = sum V x^p y^q z^r (eq. 2), every p+q+r <= 16",
           "volume": {"generator": "synth.ct_phantom", "shape_zyx": list(SHAPE), "seed": SEED},
           "max_order": K, "moments": out}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "ct512_k16_seed0.json"), "w") as fh:
        json.dump(doc, fh, separators=(",", ":"))


if __name__ == "__main__":
    main()
