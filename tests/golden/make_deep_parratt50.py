"""Writes deep_parratt50.json: 50-digit reference reflectivities of
microsliced profiles (300 to 2047 slabs), from the high-precision Parratt
recursion in oracle/mp_reference.py.  The profiles are regenerated from the
stored seeds by paper_2509_06924_amd.inputs.microsliced_stack.

    python tests/golden/make_deep_parratt50.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mp_reference  # noqa: E402
from paper_2509_06924_amd import inputs  # noqa: E402

DEPTHS = [300, 600, 1000, 1500, 2047]
DZ = 2.0
Q = np.geomspace(0.006, 0.3, 16)


def main():
    cases = []
    for i, L in enumerate(DEPTHS):
        seed = inputs.SEED_BASE + 60 + i
        rows = inputs.microsliced_stack(np.random.default_rng(seed), L, DZ)
        R = [mp_reference.parratt_R(rows.tolist(), float(q), dps=50) for q in Q]
        cases.append({"L": L, "dz": DZ, "seed": seed, "q": [float(q) for q in Q],
                      "R": [float(r) for r in R],
                      "R_text": [str(r)[:25] for r in R]})
        print(L, "done", flush=True)
    out = {"what": "R(q) of microsliced profiles (inputs.microsliced_stack(default_rng(seed), "
                   "L, dz)), unsmeared, by the Parratt recursion at 50 decimal digits "
                   "(oracle/mp_reference.py); R rounded to the nearest double",
           "cases": cases}
    with open(os.path.join(HERE, "deep_parratt50.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
