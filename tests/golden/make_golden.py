"""Writes oracle_smallcase.json: FP64 oracle outputs on a tiny seeded case.

Calls only oracle/ and the seeded input generator.  The fixture guards the oracle
against unintended changes; its values were pinned independently by
tests/test_oracle_pins.py when written.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2603_15285_amd import synth as S  # noqa: E402


def main():
    b = S.make_batch(6, 4, 2, seed=77, snr=0.5)
    out = {"seed": 77, "L": 6, "R": 4, "B": 3, "n": 12, "Kc": 4, "levels": [3, 4, 6], "steps": 3, "particles": []}
    for p in range(2):
        C = O.coeff_assemble(6, 4, b.f(p), 6, b.h, 6, b.w)
        e = O.evaluate(6, C, [0.4, 1.2, 2.2])
        best, bi, st, cand = O.align_one(b.f(p), 6, 4, b.h, 6, b.w, 3, 12, 4, [3, 4, 6], 3)
        out["particles"].append({
            "C_l2": [[float(z.real), float(z.imag)] for z in C[O.blk(2):O.blk(3)]],
            "eval_at_0.4_1.2_2.2": [float(x) for x in e],
            "best": [float(x) for x in best], "best_idx": int(bi), "status": int(st),
        })
    with open(os.path.join(HERE, "oracle_smallcase.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
