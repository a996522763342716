"""Write exact_tier_l6.json: exact-tier values (25 significant digits) of the
harmonics, gradients and Hessians at a few points, l_max = 6.

Calls only the oracle's definition tier (explicit polynomials evaluated in
mpmath).  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mpmath  # noqa: E402

from oracle import definition_eval_mp  # noqa: E402

POINTS = [(0.3, -1.25, 0.8), (1e-9, -3e-10, -0.6), (0.0, 0.0, 1.0)]
L = 6


def main():
    cases = []
    for p in POINTS:
        for normalize in (False, True):
            Y, G, H = definition_eval_mp(p, L, normalize, dps=60, hessian=True)
            s = lambda v: mpmath.nstr(v, 25)  # noqa: E731
            cases.append({
                "point": [float(c).hex() for c in p],
                "normalize": normalize,
                "Y": [s(v) for v in Y],
                "dY": [[s(v) for v in row] for row in G],
                "H": [[[s(v) for v in row] for row in blk] for blk in H],
            })
    out = {"l_max": L, "source": "oracle.definition_eval_mp at 60 digits", "cases": cases}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_tier_l6.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
