"""Write the stored expected values under tests/golden/ (calls only the oracle).

The paper prints no worked numeric example for its solver (its figures are images), so the
stored values here are the oracle's own results on small fixed inputs.  The oracle is pinned
independently (tests/test_oracle_pins.py); these files guard it against silent change and give
the GPU tests fixed small cases.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from workloads import make_random  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "oracle_cases.json")


def case(name, W, H, x, y, w, h, Mu, Mp, cite):
    E, a, I = oracle.energy(W, H, x, y, w, h, Mu, Mp)
    gx, gy = oracle.grad(W, H, x, y, w, h, a)
    return dict(name=name, cite=cite, W=W, H=H, Mu=Mu, Mp=Mp,
                x=list(map(float, x)), y=list(map(float, y)), w=list(map(float, w)), h=list(map(float, h)),
                E=E, a_corner=a[:4, :4].tolist(), gx=list(map(float, gx)), gy=list(map(float, gy)))


def main():
    cases = []
    blocks = [(2.0, 2.0, 2.0, 1.0), (5.5, 4.0, 1.0, 3.0), (4.0, 4.5, 1.5, 0.5), (6.75, 1.25, 0.5, 0.5)]
    x, y, w, h = (np.array(v) for v in zip(*blocks))
    cases.append(case("four_blocks_8x6", 8.0, 6.0, x, y, w, h, 96, 80,
                      "Sec. III-A closed-form coefficients; energy 1/2 iint rho psi (Sec. II-B)"))
    wl = make_random(37, 100.0, 60.0, 24, 20, seed=1)
    cases.append(case("random37_100x60", wl.W, wl.H, *wl.arrays(), wl.Mu, wl.Mp,
                      "Sec. III-A closed-form coefficients; energy 1/2 iint rho psi (Sec. II-B)"))
    with open(OUT, "w") as f:
        json.dump(dict(generator="tests/golden/make_golden.py (oracle only)", cases=cases), f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
