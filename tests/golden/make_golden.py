"""Write the stored expected values of tests/golden/ (calls only the oracle)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402


def main():
    _, star = oracle.riemann_conformal(1.0, 1.0, 0.1, 0.125, np.zeros(1))
    rec = {"source": "oracle.riemann_conformal(eL=1, nL=1, eR=0.1, nR=0.125)",
           "problem": "relativistic shock tube, conformal EOS p = e/3, both states at rest",
           "star": {k: float(v) for k, v in star.items()}}
    with open(os.path.join(HERE, "sod_star.json"), "w") as f:
        json.dump(rec, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    main()
