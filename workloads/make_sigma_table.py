"""Writes sigma_opt_table.json: the Boyd-Kleinman optimum sigma_m(xi) on a grid
of focusing parameters, computed only with the oracle's focusing-function
quadrature (oracle.pins).  Run from the repository root:
    python -m workloads.make_sigma_table
"""
import json
import os

import numpy as np

from oracle import pins


def main():
    xs = np.round(np.arange(0.25, 5.5001, 0.01), 2)
    sig = [pins.bk_sigma_opt(float(x)) for x in xs]
    out = {"source": "oracle.pins.bk_sigma_opt (maximiser of h(sigma, xi), Eq. 17)",
           "xi": [float(x) for x in xs], "sigma_m": sig}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sigma_opt_table.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
