"""Write tests/golden/K256_cube64.json: reference values of the K = 256
workload (64-atom cube, seed 0, order 400, beta 100, N_e = 128) computed by
the FP64 oracle only.  Run from the repository root:

    python tests/golden/make_golden.py

The values are the oracle's, not the paper's (the paper prints no worked
example of this path); they pin the oracle against accidental change and
give the GPU tests stored targets."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import WORKLOADS, workload  # noqa: E402

ENTRIES = [(0, 0), (5, 17), (100, 200), (17, 5), (255, 255), (128, 3)]


def main():
    name = "K256_cube64_fp64"
    w = WORKLOADS[name]
    c = workload(name)
    sp = O.spectrum(c)
    width = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * width, sp.e[-1] + 0.01 * width
    N, beta, ne = w["order"], w["beta"], w["n_electrons"]
    mu = O.solve_mu_poly(sp, ne, N, beta, emin, emax, tol=1e-12)
    tr, eb = O.trace_poly(sp, N, mu, beta, emin, emax)
    P = O.density_matrix_poly(sp, np.arange(c.K), N, mu, beta, emin, emax)
    m = O.moments_from_eigs(sp.e, 10, emin, emax)
    out = {
        "workload": name, "K": c.K, "order": N, "beta": beta, "n_electrons": ne,
        "emin": emin, "emax": emax, "eig_min": float(sp.e[0]), "eig_max": float(sp.e[-1]),
        "mu": mu, "tr_PS": tr, "band_energy": eb, "moments_0_9": [float(x) for x in m],
        "P_entries": [[i, j, float(P[i, j])] for i, j in ENTRIES],
        "P_sum": float(P.sum()), "P_abs_max": float(np.abs(P).max()),
        "note": "written by tests/golden/make_golden.py from oracle/ only",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "K256_cube64.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
