"""Write the oracle's stored reference series (calls only oracle/ and inputs).

    python tests/golden/make_oracle_golden.py

oracle_tg32_energy.txt: kinetic energy k(t) = (1/2)<|u - <u>|^2>, t = 0..100,
of the D3Q27 KBC (s = d+t+q) run on a 32^3 periodic box, rho = 1, Taylor-Green
start u = (U sin x cos y cos z, -U cos x sin y cos z, 0), U = 0.05,
nu = 0.001, populations initialised at the product-form equilibrium.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1507_02518_amd import inputs  # noqa: E402


def tg32():
    F = oracle.init_feq(inputs.taylor_green(32, 0.05))
    rows = []

    def cb(t, F):
        _, u = oracle.macros(F)
        rows.append((t, oracle.energy(u), oracle.enstrophy(u)))

    oracle.run(F, oracle.beta_from_nu(0.001), 100, callback=cb)
    path = os.path.join(HERE, "oracle_tg32_energy.txt")
    np.savetxt(path, np.array(rows), fmt=["%d", "%.17e", "%.17e"],
               header="t  k(t)  Omega(t)  | 32^3 Taylor-Green, U=0.05, nu=0.001, "
                      "s=d+t+q, written by make_oracle_golden.py from the oracle")
    print("wrote", path)


if __name__ == "__main__":
    tg32()
