"""Writes ed_4x4_periodic_U19.6.json: exact dynamics of the 4x4 periodic
Bose-Hubbard lattice (occupations truncated to n <= 2, the method's d = 3)
after the sudden quench of the unit-filling Mott state to U/J = 19.6
(Sec. III, the comparison with numerically exact results), in the N = 16
sector (5,196,627 states).  Calls only oracle/ed.py.  Takes about 15 minutes
and ~12 GB of memory on 8 cores.

    python tests/golden/make_ed_4x4_quench.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ed  # noqa: E402

T, NT = 1.0, 101


def main():
    t0 = time.time()
    s = ed.Sector(4, 4, 3, 16, True, 1.0, 19.6)
    print(f"sector {s.dim} states, H nnz {s.H.nnz}, {time.time() - t0:.0f} s", flush=True)
    times = np.linspace(0.0, T, NT)
    psi = s.evolve(s.fock([1] * 16), times)
    print(f"propagated, {time.time() - t0:.0f} s", flush=True)
    obs = []
    for k, p in enumerate(psi):
        obs.append(s.observables(p, translation_invariant=True).tolist())
        assert abs(np.vdot(p, p).real - 1.0) < 1e-9
    out = {
        "what": "exact <a_i^+ a_j>, <n_i n_j> class sums (oracle slots 0..9), density (10), energy per site (11)",
        "source": "Sec. III: 4x4 periodic lattice, unit-filling Mott state quenched to U/J = 19.6; "
                  "fixed-N sector ED with n <= 2 per site",
        "script": "tests/golden/make_ed_4x4_quench.py (oracle/ed.py only)",
        "Lx": 4, "Ly": 4, "d": 3, "J": 1.0, "U": 19.6, "sector_dim": int(s.dim),
        "times": times.tolist(), "obs": obs,
    }
    with open(os.path.join(HERE, "ed_4x4_periodic_U19.6.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"done, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
