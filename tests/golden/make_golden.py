"""Writes the stored regression values under tests/golden/ from the oracle only.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from workloads import configs as C  # noqa: E402
from workloads import materials as M  # noqa: E402


def main():
    c = C.small_sphere()
    out = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    doc = dict(workload=c["name"], omega_ev=c["omega_ev"].tolist(), sigma_bohr2=out["sigma"].tolist(),
               alpha_xx_re=out["alpha"][:, 0, 0].real.tolist(), alpha_xx_im=out["alpha"][:, 0, 0].imag.tolist(),
               writer="tests/golden/make_golden.py (oracle only)")
    with open(os.path.join(HERE, "small_sphere_sigma.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
