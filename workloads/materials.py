"""Synthetic material parameter sets and interband polarizability tables.

The paper takes its Ag/Au/graphene parameters and interband permittivities
from its references; none of those numbers are available here, so each set in
``params/*.json`` is a stated, builder-chosen stand-in.  This module only loads
them and tabulates the interband polarizability alpha^IB(omega) that the dipole
model needs as *input data* (the role measured permittivity tables play in the
paper, Section 2.2): a single-Lorentzian interband permittivity mapped to a
per-atom polarizability by Clausius-Mossotti with the fcc volume per atom.
"""
from __future__ import annotations

import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

# order of the flat parameter vector handed to both implementations
PARAM_FIELDS = ("a_eff_bohr2", "r_q_bohr", "r_mu_bohr", "tau_au", "density_au",
                "eff_mass_au", "fermi_d", "fermi_s", "r0_ang", "cutoff_ang",
                "fermi_energy_ev", "sheet_thickness_bohr")


def load(name: str) -> dict:
    with open(os.path.join(_HERE, "params", name + ".json")) as f:
        return json.load(f)


def param_vector(p: dict) -> np.ndarray:
    return np.array([float(p[k]) for k in PARAM_FIELDS], dtype=np.float64)


def with_overrides(p: dict, **kw) -> dict:
    q = dict(p)
    q.update(kw)
    return q


def interband_alpha(p: dict, omega_ev) -> np.ndarray:
    """Synthetic alpha^IB(omega) (bohr^3, complex) on the given grid (eV).

    eps_IB(w) = eps_inf + S w0^2 / (w0^2 - w^2 - i g w);
    alpha = (3 V / 4 pi) (eps - 1) / (eps + 2)."""
    ib = p["interband"]
    w = np.asarray(omega_ev, dtype=np.float64)
    w0, g, s = ib["omega0_ev"], ib["gamma_ev"], ib["strength"]
    eps = ib["eps_inf"] + s * w0 ** 2 / (w0 ** 2 - w ** 2 - 1j * g * w)
    vol = ib["volume_per_atom_bohr3"]
    return (3.0 * vol / (4.0 * np.pi)) * (eps - 1.0) / (eps + 2.0)


def drude_permittivity(p: dict, omega_ev) -> np.ndarray:
    """Synthetic metal permittivity for the BEM workloads (complex, on the grid):
    eps(w) = eps_inf - w_p^2 / (w^2 + i gamma w) plus the material's interband
    Lorentzian if it has one (the same single-Lorentzian form as interband_alpha)."""
    w = np.asarray(omega_ev, dtype=np.float64)
    b = p["bem"]
    eps = b["eps_inf"] - b["omega_p_ev"] ** 2 / (w * w + 1j * b["gamma_ev"] * w)
    ib = p.get("interband")
    if ib is not None and b.get("with_interband", False):
        w0, g, st = ib["omega0_ev"], ib["gamma_ev"], ib["strength"]
        eps = eps + st * w0 ** 2 / (w0 ** 2 - w ** 2 - 1j * g * w)
    return eps
