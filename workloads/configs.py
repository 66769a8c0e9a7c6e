"""The five workload recipes (sizes, grids, seeds) as concrete inputs.

Each recipe returns a plain dict:
  model      0 = omegaFQ, 1 = omegaFQFmu
  xyz        (N, 3) float64 coordinates in Angstrom
  params     material parameter dict (see materials.py)
  omega_ev   frequency grid in eV (inclusive linspace)
  pol_mask   bit0 x, bit1 y, bit2 z
  e0         applied field amplitude (a.u.)
  alpha_ib   complex interband polarizability per frequency (dipole model) or None
"""
from __future__ import annotations

import numpy as np

from . import geometry as G
from . import materials as M

E0 = 1e-4  # a.u., the field amplitude the paper uses for its timings


def _case(model, xyz, params, omega_ev, pol_mask, name, **extra):
    alpha_ib = M.interband_alpha(params, omega_ev) if model == 1 else None
    d = dict(name=name, model=model, xyz=np.ascontiguousarray(xyz, dtype=np.float64),
             params=params, omega_ev=np.asarray(omega_ev, dtype=np.float64),
             pol_mask=pol_mask, e0=E0, alpha_ib=alpha_ib)
    d.update(extra)
    return d


def small_sphere():
    """Ag fcc sphere, radius 1.0 nm (249 atoms), 50 frequencies 1-6 eV, x."""
    xyz = G.fcc_sphere_radius(10.0, jitter=0.01, seed=1)
    return _case(0, xyz, M.load("ag_wfq"), np.linspace(1.0, 6.0, 50), 0b001,
                 "ag_sphere_249_wfq_50w_x")


def sphere_20k(n=20000, n_omega=128):
    """Ag fcc sphere of 20,000 atoms, 128 frequencies 2-5 eV x {x,y,z}."""
    xyz = G.fcc_sphere_n(n, jitter=0.01, seed=2)
    return _case(0, xyz, M.load("ag_wfq"), np.linspace(2.0, 5.0, n_omega), 0b111,
                 f"ag_sphere_{n}_wfq_{n_omega}w_xyz")


def rod_10k(n=10000, n_omega=96):
    """Au fcc rod (aspect 3 along z) of 10,000 atoms, omegaFQFmu, 96 frequencies
    1.5-3.5 eV, z polarization."""
    xyz = G.fcc_rod_n(n, aspect=3.0, jitter=0.01, seed=3)
    return _case(1, xyz, M.load("au_wfqfmu"), np.linspace(1.5, 3.5, n_omega), 0b100,
                 f"au_rod_{n}_wfqfmu_{n_omega}w_z")


def graphene_batch(n_struct=64, n_min=2000, n_max=60000, n_omega=64, seed=4):
    """64 honeycomb disks and ribbons, N log-uniform in [2k, 60k], E_F ~ U(0.2, 0.6) eV,
    64 frequencies 0.1-1.0 eV, in-plane x polarization."""
    rng = np.random.default_rng(seed)
    base = M.load("graphene_wfq")
    out = []
    for k in range(n_struct):
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        ef = float(rng.uniform(0.2, 0.6))
        p = M.with_overrides(base, fermi_energy_ev=ef)
        if k % 2 == 0:
            xyz = G.graphene_disk_n(n)
            shape = "disk"
        else:
            width = float(rng.uniform(20.0, 100.0))
            zig = bool(rng.integers(0, 2))
            xyz = G.graphene_ribbon_n(n, width, zigzag=zig)
            shape = "ribbon_zz" if zig else "ribbon_ac"
        out.append(_case(0, xyz, p, np.linspace(0.1, 1.0, n_omega), 0b001,
                         f"graphene_{shape}_{n}", fermi_energy_ev=ef))
    return out


def serving_request(rng, n_min=1000, n_max=100000):
    """One seeded serving request: Ag/Au sphere, rod or gap dimer, omegaFQ or
    omegaFQFmu, 32-128 frequencies on the model's window, one polarization."""
    shape = ["sphere", "rod", "dimer"][int(rng.integers(0, 3))]
    metal = ["ag", "au"][int(rng.integers(0, 2))]
    model = int(rng.integers(0, 2))
    n = int(rng.integers(n_min, n_max + 1))
    n_omega = int(rng.integers(32, 129))
    seed = int(rng.integers(0, 2 ** 31 - 1))
    if shape == "sphere":
        xyz = G.fcc_sphere_n(n, seed=seed)
    elif shape == "rod":
        xyz = G.fcc_rod_n(n, seed=seed)
    else:
        xyz = G.gap_dimer(n, gap=float(rng.uniform(3.0, 10.0)), seed=seed)
    pol = 1 << int(rng.integers(0, 3))
    if model == 0:
        params = M.load("ag_wfq")
        grid = np.linspace(2.0, 5.0, n_omega)
    else:
        params = M.load("au_wfqfmu" if metal == "au" else "ag_wfqfmu")
        grid = np.linspace(1.5, 4.5, n_omega)
    return _case(model, xyz, params, grid, pol, f"{metal}_{shape}_{n}_m{model}_{n_omega}w")


def alloy_sphere(frac_au, n=1289, step_ev=0.01, seed=7):
    """Ag-Au nanoalloy sphere of n atoms (the paper's D = 3.5 nm, 1289-atom
    alloys), Au atoms substituted at random with fraction frac_au (the same Ag
    sphere for every fraction), omegaFQFmu with two atom types, frequencies
    2.0-4.5 eV in steps of step_ev (251 at 0.01 eV), x, y and z polarizations."""
    xyz = G.fcc_sphere_n(n, jitter=0.01, seed=seed)
    ag, au = M.load("ag_wfqfmu"), M.load("au_wfqfmu")
    om = np.round(np.arange(2.0, 4.5 + 0.5 * step_ev, step_ev), 10)
    return dict(model=1, xyz=xyz, types=G.alloy_types(n, frac_au, seed=seed + 1), params_a=ag, params_b=au,
                omega_ev=om, pol_mask=0b111, e0=E0, alpha_ib_a=M.interband_alpha(ag, om),
                alpha_ib_b=M.interband_alpha(au, om), name=f"agau_alloy_{n}_{int(round(100 * frac_au))}au_wfqfmu")
