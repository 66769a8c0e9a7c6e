"""Post-processing on the GPU: the field and density of the induced Gaussian
charges and dipoles at probe points (pxProbeField, pxInducedField) against the
oracle (or_probe), element by element.

Sources are seeded random charges (and dipoles) given to both sides, or each
side's own solve of the same spectrum.  Point sets: grid lines through and
around the structure (spatially ordered, as CUBE grids and plane maps are),
scattered points, the atom centres themselves and points inside the Taylor
series region of an atom (r < R/2), in counts that leave a ragged last wave.
Bound: 1e-11 of the largest value for given sources (FP64 on both sides; the
GPU's point path beyond 7 widths drops Gaussian tails below 1e-20); 1e-8 for
solved columns (the GPU's solve to rel_tol 1e-11, the oracle's LU).
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2510_12731_amd as px
from workloads import configs as C
from workloads import geometry as G
from workloads import materials as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return px.load()


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def point_set(xyz, rng, r_units):
    """Lines through the structure, scattered points, atom centres and points
    within r < R/2 of atoms (Angstrom)."""
    lo, hi = xyz.min(0) - 4.0, xyz.max(0) + 4.0
    line = np.linspace(lo[0], hi[0], 300)
    pts = [np.stack([line, np.full_like(line, 0.3 * lo[1] + 0.7 * hi[1]), np.full_like(line, xyz[:, 2].mean())], 1),
           np.stack([np.full(200, xyz[:, 0].mean()), np.linspace(lo[1], hi[1], 200), np.linspace(lo[2], hi[2], 200)], 1),
           lo + (hi - lo) * rng.random((237, 3)),
           xyz[rng.choice(len(xyz), 40, replace=False)],
           xyz[rng.choice(len(xyz), 60, replace=False)] + rng.normal(scale=0.15 * r_units, size=(60, 3)),
           np.array([[200.0, -150.0, 90.0]])]
    return np.concatenate(pts, 0)


def make(model, xyz, params):
    return px.Structure(model, xyz, params, px.default_stream())


@pytest.mark.parametrize("model", [0, 1])
def test_probe_given_sources_match_oracle(model):
    rng = np.random.default_rng(11 + model)
    if model == 0:
        xyz, params = G.fcc_sphere_n(700, seed=9), M.load("ag_wfq")
    else:
        xyz, params = G.fcc_rod_n(420, seed=9), M.load("au_wfqfmu")
    n = len(xyz)
    q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    mu = (rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))) * 0.3 if model else None
    rq_ang = params["r_q_bohr"] * 0.529177210903
    pts = point_set(xyz, rng, rq_ang)
    say(f"[probe] model {model}: {n} atoms, {len(pts)} points")
    s = make(model, xyz, params)
    f, rho = s.probe_field(q, mu, pts)
    st = s.probe_stats()
    ref = O.probe(model, xyz, M.param_vector(params), q, mu, pts)
    ef, er = rel(f, ref["field"]), rel(rho, ref["rho"])
    say(f"   field {ef:.2e} density {er:.2e}  kernel {st['ms_kernel']:.3f} ms, {st['pairs']:.0f} pairs")
    assert ef <= 1e-11 and er <= 1e-11
    assert st["pairs"] == len(pts) * n
    # dipoles left out of a dipole-model structure: charges only
    if model == 1:
        f0, r0 = s.probe_field(q, None, pts[:100])
        ref0 = O.probe(1, xyz, M.param_vector(params), q, np.zeros((3, n)), pts[:100])
        assert rel(f0, ref0["field"]) <= 1e-11 and rel(r0, ref0["rho"]) <= 1e-11
    s.close()


@pytest.mark.parametrize("model", [0, 1])
def test_induced_field_of_solved_column_matches_oracle_solve(model):
    if model == 0:
        c = C.small_sphere()
        xyz, params, om, pol = c["xyz"], c["params"], c["omega_ev"][20:23], 0b001
        aib = None
    else:
        xyz, params = G.fcc_sphere_n(140, seed=4), M.load("au_wfqfmu")
        om, pol = np.array([2.2, 2.5]), 0b010
        aib = M.interband_alpha(params, om)
    rng = np.random.default_rng(5)
    pts = point_set(xyz, rng, params["r_q_bohr"] * 0.529177210903)
    s = make(model, xyz, params)
    s.set_frequencies(om, pol, 1e-4, aib)
    assert s.solve(precision=px.PX_FP64, rel_tol=1e-11) == px.PX_OK
    ref = O.solve_spectrum(model, xyz, M.param_vector(params), om, pol, 1e-4, aib)
    lpol = [l for l in range(3) if pol & (1 << l)][0]
    n = len(xyz)
    for w in range(len(om)):
        f, rho = s.induced_field(w, lpol, pts)
        qo = ref["q"][w, 0]
        rq = O.probe(model, xyz, M.param_vector(params), qo[:n], qo[n:].reshape(3, n) if model else None, pts)
        ef, er = rel(f, rq["field"]), rel(rho, rq["rho"])
        say(f"[induced] model {model} w {om[w]:.2f} eV: field {ef:.2e} density {er:.2e}")
        assert ef <= 1e-8 and er <= 1e-8
    # outside the solved set / before a solve
    with pytest.raises(px.PxError):
        s.induced_field(0, 2, pts[:4])
    t = make(model, xyz, params)
    with pytest.raises(px.PxError):
        t.induced_field(0, 0, pts[:4])
    t.close()
    s.close()


def test_probe_many_points_in_batches_and_empty():
    """2^20 + 300 points (two batches) on a 200-atom sphere: a sample of them
    against the oracle; an empty point set is a no-op."""
    rng = np.random.default_rng(2)
    xyz, params = G.fcc_sphere_n(200, seed=2), M.load("ag_wfq")
    n = len(xyz)
    q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lo, hi = xyz.min(0) - 3.0, xyz.max(0) + 3.0
    m = 102
    ax = [np.linspace(lo[a], hi[a], m) for a in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)[: (1 << 20) + 300]
    s = make(0, xyz, params)
    f, rho = s.probe_field(q, None, pts)
    idx = np.concatenate([rng.choice(len(pts), 1500, replace=False), np.arange(len(pts) - 40, len(pts)),
                          np.arange((1 << 20) - 20, (1 << 20) + 20)])
    ref = O.probe(0, xyz, M.param_vector(params), q, None, pts[idx])
    say(f"[probe batches] {len(pts)} points: field {rel(f[idx], ref['field']):.2e} density {rel(rho[idx], ref['rho']):.2e}")
    assert rel(f[idx], ref["field"]) <= 1e-11 and rel(rho[idx], ref["rho"]) <= 1e-11
    f0, r0 = s.probe_field(q, None, np.zeros((0, 3)))
    assert f0.shape == (0, 3) and r0.shape == (0,) and s.probe_stats()["pairs"] == 0
    bad = pts[:10].copy()
    bad[3, 1] = np.nan
    with pytest.raises(px.PxError):
        s.probe_field(q, None, bad)
    with pytest.raises(px.PxError):
        s.probe_field(q, np.zeros((3, n)), pts[:4])   # dipoles for an omegaFQ structure
    s.close()


def test_probe_full_size_sphere_sampled():
    """The 20,000-atom sphere with seeded charges on a 64^3 grid around it (the
    launch the benchmark times): 300 sampled points against the oracle."""
    case = C.sphere_20k()
    xyz = case["xyz"]
    rng = np.random.default_rng(8)
    n = len(xyz)
    q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lo, hi = xyz.min(0) - 5.0, xyz.max(0) + 5.0
    ax = [np.linspace(lo[a], hi[a], 64) for a in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    s = make(0, xyz, case["params"])
    f, rho = s.probe_field(q, None, pts)
    st = s.probe_stats()
    idx = rng.choice(len(pts), 300, replace=False)
    ref = O.probe(0, xyz, M.param_vector(case["params"]), q, None, pts[idx])
    ef, er = rel(f[idx], ref["field"]), rel(rho[idx], ref["rho"])
    say(f"[probe 20k] {len(pts)} points: field {ef:.2e} density {er:.2e}, kernel {st['ms_kernel']:.2f} ms")
    assert ef <= 1e-11 and er <= 1e-10
    s.close()
