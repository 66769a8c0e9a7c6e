"""GPU parity of two-type structures (alloys, core-shell particles; Section 2.2,
Eqs. wfqfmu-leghe and polar-finale) against the FP64 oracle.

The second material differs from the first in every parameter the two-type
operator mixes (A, r0, d, s, cutoff, electron density, tau, alpha_IB), so a
dropped or misplaced factor of the unlike-pair exchange, the per-atom z_q or
the per-atom interband polarizability shows.  Tolerances as for one material:
operator apply 1e-11 (FP64 path) and 2e-4 (FP32 T-apply) of max|y|; spectra
1e-10 (FP64, rel_tol 1e-12) and 1e-5 (mixed, rel_tol 1e-8).
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


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


@pytest.fixture(scope="module", autouse=True)
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return px.load()


def materials(model):
    """(A, B): Ag and an Au-like material with every mixed parameter moved."""
    if model == 0:
        a = M.load("ag_wfq")
        b = M.with_overrides(a, a_eff_bohr2=2.4, r0_ang=2.80, cutoff_ang=3.35, fermi_d=10.0, fermi_s=1.05,
                             density_au=1.3 * a["density_au"], tau_au=a["tau_au"] / 3.0)
        return a, b
    a = M.load("ag_wfqfmu")
    b = M.with_overrides(M.load("au_wfqfmu"), a_eff_bohr2=2.4, r0_ang=2.80, cutoff_ang=3.35, fermi_d=10.0,
                         fermi_s=1.05, density_au=1.3 * a["density_au"])
    return a, b


def make(model, xyz, types, pa, pb):
    return px.Structure(model, xyz, pa, px.default_stream(), types=types, params_b=pb)


def aib_pair(pa, pb, om):
    return M.interband_alpha(pa, om), M.interband_alpha(pb, om)


# ------------------------------------------------------------ operator apply

@pytest.mark.parametrize("model,n", [(0, 300), (1, 300)])
def test_hetero_apply_matches_oracle(model, n):
    say(f"[hetero apply] model={model} n={n}")
    pa, pb = materials(model)
    xyz = G.fcc_sphere_n(n, seed=40 + n)
    types = G.alloy_types(n, 0.4, seed=41)
    s = make(model, xyz, types, pa, pb)
    rng = np.random.default_rng(n + model)
    nu = 4 * n if model else n
    ncol = 6
    x = rng.standard_normal((ncol, nu)) + 1j * rng.standard_normal((ncol, nu))
    om = np.linspace(1.5, 4.5, ncol)
    aa, ab = aib_pair(pa, pb, om) if model else (None, None)
    ref = O.apply_het(model, xyz, types, M.param_vector(pa), M.param_vector(pb), om, x, aa, ab)
    aib = None if aa is None else np.stack([aa, ab], axis=1)
    y64 = s.apply(px.PX_FP64, om, x, aib)
    y32 = s.apply(px.PX_MIXED, om, x, aib)
    e64, e32 = rel_err(y64, ref), rel_err(y32, ref)
    say(f"   fp64 err {e64:.2e}  fp32-T err {e32:.2e}")
    assert e64 <= 1e-11
    assert e32 <= 2e-4
    # narrow FP64 path (one complex column)
    y1 = s.apply(px.PX_FP64, om[:1], x[:1], None if aib is None else aib[:1])
    assert rel_err(y1, ref[:1]) <= 1e-11
    s.close()


# ------------------------------------------------------------ full solves

def _solve(model, xyz, types, pa, pb, om, pol, precision, rel_tol):
    s = make(model, xyz, types, pa, pb)
    aib = None
    if model == 1:
        aib = np.stack(aib_pair(pa, pb, om), axis=1)
    s.set_frequencies(om, pol, 1e-4, aib)
    st = s.solve(precision=precision, rel_tol=rel_tol)
    return s, st


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_alloy_dipole_spectrum_matches_oracle(precision, tol, bound):
    n = 260
    pa, pb = materials(1)
    xyz = G.fcc_sphere_n(n, seed=43)
    types = G.alloy_types(n, 0.5, seed=44)
    om = np.linspace(2.0, 4.0, 6)
    say(f"[hetero solve alloy] n={n} precision={precision}")
    aa, ab = aib_pair(pa, pb, om)
    ref = O.solve_spectrum_het(1, xyz, types, M.param_vector(pa), M.param_vector(pb), om, 0b011, 1e-4, aa, ab)
    assert ref["status"] == 0
    s, st = _solve(1, xyz, types, pa, pb, om, 0b011, precision, tol)
    it, cyc, rr = s.stats()
    alpha, sigma = s.spectrum()
    say(f"   status {st} iters max {it.max()} relres max {rr.max():.2e}")
    assert st == px.PX_OK and np.all(rr <= tol)
    e = rel_err(sigma, ref["sigma"])
    ea = rel_err(alpha[:, :, :2], ref["alpha"][:, :, :2])
    say(f"   rel_err sigma {e:.2e} alpha {ea:.2e}")
    assert e <= bound and ea <= 10 * bound
    q, mu = s.charges(4, 1, with_dipoles=True)
    assert rel_err(np.concatenate([q, mu.ravel()]), ref["q"][4, 1]) <= 100 * bound
    s.close()


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_core_shell_charge_model_matches_oracle(precision, tol, bound):
    """omegaFQ with two types: an Ag core in a shell of the second metal,
    ~700 atoms (several row tiles and a ragged tail), x and z columns."""
    n = 700
    pa, pb = materials(0)
    xyz = G.fcc_sphere_n(n, seed=45)
    types = G.core_shell_types(xyz, 0.6 * np.linalg.norm(xyz - xyz.mean(0), axis=1).max())
    om = np.array([2.4, 3.1, 3.6, 4.2])
    say(f"[hetero solve core-shell] n={n} shell atoms {int(types.sum())} precision={precision}")
    ref = O.solve_spectrum_het(0, xyz, types, M.param_vector(pa), M.param_vector(pb), om, 0b101, 1e-4)
    s, st = _solve(0, xyz, types, pa, pb, om, 0b101, precision, tol)
    it, cyc, rr = s.stats()
    say(f"   status {st} iters max {it.max()} relres max {rr.max():.2e}")
    assert st == px.PX_OK
    e = rel_err(s.spectrum()[1], ref["sigma"])
    say(f"   rel_err sigma {e:.2e}")
    assert e <= bound
    s.close()


def test_one_type_structure_equals_homogeneous():
    """All atoms of type A (or all of type B) is the one-material structure of
    A (or B): the two-type kernels must give its spectrum."""
    n = 240
    pa, pb = materials(1)
    xyz = G.fcc_rod_n(n, seed=46)
    om = np.linspace(2.2, 3.8, 5)
    for t, p in ((0, pa), (1, pb)):
        types = np.full(n, t, dtype=np.int32)
        s, st = _solve(1, xyz, types, pa, pb, om, 0b001, px.PX_FP64, 1e-12)
        assert st == px.PX_OK
        h = px.Structure(1, xyz, p, px.default_stream())
        h.set_frequencies(om, 0b001, 1e-4, M.interband_alpha(p, om))
        assert h.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
        e = rel_err(s.spectrum()[1], h.spectrum()[1])
        say(f"[hetero one type] all type {t}: vs one-material structure {e:.1e}")
        assert e <= 1e-10
        s.close()
        h.close()


def test_paper_alloy_full_size_residual_against_oracle_operator():
    """The 1289-atom Ag-Au alloy sphere at 50% Au, solved on the mixed path:
    at this size the oracle's dense solve takes minutes, so the check is the
    residual of the GPU solution under the oracle's own operator and
    right-hand side, ||b - A x|| / ||b|| <= 1e-7, at three frequencies."""
    c = C.alloy_sphere(0.5)
    om = c["omega_ev"]
    say(f"[hetero alloy 1289] {c['name']}")
    s = make(1, c["xyz"], c["types"], c["params_a"], c["params_b"])
    s.set_frequencies(om, c["pol_mask"], c["e0"], np.stack([c["alpha_ib_a"], c["alpha_ib_b"]], axis=1))
    assert s.solve(precision=px.PX_MIXED, rel_tol=1e-8) == px.PX_OK
    it, cyc, rr = s.stats()
    say(f"   iters max {it.max()} relres max {rr.max():.2e}")
    pa, pb = M.param_vector(c["params_a"]), M.param_vector(c["params_b"])
    for w in (0, len(om) // 2, len(om) - 1):
        q, mu = s.charges(w, 0, with_dipoles=True)
        x = np.concatenate([q, mu.ravel()])
        b = O.rhs_het(1, c["xyz"], c["types"], pa, pb, om[w], 0, c["e0"])
        ax = O.apply_het(1, c["xyz"], c["types"], pa, pb, om[w:w + 1], x, c["alpha_ib_a"][w:w + 1],
                         c["alpha_ib_b"][w:w + 1])[0]
        r = np.linalg.norm(b - ax) / np.linalg.norm(b)
        say(f"   w={om[w]:.3f} eV: oracle residual {r:.2e}")
        assert r <= 1e-7
    s.close()


def test_two_type_structures_refused_by_batch_and_server():
    pa, pb = materials(0)
    xyz = G.fcc_sphere_n(60, seed=47)
    s = make(0, xyz, G.alloy_types(60, 0.3, seed=48), pa, pb)
    s.set_frequencies(np.array([3.0]), 0b001)
    with pytest.raises(px.PxError) as e:
        px.solve_batch([s])
    assert e.value.status == px.PX_E_INVALID
    sv = px.Server(1e9, px.default_stream())
    with pytest.raises(px.PxError) as e:
        sv.submit(s)
    assert e.value.status == px.PX_E_INVALID
    sv.close()
    s.close()
