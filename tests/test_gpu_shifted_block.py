"""The shared-Krylov phase over a block of polarizations (shifted = 2): one
block Arnoldi process for the 2 or 3 right-hand sides of a one-material
omegaFQ structure, every (frequency, polarization) pair's GMRES iterate over
all kR directions from one banded QR per frequency, then the blocked solver
for whatever is left.

Parity with the oracle at the bounds of test_gpu_parity (FP64 at rel_tol
1e-12 / 1e-11: 1e-10 on sigma; mixed at 1e-8: 1e-5) for two and three
polarizations, with the phase capped so that the blocked solver finishes from
its iterate; a flat structure whose z right-hand side is zero falls back to one
process per polarization; against the per-polarization phase on a 1,500-atom
sphere (same spectrum, fewer steps); identical right-hand sides (a block
deflated at step 0) and a single frequency.
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


def solve(xyz, params, om, pol, precision, tol, **kw):
    s = px.Structure(0, xyz, params, px.default_stream())
    s.set_frequencies(om, pol, 1e-4)
    st = s.solve(precision=precision, rel_tol=tol, **kw)
    alpha, sigma = s.spectrum()
    it, cyc, rr = s.stats()
    return s, st, alpha, sigma, it, cyc, rr


@pytest.mark.parametrize("pol", [0b111, 0b011, 0b110])
def test_block_phase_matches_oracle(pol):
    """The small sphere (spread frequencies, ragged pair count), FP64 at
    rel_tol 1e-12: every pair converges inside the block phase."""
    c = C.small_sphere()
    om = c["omega_ev"][::3]
    say(f"[block] small sphere {len(c['xyz'])} atoms, {len(om)} frequencies, pol {pol:03b}")
    ref = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), om, pol, 1e-4)
    s, st, alpha, sigma, it, cyc, rr = solve(c["xyz"], c["params"], om, pol, px.PX_FP64, 1e-12, shifted=2)
    say(f"   status {st} block steps max {it.max()} cycles max {cyc.max()} relres max {rr.max():.2e}")
    assert st == px.PX_OK and rr.max() <= 1e-12
    assert cyc.max() == 1, "every column converges in the block phase"
    e, ea = rel_err(sigma, ref["sigma"]), rel_err(alpha, ref["alpha"])
    say(f"   rel_err sigma {e:.2e} alpha {ea:.2e}")
    assert e <= 1e-10 and ea <= 1e-9
    for w in (0, len(om) // 2, len(om) - 1):
        for ip, l in enumerate(k for k in range(3) if pol & (1 << k)):
            assert rel_err(s.charges(w, l), ref["q"][w, ip]) <= 1e-8
    s.close()


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_capped_block_phase_hands_over_to_blocked_solver(precision, tol, bound):
    """With the block phase capped at 7 steps the blocked solver finishes
    every column from the phase's iterate."""
    c = C.small_sphere()
    ref = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], 0b111, 1e-4)
    s, st, alpha, sigma, it, cyc, rr = solve(c["xyz"], c["params"], c["omega_ev"], 0b111, precision, tol,
                                             shifted=2, shifted_max_steps=7)
    say(f"[block capped] precision={precision}: status {st} iters max {it.max()} cycles max {cyc.max()} "
        f"relres max {rr.max():.2e}")
    assert st == px.PX_OK and rr.max() <= tol
    assert cyc.max() >= 2
    e = rel_err(sigma, ref["sigma"])
    say(f"   rel_err sigma {e:.2e}")
    assert e <= bound
    s.close()


def test_block_phase_checks_true_residuals_through_its_basis():
    """128 frequencies x 3 polarizations of the small sphere: the phase's
    basis (k R real columns) is narrower than the pairs' 768 real columns, so
    every pair's true FP64 residual comes from one apply over the basis
    (T x = (T V) y, then b - (Kbar T x - z x)) instead of one over all pairs;
    the spectrum matches the oracle and every pair ends inside the phase."""
    c = C.small_sphere()
    om = np.linspace(float(c["omega_ev"].min()), float(c["omega_ev"].max()), 128)
    say(f"[block basis residual] small sphere {len(c['xyz'])} atoms, {len(om)} frequencies, xyz")
    ref = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), om, 0b111, 1e-4)
    s, st, alpha, sigma, it, cyc, rr = solve(c["xyz"], c["params"], om, 0b111, px.PX_FP64, 1e-11, shifted=2)
    tm = s.timings()
    applied = tm["cols_f64_padded"] - 3 * (tm["n_tapply_f64"] - 1)
    say(f"   status {st} block steps max {it.max()} cycles max {cyc.max()} relres max {rr.max():.2e}; "
        f"residual apply over {applied} real columns")
    assert st == px.PX_OK and rr.max() <= 1e-11 and cyc.max() == 1
    assert applied < 2 * len(om) * 3, "the residual check went through the basis"
    e, ea = rel_err(sigma, ref["sigma"]), rel_err(alpha, ref["alpha"])
    say(f"   rel_err sigma {e:.2e} alpha {ea:.2e}")
    assert e <= 1e-10 and ea <= 1e-9
    s.close()


def test_flat_structure_falls_back_per_polarization():
    """A graphene disk's z right-hand side is zero: shifted = 2 runs one
    process per polarization there, with the same result as shifted = 1; its
    in-plane pair (x, y) takes the block phase."""
    xyz = G.graphene_disk_n(400)
    p = M.with_overrides(M.load("graphene_wfq"), fermi_energy_ev=0.4)
    om = np.linspace(0.15, 1.0, 24)
    ref = O.solve_spectrum(0, xyz, M.param_vector(p), om, 0b111, 1e-4)
    s2, st2, a2, sig2, it2, cyc2, rr2 = solve(xyz, p, om, 0b111, px.PX_FP64, 1e-11, shifted=2)
    s1, st1, a1, sig1, it1, cyc1, rr1 = solve(xyz, p, om, 0b111, px.PX_FP64, 1e-11, shifted=1)
    say(f"[block flat] status {st2}/{st1} steps {it2.max()}/{it1.max()} relres {rr2.max():.1e}")
    assert st2 == px.PX_OK and np.array_equal(it2, it1)
    assert rel_err(sig2, ref["sigma"]) <= 1e-10 and rel_err(sig2, sig1) <= 1e-13
    s2.close()
    s1.close()
    ref = O.solve_spectrum(0, xyz, M.param_vector(p), om, 0b011, 1e-4)
    s, st, alpha, sigma, it, cyc, rr = solve(xyz, p, om, 0b011, px.PX_FP64, 1e-11, shifted=2)
    e = rel_err(sigma, ref["sigma"])
    say(f"[block flat xy] status {st} block steps {it.max()} cycles {cyc.max()} sigma {e:.2e}")
    assert st == px.PX_OK and cyc.max() == 1 and e <= 1e-10
    s.close()


def test_block_phase_agrees_with_per_polarization_phase_in_fewer_steps():
    """1,500-atom sphere, 40 frequencies x 3 polarizations, FP64 at 1e-11:
    the same spectrum as one process per polarization, in fewer steps (each
    one T-apply of the same three vectors)."""
    xyz = G.fcc_sphere_n(1500, seed=23)
    p = M.load("ag_wfq")
    om = np.linspace(2.0, 5.0, 40)
    s2, st2, a2, sig2, it2, cyc2, rr2 = solve(xyz, p, om, 0b111, px.PX_FP64, 1e-11, shifted=2)
    s1, st1, a1, sig1, it1, cyc1, rr1 = solve(xyz, p, om, 0b111, px.PX_FP64, 1e-11, shifted=1)
    e, ea = rel_err(sig2, sig1), rel_err(a2, a1)
    tm2, tm1 = s2.timings(), s1.timings()
    say(f"[block vs per-pol] N=1500: steps {it2.max()} vs {it1.max()}, cycles {cyc2.max()}/{cyc1.max()}, "
        f"sigma {e:.1e} alpha {ea:.1e}, T-apply launches {tm2['n_tapply_f64']:.0f} vs {tm1['n_tapply_f64']:.0f}")
    assert st2 == px.PX_OK and st1 == px.PX_OK and cyc2.max() == 1
    assert e <= 1e-10 and ea <= 1e-9
    assert it2.max() < it1.max()
    s2.close()
    s1.close()


def test_block_step_cap_reports_not_converged():
    c = C.small_sphere()
    s = px.Structure(0, c["xyz"], c["params"], px.default_stream())
    s.set_frequencies([3.5, 3.6], 0b011)
    st = s.solve(precision=px.PX_FP64, rel_tol=1e-12, shifted=2, shifted_max_steps=3, max_cycles=1)
    assert st == px.PX_E_NOTCONV
    it, cyc, rr = s.stats()
    assert (it == 3).all() and (cyc == 1).all() and (rr > 1e-12).all()
    assert np.isfinite(s.spectrum()[1]).all()
    s.close()


def test_block_deflates_identical_right_hand_sides():
    """A chain along (1, 1, 0) has x_i = y_i, so b_x = b_y: the block of step 0
    is rank-deficient, its second column is deflated at once and both
    polarizations share one Krylov space.  Also one frequency with three
    polarizations (a single banded QR)."""
    d = 2.9
    t = np.arange(60, dtype=float)
    xyz = np.stack([d * t / np.sqrt(2.0), d * t / np.sqrt(2.0), np.zeros_like(t)], 1)
    p = M.load("ag_wfq")
    om = np.linspace(1.5, 5.0, 9)
    ref = O.solve_spectrum(0, xyz, M.param_vector(p), om, 0b011, 1e-4)
    s, st, alpha, sigma, it, cyc, rr = solve(xyz, p, om, 0b011, px.PX_FP64, 1e-11, shifted=2)
    e = rel_err(sigma, ref["sigma"])
    say(f"[block deflation] chain 60: status {st} steps {it.max()} cycles {cyc.max()} relres {rr.max():.1e} sigma {e:.2e}")
    assert st == px.PX_OK and cyc.max() == 1 and e <= 1e-10
    for w in (0, 8):
        qx, qy = s.charges(w, 0), s.charges(w, 1)
        assert rel_err(qx, ref["q"][w, 0]) <= 1e-8 and rel_err(qy, ref["q"][w, 1]) <= 1e-8
    s.close()
    c = C.small_sphere()
    ref = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), [3.3], 0b111, 1e-4)
    s, st, alpha, sigma, it, cyc, rr = solve(c["xyz"], c["params"], [3.3], 0b111, px.PX_FP64, 1e-12, shifted=2)
    say(f"[block one frequency] status {st} steps {it.max()} sigma {rel_err(sigma, ref['sigma']):.2e}")
    assert st == px.PX_OK and cyc.max() == 1 and rel_err(sigma, ref["sigma"]) <= 1e-10
    s.close()
