"""The shared-Krylov phase for one-material omegaFQ structures: one real
Arnoldi process per polarization on Kbar T, every frequency's GMRES iterate
from its own Givens QR of the shifted Hessenberg matrix, then the blocked
solver for whatever is left.

Parity with the oracle at the bounds of test_gpu_parity (FP64 at rel_tol
1e-12, 1e-11 for graphene: 1e-10 on sigma; mixed at 1e-8: 1e-5), for one, two and three
polarizations (2 and 4 interleaved slots, a polarization whose right-hand
side is zero), with the phase capped so that the blocked solver has to finish
from its iterate, and against the blocked solver alone.
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
    kw.setdefault("shifted", 1)
    s = px.Structure(0, xyz, params, px.default_stream())
    s.set_frequencies(om, pol, 1e-4)
    st = s.solve(precision=precision, rel_tol=tol, **kw)
    alpha, sigma = s.spectrum()
    it, cyc, rr = s.stats()
    return s, st, alpha, sigma, it, cyc, rr


def graphene(n):
    return G.graphene_disk_n(n), M.with_overrides(M.load("graphene_wfq"), fermi_energy_ev=0.4)


@pytest.mark.parametrize("pol", [0b001, 0b011, 0b111, 0b101])
def test_polarization_layouts_match_oracle(pol):
    """Graphene disk (flat: its z right-hand side is zero), FP64 at rel_tol
    1e-11 (the disk's FP64 residual floor near its plasmon is ~2e-12)."""
    xyz, p = graphene(400)
    om = np.linspace(0.15, 1.0, 24)
    say(f"[shifted] graphene 400, pol {pol:03b}")
    ref = O.solve_spectrum(0, xyz, M.param_vector(p), om, pol, 1e-4)
    s, st, alpha, sigma, it, cyc, rr = solve(xyz, p, om, pol, px.PX_FP64, 1e-11)
    say(f"   status {st} iters max {it.max()} cycles max {cyc.max()} relres max {rr.max():.2e}")
    assert st == px.PX_OK and rr.max() <= 1e-11
    assert cyc.max() == 1, "every column converges in the shared-Krylov phase"
    e = rel_err(sigma, ref["sigma"])
    ea = rel_err(alpha, ref["alpha"])
    say(f"   rel_err sigma {e:.2e} alpha {ea:.2e}")
    assert e <= 1e-10 and ea <= 1e-9
    npol = bin(pol).count("1")
    for w in (0, 11, 23):
        for ip, l in enumerate(k for k in range(3) if pol & (1 << k)):
            q = s.charges(w, l)
            assert rel_err(q, ref["q"][w, ip]) <= 1e-8 if np.abs(ref["q"][w, ip]).max() > 0 else \
                np.abs(q).max() == 0.0
    s.close()


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_capped_phase_hands_over_to_blocked_solver(precision, tol, bound):
    """With the phase capped at 20 steps most columns are left above rel_tol
    and the blocked solver finishes them from the phase's iterate."""
    c = C.small_sphere()
    ref = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    s, st, alpha, sigma, it, cyc, rr = solve(c["xyz"], c["params"], c["omega_ev"], c["pol_mask"], precision, tol,
                                             shifted_max_steps=20)
    say(f"[shifted capped] precision={precision}: status {st} iters max {it.max()} cycles max {cyc.max()} "
        f"relres max {rr.max():.2e}")
    assert st == px.PX_OK and rr.max() <= tol
    assert cyc.max() >= 2
    e = rel_err(sigma, ref["sigma"])
    say(f"   rel_err sigma {e:.2e}")
    assert e <= bound
    s.close()


def test_shared_phase_agrees_with_blocked_solver_and_uses_fewer_t_applies():
    """Same spectrum as the blocked solver alone (both FP64 at 1e-11, above
    the FP64 residual floor at this size), with one narrow T-apply per step
    instead of one per column block and step."""
    xyz = G.fcc_sphere_n(1500, seed=23)
    p = M.load("ag_wfq")
    om = np.linspace(2.0, 5.0, 40)
    s1, st1, a1, sig1, it1, cyc1, rr1 = solve(xyz, p, om, 0b111, px.PX_FP64, 1e-11)
    s0, st0, a0, sig0, it0, cyc0, rr0 = solve(xyz, p, om, 0b111, px.PX_FP64, 1e-11, shifted=0)
    say(f"[shifted vs blocked] status {st1} / {st0}, relres max {rr1.max():.2e} / {rr0.max():.2e}, "
        f"cycles max {cyc1.max()} / {cyc0.max()}")
    assert st1 == px.PX_OK and st0 == px.PX_OK
    e = rel_err(sig1, sig0)
    ea = rel_err(a1, a0)
    tm1, tm0 = s1.timings(), s0.timings()
    say(f"[shifted vs blocked] N=1500, 120 columns: steps {it1.max()} vs iterations {it0.max()}, "
        f"sigma {e:.1e} alpha {ea:.1e}, T-apply launches {tm1['n_tapply_f64']:.0f} "
        f"(cols {tm1['cols_f64']:.0f}) vs {tm0['n_tapply_f64']:.0f} (cols {tm0['cols_f64']:.0f})")
    assert e <= 1e-10 and ea <= 1e-9
    assert tm1["cols_f64"] < tm0["cols_f64"]
    s1.close()
    s0.close()


def test_step_cap_reports_not_converged():
    c = C.small_sphere()
    s = px.Structure(0, c["xyz"], c["params"], px.default_stream())
    s.set_frequencies([3.5], 0b001)
    st = s.solve(precision=px.PX_FP64, rel_tol=1e-12, shifted=1, shifted_max_steps=3, max_cycles=1)
    assert st == px.PX_E_NOTCONV
    it, cyc, rr = s.stats()
    assert it[0] == 3 and cyc[0] == 1 and rr[0] > 1e-12
    assert np.isfinite(s.spectrum()[1]).all()
    s.close()
