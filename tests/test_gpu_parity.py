"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Tolerances (stated here, derived in the design notes):
  * operator apply, FP64 path: max|dy| <= 1e-11 max|y| (FP64 rounding over
    N-term sums, conditioned by the Kbar cancellation);
  * operator apply, FP32 T-apply: max|dy| <= 2e-4 max|y| (FP32 T entries and
    accumulation, amplified by the row-sum-zero Kbar that differences
    neighbouring values of T x);
  * spectra, FP64 path solved to rel_tol 1e-12: rel_err_sigma <= 1e-10;
  * spectra, mixed path at rel_tol 1e-8: rel_err_sigma <= 1e-5,
  where rel_err_sigma = max_w |sigma_gpu - sigma_ref| / max_w |sigma_ref|.
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


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def make(case_model, xyz, params):
    return px.Structure(case_model, xyz, params, px.default_stream())


# ------------------------------------------------------------ operator apply

@pytest.mark.parametrize("model,n", [(0, 249), (0, 1000), (1, 300)])
def test_operator_apply_matches_oracle(model, n):
    say(f"[apply] model={model} n={n}")
    params = M.load("ag_wfq" if model == 0 else "au_wfqfmu")
    xyz = G.fcc_sphere_n(n, seed=10 + n)
    pv = M.param_vector(params)
    s = make(model, xyz, params)
    rng = np.random.default_rng(n)
    nu = 4 * n if model else n
    ncol = 6
    x = rng.standard_normal((ncol, nu)) + 1j * rng.standard_normal((ncol, nu))
    om = np.linspace(1.5, 4.5, ncol)
    aib = M.interband_alpha(M.load("au_wfqfmu"), om) if model else None
    ref = O.apply(model, xyz, pv, om, x, aib)
    y64 = s.apply(px.PX_FP64, om, x, aib)
    y32 = s.apply(px.PX_MIXED, om, x, aib)
    e64, e32 = rel_err(y64, ref), rel_err(y32, ref)
    say(f"   fp64 err {e64:.2e}  fp32-T err {e32:.2e}")
    assert e64 <= 1e-11
    assert e32 <= 2e-4
    # narrow FP64 path (<= 4 complex columns) against the same reference
    y1 = s.apply(px.PX_FP64, om[:1], x[:1], None if aib is None else aib[:1])
    assert rel_err(y1, ref[:1]) <= 1e-11
    s.close()


# ------------------------------------------------------------ full solves

def _solve(model, xyz, params, om, pol, aib, precision, rel_tol, max_block_cols=0, **kw):
    s = make(model, xyz, params)
    s.set_frequencies(om, pol, 1e-4, aib)
    st = s.solve(precision=precision, rel_tol=rel_tol, max_block_cols=max_block_cols, **kw)
    alpha, sigma = s.spectrum()
    it, cyc, rr = s.stats()
    return s, st, alpha, sigma, it, rr


@pytest.mark.parametrize("shifted", [0, 1])
@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_small_sphere_spectrum_matches_oracle(precision, tol, bound, shifted):
    """Blocked solver (shifted = 0) and the shared-Krylov phase (shifted = 1)."""
    c = C.small_sphere()
    say(f"[solve small sphere] precision={precision} tol={tol} shifted={shifted}")
    ref = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    s, st, alpha, sigma, it, rr = _solve(0, c["xyz"], c["params"], c["omega_ev"], c["pol_mask"], None, precision,
                                         tol, shifted=shifted)
    say(f"   status {st} iters max {it.max()} mean {it.mean():.1f} relres max {rr.max():.2e}")
    assert st == px.PX_OK
    assert np.all(rr <= tol)
    e = rel_err(sigma, ref["sigma"])
    ea = rel_err(alpha[:, :, 0], ref["alpha"][:, :, 0])
    say(f"   rel_err sigma {e:.2e} alpha {ea:.2e}")
    assert e <= bound
    assert ea <= bound * 10
    # charges in the caller's atom order
    q = s.charges(17, 0)
    assert rel_err(q, ref["q"][17, 0]) <= bound * 100
    s.close()


@pytest.mark.parametrize("shifted", [0, 1])
@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_mid_size_sphere_three_polarizations(precision, tol, bound, shifted):
    """~1000 atoms (several row tiles and a ragged tail), x/y/z columns."""
    xyz = G.fcc_sphere_n(1000, seed=21)
    p = M.load("ag_wfq")
    om = np.array([2.3, 3.4, 4.6])
    say(f"[solve mid sphere] precision={precision} shifted={shifted}")
    ref = O.solve_spectrum(0, xyz, M.param_vector(p), om, 0b111, 1e-4)
    s, st, alpha, sigma, it, rr = _solve(0, xyz, p, om, 0b111, None, precision, tol, shifted=shifted)
    say(f"   status {st} iters max {it.max()} relres max {rr.max():.2e}")
    assert st == px.PX_OK
    e = rel_err(sigma, ref["sigma"])
    say(f"   rel_err sigma {e:.2e}")
    assert e <= bound
    for a in alpha:
        assert np.abs(a - a.T).max() <= 1e3 * bound * np.abs(a).max()
    s.close()


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_dipole_model_rod_matches_oracle(precision, tol, bound):
    xyz = G.fcc_rod_n(300, seed=31)
    p = M.load("au_wfqfmu")
    om = np.linspace(1.6, 3.4, 7)
    aib = M.interband_alpha(p, om)
    say(f"[solve dipole rod] precision={precision}")
    ref = O.solve_spectrum(1, xyz, M.param_vector(p), om, 0b101, 1e-4, aib)
    s, st, alpha, sigma, it, rr = _solve(1, xyz, p, om, 0b101, aib, precision, tol)
    say(f"   status {st} iters max {it.max()} relres max {rr.max():.2e}")
    assert st == px.PX_OK
    e = rel_err(sigma, ref["sigma"])
    say(f"   rel_err sigma {e:.2e}")
    assert e <= bound
    q, mu = s.charges(3, 2, with_dipoles=True)
    n = len(xyz)
    assert rel_err(np.concatenate([q, mu.ravel()]), ref["q"][3, 1]) <= bound * 100
    s.close()


def test_one_column_solver_matches_blocked_solver():
    c = C.small_sphere()
    om = c["omega_ev"][::5]
    say("[one-column vs blocked]")
    _, st1, _, s1, it1, _ = _solve(0, c["xyz"], c["params"], om, 0b001, None, px.PX_FP64, 1e-12, max_block_cols=1,
                                   shifted=0)
    _, st2, _, s2, it2, _ = _solve(0, c["xyz"], c["params"], om, 0b001, None, px.PX_FP64, 1e-12, shifted=0)
    assert st1 == px.PX_OK and st2 == px.PX_OK
    assert rel_err(s1, s2) <= 1e-9


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_orthogonalisation_variants_agree(precision, tol, bound):
    """Both Arnoldi orthogonalisations (two passes in the same step, or the
    second delayed into the next step) reach the oracle's spectrum.  With
    restart_m = 12 the cases take several cycles (full-length cycles that end
    with the final correction, and columns finishing at different steps), on
    both models."""
    xyz = G.fcc_rod_n(300, seed=31)
    p = M.load("au_wfqfmu")
    om = np.linspace(1.6, 3.4, 7)
    aib = M.interband_alpha(p, om)
    ref = O.solve_spectrum(1, xyz, M.param_vector(p), om, 0b101, 1e-4, aib)
    c = C.small_sphere()
    ref_s = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    for ortho in (px.PX_ORTHO_CGS2, px.PX_ORTHO_DCGS2):
        say(f"[ortho {ortho}] precision={precision}")
        s, st, alpha, sigma, it, rr = _solve(1, xyz, p, om, 0b101, aib, precision, tol, ortho=ortho, restart_m=12,
                                             max_restart_m=12, stall_cycles=0)
        e = rel_err(sigma, ref["sigma"])
        say(f"   rod: status {st} iters max {it.max()} relres max {rr.max():.2e} rel_err {e:.2e}")
        assert st == px.PX_OK and e <= bound
        s.close()
        s, st, alpha, sigma, it, rr = _solve(0, c["xyz"], c["params"], c["omega_ev"], c["pol_mask"], None, precision,
                                             tol, ortho=ortho, restart_m=12, max_restart_m=12, stall_cycles=0,
                                             shifted=0)
        e = rel_err(sigma, ref_s["sigma"])
        say(f"   sphere: status {st} iters max {it.max()} relres max {rr.max():.2e} rel_err {e:.2e}")
        assert st == px.PX_OK and e <= bound
        s.close()


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)])
def test_stored_t_apply_matches_oracle(precision, tol, bound):
    """The stored-T apply (dense T built once per structure, the hand-written
    FP32/FP64 MFMA products and the narrow FP64 pass over T) reaches the
    oracle's spectrum on both models, forced and under the autotuner, in the
    blocked solver and in the shared-Krylov phase."""
    xyz = G.fcc_rod_n(300, seed=31)
    p = M.load("au_wfqfmu")
    om = np.linspace(1.6, 3.4, 7)
    aib = M.interband_alpha(p, om)
    ref = O.solve_spectrum(1, xyz, M.param_vector(p), om, 0b101, 1e-4, aib)
    c = C.small_sphere()
    ref_s = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    for mode in (px.PX_TAPPLY_STORED, px.PX_TAPPLY_AUTO, px.PX_TAPPLY_ON_THE_FLY):
        s, st, alpha, sig_r, it, rr = _solve(1, xyz, p, om, 0b101, aib, precision, tol, t_apply=mode)
        ts = s.tapply_stats()
        e = rel_err(sig_r, ref["sigma"])
        say(f"[t_apply {mode}] rod: status {st} iters max {it.max()} rel_err {e:.2e} launches {ts}")
        assert st == px.PX_OK and e <= bound
        if mode == px.PX_TAPPLY_STORED:
            assert ts["f64_stored"] > 0 and ts["f64_on_the_fly"] == 0
            if precision == px.PX_MIXED:
                assert ts["f32_stored"] > 0 and ts["f32_on_the_fly"] == 0
        if mode == px.PX_TAPPLY_ON_THE_FLY:
            assert ts["f32_stored"] == 0 and ts["f64_stored"] == 0
        s.close()
        s, st, alpha, sig_s, it, rr = _solve(0, c["xyz"], c["params"], c["omega_ev"], c["pol_mask"], None, precision,
                                             tol, t_apply=mode, shifted=0)
        e = rel_err(sig_s, ref_s["sigma"])
        say(f"[t_apply {mode}] sphere: status {st} iters max {it.max()} rel_err {e:.2e} launches {s.tapply_stats()}")
        assert st == px.PX_OK and e <= bound
        s.close()
        # the shared-Krylov phase: its narrow FP64 T-apply (one real column)
        # on the stored T too, then the true residuals
        s, st, alpha, sig_s, it, rr = _solve(0, c["xyz"], c["params"], c["omega_ev"], c["pol_mask"], None, precision,
                                             tol, t_apply=mode)
        ts = s.tapply_stats()
        e = rel_err(sig_s, ref_s["sigma"])
        say(f"[t_apply {mode}] sphere, shared phase: status {st} rel_err {e:.2e} launches {ts}")
        assert st == px.PX_OK and e <= bound
        if mode == px.PX_TAPPLY_STORED:
            assert ts["f64_stored"] > 10 and ts["f64_on_the_fly"] == 0
        s.close()


@pytest.mark.parametrize("precision,tol,bound", [(px.PX_MIXED, 1e-8, 1e-5), (px.PX_FP64, 1e-12, 1e-10)])
def test_stored_t_half_tile_block(precision, tol, bound):
    """96 columns: the blocked solver pads them to 128, so the stored FP32
    product runs one full 128-column block and, for the next block, whose 64
    active real columns fill half a tile, a 64-column tile; as columns retire
    the block shrinks to 64 (one half tile).  In FP64 the stored product runs
    on the 192 active real columns alone.  Against the oracle, and against the
    on-the-fly apply."""
    xyz = G.fcc_rod_n(100, seed=33)
    p = M.load("au_wfqfmu")
    om = np.linspace(1.6, 3.4, 48)
    aib = M.interband_alpha(p, om)
    ref = O.solve_spectrum(1, xyz, M.param_vector(p), om, 0b011, 1e-4, aib)
    out = {}
    for mode in (px.PX_TAPPLY_STORED, px.PX_TAPPLY_ON_THE_FLY):
        s, st, alpha, sig, it, rr = _solve(1, xyz, p, om, 0b011, aib, precision, tol, t_apply=mode)
        ts = s.tapply_stats()
        e = rel_err(sig, ref["sigma"])
        say(f"[half tile] precision {precision} t_apply {mode}: status {st} iters max {it.max()} rel_err {e:.2e} "
            f"launches {ts}")
        assert st == px.PX_OK and rr.max() <= tol and e <= bound
        if mode == px.PX_TAPPLY_STORED:
            key = "f32" if precision == px.PX_MIXED else "f64"
            assert ts[key + "_stored"] > 0 and ts[key + "_on_the_fly"] == 0
        out[mode] = sig
        s.close()
    e = rel_err(out[px.PX_TAPPLY_STORED], out[px.PX_TAPPLY_ON_THE_FLY])
    say(f"[half tile] stored vs on the fly: {e:.2e}")
    assert e <= (1e-6 if precision == px.PX_MIXED else 1e-10)


def test_gap_dimer_conserves_charge_per_fragment():
    xyz = G.gap_dimer(600, gap=5.0, seed=41)
    p = M.load("ag_wfq")
    say("[gap dimer]")
    s, st, alpha, sigma, it, rr = _solve(0, xyz, p, np.array([2.5, 3.5]), 0b001, None, px.PX_MIXED, 1e-8)
    assert st == px.PX_OK
    q = s.charges(1, 0)
    assert abs(q[:300].sum()) <= 1e-7 * np.abs(q).max()
    assert abs(q[300:].sum()) <= 1e-7 * np.abs(q).max()
    s.close()


# ------------------------------------------------------------ edge cases

def test_single_atom_and_pair():
    p = M.load("ag_wfq")
    s = make(0, np.zeros((1, 3)), p)
    s.set_frequencies([3.0], 0b111, 1e-4)
    assert s.solve() == px.PX_OK
    alpha, sigma = s.spectrum()
    assert np.all(alpha == 0) and sigma[0] == 0.0
    s.close()
    l_ang = p["fermi_s"] * p["r0_ang"]
    xyz = G.two_atoms(l_ang)
    om = np.array([0.7, 3.0, 9.0])
    ref = O.solve_spectrum(0, xyz, M.param_vector(p), om, 0b011, 1e-4)
    s, st, alpha, sigma, it, rr = _solve(0, xyz, p, om, 0b011, None, px.PX_FP64, 1e-12)
    assert st == px.PX_OK
    assert rel_err(alpha[:, 0, 0], ref["alpha"][:, 0, 0]) <= 1e-12
    assert np.abs(alpha[:, 1, 1]).max() <= 1e-12 * np.abs(alpha[:, 0, 0]).max()
    s.close()


def test_state_and_argument_errors():
    p = M.load("ag_wfq")
    xyz = G.fcc_sphere_radius(6.0)
    s = make(0, xyz, p)
    with pytest.raises(px.PxError) as e:
        s.spectrum()
    assert e.value.status == px.PX_E_STATE
    with pytest.raises(px.PxError) as e:
        s.solve()
    assert e.value.status == px.PX_E_STATE
    for bad in ([0.0], [-1.0], [np.nan]):
        with pytest.raises(px.PxError) as e:
            s.set_frequencies(bad, 0b001)
        assert e.value.status == px.PX_E_INVALID
    with pytest.raises(px.PxError) as e:
        s.set_frequencies([2.0], 0)
    assert e.value.status == px.PX_E_INVALID
    s.set_frequencies([2.0, 3.0], 0b001)
    with pytest.raises(px.PxError) as e:
        s.charges(0, 1)
    s.close()
    dup = np.concatenate([xyz, xyz[:1]])
    with pytest.raises(px.PxError) as e:
        make(0, dup, p)
    assert e.value.status == px.PX_E_INVALID


def test_not_converged_is_reported():
    c = C.small_sphere()
    s = make(0, c["xyz"], c["params"])
    s.set_frequencies([3.5], 0b001)
    st = s.solve(precision=px.PX_FP64, rel_tol=1e-13, restart_m=5, max_cycles=1, shifted=0)
    assert st == px.PX_E_NOTCONV
    it, cyc, rr = s.stats()
    assert cyc[0] == 1 and rr[0] > 1e-13
    alpha, sigma = s.spectrum()
    assert np.isfinite(sigma).all()
    s.close()
