"""Pins of the reference oracle against what the paper and mathematics fix.

Nothing here re-types the oracle's formulas and compares them with
themselves.  Each pin uses an independent route: quadrature of the Gaussian
densities the paper defines (Section 2.1), finite differences (the paper
derives T^qmu and T^mumu by differentiation, Section 2.2), textbook limits
(point charges and point dipoles), closed forms derived by hand for tiny
systems, a library linear solver and eigensolver, and physical invariants
(charge conservation, reciprocity, passivity, the f-sum rule, isotropy).
"""
import json
import os

import numpy as np
import pytest
import scipy.constants as sc
import scipy.integrate as si
import scipy.special as sp

import oracle as O
from workloads import configs as C
from workloads import geometry as G
from workloads import materials as M

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")

# unit conversions as the oracle carries them (pinned to CODATA below)
BOHR = O.constants()["ang_per_bohr"]
HARTREE_EV = O.constants()["ev_per_hartree"]
AG = M.load("ag_wfq")
AU = M.load("au_wfqfmu")


def pv(p, **kw):
    return M.param_vector(M.with_overrides(p, **kw))


def gauss_coulomb(d, s2):
    """Coulomb energy of two unit Gaussian charges rho = exp(-r^2/R^2)/(pi^1.5 R^3)
    with R1^2 + R2^2 = s2 at distance d (bohr), by 1-D quadrature in Fourier
    space: (2/pi) int_0^inf exp(-k^2 s2 / 4) sin(k d)/(k d) dk."""
    if d == 0.0:
        f = lambda k: np.exp(-k * k * s2 / 4.0)
    else:
        f = lambda k: np.exp(-k * k * s2 / 4.0) * np.sinc(k * d / np.pi)
    kmax = 40.0 / np.sqrt(s2)
    val, _ = si.quad(f, 0.0, kmax, limit=400, epsabs=1e-15, epsrel=1e-13)
    return 2.0 / np.pi * val


# ---------------------------------------------------------------- constants

def test_unit_constants_are_codata():
    """The oracle carries CODATA 2018; the library of record may carry a later
    adjustment, which moves these by < 1e-9 relative."""
    c = O.constants()
    assert c["ang_per_bohr"] == pytest.approx(sc.physical_constants["Bohr radius"][0] * 1e10, rel=1e-8)
    assert c["ev_per_hartree"] == pytest.approx(sc.physical_constants["Hartree energy in eV"][0], rel=1e-8)
    assert c["c_au"] == pytest.approx(1.0 / sc.fine_structure, rel=1e-8)


# ---------------------------------------------------------------- kernels

@pytest.mark.parametrize("d_bohr", [0.0, 0.3, 1.0, 2.5, 4.0, 7.5, 15.0])
def test_tqq_equals_gaussian_charge_coulomb_energy(d_bohr):
    """T^qq (Eq. tqq) including its diagonal is the Coulomb energy between the
    Gaussian densities of Section 2.1."""
    rq = AG["r_q_bohr"]
    if d_bohr == 0.0:
        xyz = np.zeros((1, 3))
        t = O.tqq(xyz, pv(AG))[0, 0]
    else:
        xyz = G.two_atoms(d_bohr * BOHR)
        t = O.tqq(xyz, pv(AG))[0, 1]
    ref = gauss_coulomb(d_bohr, 2 * rq * rq)
    assert t == pytest.approx(ref, rel=1e-10)


def test_tqq_tends_to_point_charges():
    xyz = G.two_atoms(60.0)
    t = O.tqq(xyz, pv(AG))[0, 1]
    assert t == pytest.approx(1.0 / (60.0 / BOHR), rel=1e-14)


def _charge_kernel(ri, rj, s2):
    d = np.linalg.norm(np.asarray(ri) - np.asarray(rj))
    return sp.erf(d / np.sqrt(s2)) / d


@pytest.mark.parametrize("d_ang", [1.2, 2.9, 4.1, 6.5])
def test_dipole_kernels_are_derivatives_of_charge_kernel(d_ang):
    """T^qmu, T^muq, T^mumu (Eq. wfqfmu-system) as finite differences of the
    charge kernel (pinned above) with respect to the dipole positions."""
    p = AU
    rq, rm = p["r_q_bohr"], p["r_mu_bohr"]
    direction = np.array([0.3, -0.5, 0.81])
    direction /= np.linalg.norm(direction)
    xyz = np.array([[0.0, 0.0, 0.0], d_ang * direction])
    n = 2
    t = O.tfull(xyz, pv(p))
    rb = xyz / BOHR
    h = 1e-4
    e = np.eye(3)
    i, j = 0, 1
    for a in range(3):
        # potential at i from a unit dipole at j along a  = d/d r_j,a of the kernel
        fd = (_charge_kernel(rb[i], rb[j] + h * e[a], rq * rq + rm * rm)
              - _charge_kernel(rb[i], rb[j] - h * e[a], rq * rq + rm * rm)) / (2 * h)
        assert t[0 * n + i, (1 + a) * n + j] == pytest.approx(fd, rel=1e-7, abs=1e-12)
        # minus field at i from a unit charge at j = d/d r_i,a of the kernel
        fd2 = (_charge_kernel(rb[i] + h * e[a], rb[j], rm * rm + rq * rq)
               - _charge_kernel(rb[i] - h * e[a], rb[j], rm * rm + rq * rq)) / (2 * h)
        assert t[(1 + a) * n + i, 0 * n + j] == pytest.approx(fd2, rel=1e-7, abs=1e-12)
        for b in range(3):
            s2 = 2 * rm * rm
            fpp = _charge_kernel(rb[i] + h * e[a], rb[j] + h * e[b], s2)
            fpm = _charge_kernel(rb[i] + h * e[a], rb[j] - h * e[b], s2)
            fmp = _charge_kernel(rb[i] - h * e[a], rb[j] + h * e[b], s2)
            fmm = _charge_kernel(rb[i] - h * e[a], rb[j] - h * e[b], s2)
            fd3 = (fpp - fpm - fmp + fmm) / (4 * h * h)
            assert t[(1 + a) * n + i, (1 + b) * n + j] == pytest.approx(fd3, rel=2e-6, abs=1e-9)
    # the self blocks (hardness reading): only T^qq_ii is non-zero
    assert t[0, 0] == pytest.approx(np.sqrt(2 / np.pi) / rq, rel=1e-14)
    for a in range(3):
        assert t[0, (1 + a) * n] == 0.0 and t[(1 + a) * n, 0] == 0.0
        for b in range(3):
            assert t[(1 + a) * n, (1 + b) * n] == 0.0


def test_dipole_kernel_point_limit_is_textbook_dipole_tensor():
    """With vanishing widths, T^mumu is minus the point-dipole field tensor
    (3 r r^T - r^2 I)/r^5 and T^qmu the point-dipole potential r^T/r^3."""
    p = M.with_overrides(AU, r_mu_bohr=1e-7, r_q_bohr=1e-7)
    xyz = np.array([[0.0, 0.0, 0.0], [3.1, -1.7, 2.2]])
    t = O.tfull(xyz, M.param_vector(p))
    r = (xyz[0] - xyz[1]) / BOHR
    d = np.linalg.norm(r)
    tensor = (d * d * np.eye(3) - 3 * np.outer(r, r)) / d ** 5
    n = 2
    assert np.allclose(t[n:, n:].reshape(3, 2, 3, 2)[:, 0, :, 1], tensor, rtol=1e-12, atol=0)
    assert np.allclose(t[0, n:].reshape(3, 2)[:, 1], r / d ** 3, rtol=1e-12)


def test_tfull_is_symmetric_and_tqq_is_positive_definite():
    xyz = G.fcc_sphere_radius(6.0, seed=7)
    t = O.tfull(xyz, pv(AU))
    assert np.abs(t - t.T).max() <= 1e-15 * np.abs(t).max()
    tq = O.tqq(xyz, pv(AG))
    np.linalg.cholesky(tq)                       # Gram matrix of Gaussians: SPD
    assert np.linalg.eigvalsh(tq).min() > 0


def test_fermi_damping_half_point_and_cutoff():
    """Eq. (fermi) gives f = 1/2 at r = s r0, so K = A / (2 s r0) there;
    pairs beyond the exchange cutoff do not exchange charge."""
    s, r0 = AG["fermi_s"], AG["r0_ang"]
    assert s * r0 < AG["cutoff_ang"]
    k = O.kbar(G.two_atoms(s * r0), pv(AG))
    assert k[0, 1] == pytest.approx(AG["a_eff_bohr2"] / (2 * s * r0 / BOHR), rel=1e-14)
    assert k[0, 0] == pytest.approx(-k[0, 1], rel=1e-15)
    k2 = O.kbar(G.two_atoms(AG["cutoff_ang"] * 1.0001), pv(AG))
    assert np.all(k2 == 0.0)
    # deep inside the tunnelling region (r << s r0) the damping vanishes
    k3 = O.kbar(G.two_atoms(0.2 * r0), pv(AG))
    assert k3[0, 1] == pytest.approx(AG["a_eff_bohr2"] / (0.2 * r0 / BOHR), rel=1e-4)


def test_kbar_laplacian_structure():
    xyz = C.small_sphere()["xyz"]
    k = O.kbar(xyz, pv(AG))
    assert np.abs(k.sum(axis=1)).max() < 1e-14 * np.abs(k).max()
    assert np.array_equal(k, k.T)
    assert np.linalg.eigvalsh(k).max() < 1e-12
    # every fcc site inside the sphere has at most 12 neighbours within 1.2 r0
    off = (k != 0) & ~np.eye(len(k), dtype=bool)
    assert off.sum(axis=1).max() == 12


# ---------------------------------------------------------------- solver

def test_own_lu_matches_library_solver():
    rng = np.random.default_rng(11)
    for n in (1, 5, 60, 200):
        a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        b = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
        x = O.lu_solve(a, b)
        ref = np.linalg.solve(a, b)
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()
    # a matrix that needs pivoting (zero leading entry)
    a = np.array([[0, 1, 2], [3, 0, 1], [1, 1, 0]], dtype=complex)
    b = np.array([1, 2, 3], dtype=complex)
    assert np.allclose(O.lu_solve(a, b), np.linalg.solve(a, b), rtol=1e-14)


def test_two_atom_closed_form():
    """Two atoms at distance l = s r0 along x:  alpha_xx = k l^2 / (2 k (eta - t) + z)
    with k = A/(2 s r0), eta = sqrt(2/pi)/R_q, t = erf(l/(sqrt2 R_q))/l,
    and alpha_yy = alpha_zz = 0 (derived by hand from Eq. wfq-system)."""
    p = AG
    l_ang = p["fermi_s"] * p["r0_ang"]
    l = l_ang / BOHR
    k = p["a_eff_bohr2"] / (2 * l)
    rq = p["r_q_bohr"]
    eta = np.sqrt(2 / np.pi) / rq
    t = sp.erf(l / (np.sqrt(2) * rq)) / l
    dw = p["density_au"] / p["eff_mass_au"]
    om_ev = np.array([0.5, 2.0, 3.3, 7.0])
    out = O.solve_spectrum(0, G.two_atoms(l_ang), pv(p), om_ev, 0b111, 1e-4)
    for w_i, wev in enumerate(om_ev):
        w = wev / HARTREE_EV
        z = -(w / (2 * dw * p["tau_au"])) * (w * p["tau_au"] + 1j)
        axx = k * l * l / (2 * k * (eta - t) + z)
        al = out["alpha"][w_i]
        assert al[0, 0] == pytest.approx(axx, rel=1e-12)
        assert abs(al[1, 1]) < 1e-12 * abs(axx) and abs(al[2, 2]) < 1e-12 * abs(axx)
        assert abs(al[0, 1]) < 1e-12 * abs(axx)


def test_two_atom_response_is_a_drude_lorentz_oscillator():
    """The pair's alpha(w) must be f / (w0^2 - w^2 - i w / tau): damping rate
    exactly 1/tau and oscillator strength f = 2 (n/m*) K_12 l^2 (the f-sum
    rule of the Drude model), whatever the kernel values."""
    p = AG
    l_ang = 2.95
    xyz = G.two_atoms(l_ang)
    k12 = O.kbar(xyz, pv(p))[0, 1]
    l = l_ang / BOHR
    om_ev = np.linspace(0.5, 8.0, 9)
    al = O.solve_spectrum(0, xyz, pv(p), om_ev, 0b001, 1e-4)["alpha"][:, 0, 0]
    w = om_ev / HARTREE_EV
    inv = 1.0 / al
    # Re(1/alpha) = (w0^2 - w^2)/f  -> slope in w^2 is -1/f
    slope, icpt = np.polyfit(w * w, inv.real, 1)
    f = -1.0 / slope
    gamma = -(inv.imag * f) / w
    dw = p["density_au"] / p["eff_mass_au"]
    assert f == pytest.approx(2 * dw * k12 * l * l, rel=1e-10)
    assert np.allclose(gamma, 1.0 / p["tau_au"], rtol=1e-10)
    assert icpt * f > 0                                   # w0^2 > 0


def test_spectral_route_matches_direct_solve():
    """alpha_xx(w) = sum_m w_m^2 / (lambda_m + z(w)) with (lambda, U) the
    eigenpairs of L^1/2 T L^1/2 (L = -Kbar) and w = U^T L^1/2 x."""
    xyz = G.fcc_sphere_radius(7.0, seed=3)
    p = pv(AG)
    kb = O.kbar(xyz, p)
    t = O.tqq(xyz, p)
    lw, lu = np.linalg.eigh(-kb)
    lh = (lu * np.sqrt(np.clip(lw, 0, None))) @ lu.T
    lam, u = np.linalg.eigh(lh @ t @ lh)
    x = xyz[:, 0] / BOHR
    wts = u.T @ lh @ x
    om_ev = np.linspace(1.0, 6.0, 23)
    out = O.solve_spectrum(0, xyz, p, om_ev, 0b001, 1e-4)
    dw = AG["density_au"] / AG["eff_mass_au"]
    tau = AG["tau_au"]
    for i, wev in enumerate(om_ev):
        w = wev / HARTREE_EV
        z = -(w / (2 * dw * tau)) * (w * tau + 1j)
        ref = np.sum(wts ** 2 / (lam + z))
        assert out["alpha"][i, 0, 0] == pytest.approx(ref, rel=1e-9)


# ---------------------------------------------------------------- invariants

def test_invariants_on_jittered_sphere():
    c = C.small_sphere()
    p = pv(c["params"])
    om = np.array([2.0, 3.5, 3.55, 5.0])
    out = O.solve_spectrum(0, c["xyz"], p, om, 0b111, 1e-4)
    q = out["q"]
    al = out["alpha"]
    # charge conservation (a single connected fragment)
    assert np.abs(q.sum(axis=2)).max() <= 1e-12 * np.abs(q).max()
    # reciprocity: alpha is complex symmetric
    for a in al:
        assert np.abs(a - a.T).max() <= 1e-9 * np.abs(a).max()
    # passivity
    assert np.all(np.diagonal(al, axis1=1, axis2=2).imag > 0)
    assert np.all(out["sigma"] > 0)
    # linear in E0 and independent of the origin
    out2 = O.solve_spectrum(0, c["xyz"] + np.array([3.0, -7.0, 11.0]), p, om, 0b111, 3e-3)
    assert np.allclose(out2["alpha"], al, rtol=1e-10, atol=1e-10 * np.abs(al).max())
    assert np.allclose(out2["q"] / 30.0, q, rtol=1e-9, atol=1e-12 * np.abs(q).max())


def test_charge_conserved_per_fragment():
    """Two clusters farther apart than the exchange cutoff: each keeps zero net
    charge (the nullspace of Kbar is one constant per connected fragment)."""
    xyz = G.gap_dimer(160, gap=6.0, seed=9)
    n1 = 80
    out = O.solve_spectrum(0, xyz, pv(AG), np.array([3.0]), 0b001, 1e-4)
    q = out["q"][0, 0]
    assert abs(q[:n1].sum()) <= 1e-12 * np.abs(q).max()
    assert abs(q[n1:].sum()) <= 1e-12 * np.abs(q).max()
    assert np.abs(q[:n1]).max() > 1e-3 * np.abs(q).max()


def test_oh_cluster_is_isotropic():
    xyz = G.fcc_sphere_radius(9.0, jitter=0.0)
    out = O.solve_spectrum(0, xyz, pv(AG), np.array([2.5, 3.6, 4.4]), 0b111, 1e-4)
    for a in out["alpha"]:
        iso = np.trace(a) / 3
        assert np.abs(a - iso * np.eye(3)).max() <= 1e-10 * abs(iso)


def test_high_frequency_limit_is_the_f_sum_rule():
    """w^2 alpha_xx(w) -> -2 (n/m*) sum_{i<j} K_ij (x_i - x_j)^2 (free-electron
    limit: independent of T)."""
    xyz = G.fcc_sphere_radius(8.0, seed=5)
    p = pv(AG)
    kb = O.kbar(xyz, p)
    x = xyz[:, 0] / BOHR
    bond = 0.0
    n = len(x)
    for i in range(n):
        for j in range(i + 1, n):
            bond += kb[i, j] * (x[i] - x[j]) ** 2
    dw = AG["density_au"] / AG["eff_mass_au"]
    wev = 2.0e5
    al = O.solve_spectrum(0, xyz, p, np.array([wev]), 0b001, 1e-4)["alpha"][0, 0, 0]
    w = wev / HARTREE_EV
    assert (w * w * al).real == pytest.approx(-2 * dw * bond, rel=1e-6)


# ---------------------------------------------------------------- dipole model

def test_single_atom_dipole_model_is_alpha_ib():
    aib = np.array([17.0 + 2.0j, 9.0 + 0.5j])
    out = O.solve_spectrum(1, np.zeros((1, 3)), pv(AU), np.array([2.0, 3.0]), 0b111, 1e-4, aib)
    for w in range(2):
        assert np.allclose(out["alpha"][w], aib[w] * np.eye(3), rtol=1e-13, atol=1e-13)
        assert np.abs(out["q"][w][:, 0]).max() == 0.0


def test_point_dipole_pair_is_applequist():
    """Two atoms beyond the exchange cutoff with (nearly) point dipoles: no
    charge flows and the pair polarizability is the classical coupled-dipole
    result 2a/(1 - 2a/r^3) along the axis and 2a/(1 + a/r^3) across it."""
    p = M.with_overrides(AU, r_mu_bohr=1e-6)
    d_ang = 5.0
    r = d_ang / BOHR
    a = 11.0 + 1.5j
    out = O.solve_spectrum(1, G.two_atoms(d_ang), M.param_vector(p), np.array([2.4]), 0b111, 1e-4, np.array([a]))
    al = out["alpha"][0]
    assert al[0, 0] == pytest.approx(2 * a / (1 - 2 * a / r ** 3), rel=1e-10)
    assert al[1, 1] == pytest.approx(2 * a / (1 + a / r ** 3), rel=1e-10)
    assert al[2, 2] == pytest.approx(2 * a / (1 + a / r ** 3), rel=1e-10)
    assert np.abs(out["q"][0][:, :2]).max() == 0.0


def test_dipole_model_without_interband_term_reduces_to_charges():
    xyz = G.fcc_sphere_radius(7.0, seed=4)
    om = np.array([2.0, 3.2, 4.5])
    aib = np.full(3, 1e-13 + 0j)
    a1 = O.solve_spectrum(1, xyz, pv(AU), om, 0b001, 1e-4, aib)["alpha"][:, 0, 0]
    a0 = O.solve_spectrum(0, xyz, pv(AU), om, 0b001, 1e-4)["alpha"][:, 0, 0]
    assert np.allclose(a1, a0, rtol=1e-8)


def test_dipole_model_reciprocity_passivity_conservation():
    xyz = G.fcc_sphere_radius(6.5, seed=8)
    om = np.array([1.8, 2.6, 3.4])
    aib = M.interband_alpha(AU, om)
    out = O.solve_spectrum(1, xyz, pv(AU), om, 0b111, 1e-4, aib)
    n = len(xyz)
    for a in out["alpha"]:
        assert np.abs(a - a.T).max() <= 1e-9 * np.abs(a).max()
        assert np.all(np.diag(a).imag > 0)
    assert np.abs(out["q"][:, :, :n].sum(axis=2)).max() <= 1e-12 * np.abs(out["q"]).max()


# ---------------------------------------------------------------- paper trend

def _prf(xyz, p, lo, hi):
    grid = np.linspace(lo, hi, 25)
    s = O.solve_spectrum(0, xyz, p, grid, 0b001, 1e-4)["sigma"]
    i = int(np.argmax(s))
    fine = np.linspace(grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)], 25)
    s2 = O.solve_spectrum(0, xyz, p, fine, 0b001, 1e-4)["sigma"]
    return fine[int(np.argmax(s2))]


def test_graphene_disk_plasmon_trend_matches_paper_ratio():
    """Doubling a graphene disk's atom count at fixed E_F red-shifts its plasmon
    by the ratio the paper prints for its 10k -> 20k-atom disks (0.26/0.30
    eV), within the spread expected between small and large disks."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_graphene_prf.json")) as f:
        gold = json.load(f)
    ratio_paper = gold["prf_ev"]["20000"] / gold["prf_ev"]["10000"]
    p = pv(M.load("graphene_wfq"))
    w1 = _prf(G.graphene_disk_n(300), p, 0.2, 1.2)
    w2 = _prf(G.graphene_disk_n(600), p, 0.2, 1.2)
    assert w2 / w1 == pytest.approx(ratio_paper, rel=0.06)


def test_stored_small_sphere_spectrum_is_reproduced():
    """Regression fixture written by tests/golden/make_golden.py (oracle only)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "small_sphere_sigma.json")) as f:
        gold = json.load(f)
    c = C.small_sphere()
    out = O.solve_spectrum(0, c["xyz"], pv(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    assert np.allclose(out["sigma"], gold["sigma_bohr2"], rtol=1e-12, atol=0)


def test_sigma_is_textbook_absorption_cross_section():
    """Quasi-static absorption cross section of a polarizable particle
    (Gaussian units): C_abs = 4 pi k Im alpha, k = w / c, averaged over the
    solved polarizations; the speed of light from the library of record."""
    c_au = 1.0 / sc.fine_structure
    c = C.small_sphere()
    out = O.solve_spectrum(0, c["xyz"], pv(c["params"]), c["omega_ev"], 0b001, 1e-4)
    k = c["omega_ev"] / HARTREE_EV / c_au
    assert np.allclose(out["sigma"], 4 * np.pi * k * out["alpha"][:, 0, 0].imag, rtol=1e-8)
    out3 = O.solve_spectrum(0, c["xyz"], pv(c["params"]), c["omega_ev"][:5], 0b111, 1e-4)
    tr = np.trace(out3["alpha"], axis1=1, axis2=2).imag
    assert np.allclose(out3["sigma"], 4 * np.pi * k[:5] * tr / 3, rtol=1e-8)


# ---------------------------------------------------------------- two atom types (Eqs. wfqfmu-leghe, polar-finale)

AG_MU = M.load("ag_wfqfmu")


def test_two_type_system_reduces_to_the_homogeneous_model():
    """Eq. (wfqfmu-leghe) reduces to Eq. (wfqfmu-system) for one atom type: all
    atoms A, all atoms B, and random types with identical parameter sets all
    give the homogeneous spectrum (charges and dipoles)."""
    xyz = G.fcc_sphere_n(43, seed=3)
    om = np.array([2.2, 3.1, 3.9])
    pa, pb = pv(AG_MU), pv(AU)
    aa, ab = M.interband_alpha(AG_MU, om), M.interband_alpha(AU, om)
    rand = G.alloy_types(len(xyz), 0.4, seed=2)
    cases = [(np.zeros(len(xyz)), pa, aa), (np.ones(len(xyz)), pb, ab)]
    for types, p, aib in cases:
        ref = O.solve_spectrum(1, xyz, p, om, 0b011, 1e-4, aib)
        het = O.solve_spectrum_het(1, xyz, types, pa, pb, om, 0b011, 1e-4, aa, ab)
        assert np.abs(het["alpha"] - ref["alpha"]).max() <= 1e-11 * np.abs(ref["alpha"]).max()
    ref = O.solve_spectrum(1, xyz, pa, om, 0b011, 1e-4, aa)
    het = O.solve_spectrum_het(1, xyz, rand, pa, pa, om, 0b011, 1e-4, aa, aa)
    assert np.abs(het["q"] - ref["q"]).max() <= 1e-11 * np.abs(ref["q"]).max()


def test_unlike_pair_closed_form():
    """Charges only, an A-B pair at distance l along x: the exchange current
    through the mean Drude factor sigma = (sigma_A + sigma_B)/2,
    sigma_t = 2 n_t tau_t / (1 - i w tau_t), gives (derived by hand)
    alpha_xx = sigma K l^2 / (sigma K eta - i w),  eta = T_11 + T_22 - 2 T_12."""
    l_ang = 2.95
    xyz = G.two_atoms(l_ang)
    pa, pb = pv(AG_MU), pv(AU)
    k = O.kbar(xyz, pa)[0, 1]             # the two types share A, r0, d, s here
    t = O.tqq(xyz, pa)
    eta = t[0, 0] + t[1, 1] - 2 * t[0, 1]
    l = l_ang / BOHR
    om = np.array([0.7, 2.5, 3.4, 6.0])
    out = O.solve_spectrum_het(0, xyz, [0, 1], pa, pb, om, 0b001, 1e-4)
    for i, wev in enumerate(om):
        w = wev / HARTREE_EV
        sig = [2 * (p["density_au"] / p["eff_mass_au"]) * p["tau_au"] / (1 - 1j * w * p["tau_au"]) for p in (AG_MU, AU)]
        s = 0.5 * (sig[0] + sig[1])
        axx = s * k * l * l / (s * k * eta - 1j * w)
        assert out["alpha"][i, 0, 0] == pytest.approx(axx, rel=1e-11)


def test_two_type_reciprocity_passivity_conservation():
    """A random Ag-Au alloy (dipole model): alpha symmetric (the exchange matrix
    diag(sigma) (Kbar + Hbar) / 2 is symmetric), Im alpha_ll > 0, and the
    charges of every column sum to zero."""
    xyz = G.fcc_sphere_n(55, seed=4)
    types = G.alloy_types(len(xyz), 0.5, seed=5)
    om = np.array([2.0, 3.0, 3.6, 4.4])
    out = O.solve_spectrum_het(1, xyz, types, pv(AG_MU), pv(AU), om, 0b111, 1e-4,
                               M.interband_alpha(AG_MU, om), M.interband_alpha(AU, om))
    n = len(xyz)
    for a in out["alpha"]:
        assert np.abs(a - a.T).max() <= 1e-10 * np.abs(a).max()
        assert np.all(np.diagonal(a).imag > 0)
    q = out["q"][:, :, :n]
    assert np.abs(q.sum(axis=2)).max() <= 1e-10 * np.abs(q).sum(axis=2).max()


def test_isolated_atom_of_type_b_has_its_own_interband_polarizability():
    """Eq. (polar-finale) with no neighbours gives alpha_i = alpha_IB of the
    atom's own type: a lone B atom's alpha is alpha_IB,B I."""
    om = np.array([2.0, 3.5])
    ab = M.interband_alpha(AU, om)
    out = O.solve_spectrum_het(1, np.zeros((1, 3)), [1], pv(AG_MU), pv(AU), om, 0b111, 1e-4,
                               M.interband_alpha(AG_MU, om), ab)
    for i in range(2):
        assert np.allclose(out["alpha"][i], ab[i] * np.eye(3), rtol=1e-12, atol=0)


def test_two_type_apply_and_rhs_satisfy_the_direct_solution():
    """The matrix-free apply and the right-hand side agree with the dense
    direct solve: A(w) q = b for the solved charges and dipoles."""
    xyz = G.fcc_sphere_n(38, seed=8)
    types = G.alloy_types(len(xyz), 0.3, seed=9)
    pa, pb = pv(AG_MU), pv(AU)
    om = np.array([2.6, 3.3])
    aa, ab = M.interband_alpha(AG_MU, om), M.interband_alpha(AU, om)
    out = O.solve_spectrum_het(1, xyz, types, pa, pb, om, 0b100, 1e-4, aa, ab)
    for i in range(len(om)):
        q = out["q"][i, 0]
        y = O.apply_het(1, xyz, types, pa, pb, om[i:i + 1], q[None, :], aa[i:i + 1], ab[i:i + 1])[0]
        b = O.rhs_het(1, xyz, types, pa, pb, om[i], 2, 1e-4)
        assert np.abs(y - b).max() <= 1e-10 * np.abs(b).max()


# --------------------------- matrix-free operator, right-hand side, sampled rows
# These three are the checkers of the GPU operator-apply and full-size tests.
# Each is pinned to the dense, separately pinned pieces: K-bar (Laplacian
# structure, Fermi damping), T (quadrature, finite differences) and z_q (the
# two-atom Drude-Lorentz closed form), composed here as Eqs. (wfq-system) and
# (wfqfmu-system) state them, and to the oracle's own dense LU solution.

def _dense_operator(model, xyz, p, om_ev, aib):
    """A(w) of Eq. (wfq-system) / (wfqfmu-system) from the pinned dense pieces:
    charge rows Kbar (T x)_q - z_q x_q, dipole rows (T x)_mu - z_mu x_mu."""
    n = len(xyz)
    kb = O.kbar(xyz, p)
    z = O.zq(p, om_ev / HARTREE_EV)
    if model == 0:
        return kb @ O.tqq(xyz, p) - z * np.eye(n)
    t = O.tfull(xyz, p)
    a = t.astype(np.complex128)
    a[:n] = kb @ t[:n]
    zmu = -1.0 / aib
    return a - np.diag(np.r_[np.full(n, z), np.full(3 * n, zmu)])


@pytest.mark.parametrize("model", [0, 1])
def test_matrix_free_apply_is_the_dense_operator(model):
    """or_apply(x) = A(w) x column by column, each column at its own frequency,
    with A built from the pinned K-bar, T and z_q (and z_mu = -1/alpha_IB)."""
    p = AG if model == 0 else AU
    xyz = G.fcc_sphere_n(60, seed=31) if model == 0 else G.fcc_rod_n(48, seed=32)
    n = len(xyz)
    nu = n if model == 0 else 4 * n
    om = np.array([1.7, 2.9, 4.1])
    aib = M.interband_alpha(p, om) if model == 1 else None
    rng = np.random.default_rng(33)
    x = rng.standard_normal((3, nu)) + 1j * rng.standard_normal((3, nu))
    y = O.apply(model, xyz, pv(p), om, x, aib)
    for c in range(3):
        a = _dense_operator(model, xyz, pv(p), om[c], None if aib is None else aib[c])
        ref = a @ x[c]
        assert np.abs(y[c] - ref).max() <= 1e-12 * np.abs(ref).max()
        # and the oracle's own dense assembly agrees
        a2 = O.assemble(model, xyz, pv(p), om[c], None if aib is None else aib[c:c + 1])
        assert np.abs(a2 @ x[c] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("model", [0, 1])
def test_rhs_is_minus_kbar_v_and_the_direct_solution_satisfies_it(model):
    """or_rhs(l) = -Kbar V with V_i = -E0 r_{i,l} (and E0 on the dipole rows of
    component l), built from the pinned K-bar; and A(w) q = b holds for the
    charges (and dipoles) of the oracle's dense LU solve."""
    p = AG if model == 0 else AU
    xyz = G.fcc_sphere_n(60, seed=34) if model == 0 else G.fcc_rod_n(48, seed=35)
    n = len(xyz)
    nu = n if model == 0 else 4 * n
    e0 = 1e-4
    rb = np.asarray(xyz) / BOHR
    kb = O.kbar(xyz, pv(p))
    om = np.array([2.2, 3.6])
    aib = M.interband_alpha(p, om) if model == 1 else None
    out = O.solve_spectrum(model, xyz, pv(p), om, 0b111, e0, aib)
    for l in range(3):
        b = O.rhs(model, xyz, pv(p), l, e0)
        ref = np.zeros(nu, dtype=np.complex128)
        ref[:n] = -kb @ (-e0 * rb[:, l])
        if model == 1:
            ref[(1 + l) * n:(2 + l) * n] = e0
        assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max()
        for i in range(len(om)):
            a = _dense_operator(model, xyz, pv(p), om[i], None if aib is None else aib[i])
            assert np.abs(a @ out["q"][i, l] - b).max() <= 1e-10 * np.abs(b).max()


@pytest.mark.parametrize("model", [0, 1])
def test_tapply_rows_are_rows_of_the_dense_t(model):
    """or_tapply_rows gives the requested rows of T X (T^qq, or the 4N x 4N
    dipole-model T in [q | mu_x | mu_y | mu_z] order), including the first and
    last unknown and a row of every component block."""
    p = AG if model == 0 else AU
    xyz = G.fcc_sphere_n(60, seed=36) if model == 0 else G.fcc_rod_n(48, seed=37)
    n = len(xyz)
    nu = n if model == 0 else 4 * n
    t = O.tqq(xyz, pv(p)) if model == 0 else O.tfull(xyz, pv(p))
    rows = np.array(sorted({0, nu - 1, 5, n - 1} | ({n, n + 7, 2 * n + 3, 3 * n + 11} if model == 1 else set())))
    x = np.random.default_rng(38).standard_normal((4, nu))
    y = O.tapply_rows(model, xyz, pv(p), rows, x)
    ref = (t @ x.T)[rows].T
    assert y.shape == ref.shape
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_alloy_plasmon_red_shifts_and_weakens_with_gold_fraction():
    """The paper's nanoalloy trend (its Ag-Au alloy example): the plasmon peak
    of an Ag-Au sphere moves to lower energy and loses intensity as the Au
    fraction grows (peak searched in the plasmon window 1.5-3.5 eV, below the
    interband absorption)."""
    xyz = G.fcc_sphere_n(135, seed=10)
    om = np.linspace(1.5, 3.5, 81)
    peaks, heights = [], []
    for frac in (0.0, 0.5, 1.0):
        types = G.alloy_types(len(xyz), frac, seed=11)
        out = O.solve_spectrum_het(1, xyz, types, pv(AG_MU), pv(AU), om, 0b001, 1e-4,
                                   M.interband_alpha(AG_MU, om), M.interband_alpha(AU, om))
        i = int(np.argmax(out["sigma"]))
        assert 0 < i < len(om) - 1          # an interior maximum
        peaks.append(om[i])
        heights.append(out["sigma"][i])
    assert peaks[0] > peaks[1] > peaks[2]
    assert heights[0] > heights[1] > heights[2]


# ------------------------------------------------ probe fields (post-processing)

def _probe_case(model, n=6, seed=3):
    """A few atoms with seeded complex charges (and dipoles)."""
    rng = np.random.default_rng(seed)
    xyz = G.fcc_sphere_n(n)
    q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    mu = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n)) if model == 1 else None
    return xyz, pv(AU if model else AG), q, mu


@pytest.mark.parametrize("model", [0, 1])
def test_probe_field_is_minus_gradient_of_potential(model):
    """E = -grad phi by central differences, at points in the Taylor-series
    region of an atom (x < 1/2), at moderate and at large distance."""
    xyz, p, q, mu = _probe_case(model)
    pts = np.array([xyz[0] + [0.3, -0.2, 0.25], xyz[1] + [0.05, 0.02, -0.04], xyz[2] + [1.7, 0.9, -1.1],
                    [6.0, -4.0, 3.0], [30.0, 12.0, -20.0]])
    r = O.probe(model, xyz, p, q, mu, pts)
    h = 1e-4   # Angstrom
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fp = O.probe(model, xyz, p, q, mu, pts + e)["phi"]
        fm = O.probe(model, xyz, p, q, mu, pts - e)["phi"]
        grad = (fp - fm) / (2 * h / BOHR)
        assert np.allclose(-grad, r["field"][:, a], rtol=1e-6, atol=1e-8 * np.abs(r["field"]).max())


@pytest.mark.parametrize("model", [0, 1])
def test_probe_gauss_law(model):
    """div E = 4 pi rho (atomic units), by central differences of the field
    at points inside the atoms' Gaussians."""
    xyz, p, q, mu = _probe_case(model)
    pts = np.array([xyz[0] + [0.4, 0.1, -0.3], xyz[3] + [-0.2, 0.6, 0.1], xyz[5] + [0.05, -0.05, 0.1]])
    h = 2e-3   # Angstrom
    div = np.zeros(len(pts), dtype=complex)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        div += (O.probe(model, xyz, p, q, mu, pts + e)["field"][:, a] -
                O.probe(model, xyz, p, q, mu, pts - e)["field"][:, a]) / (2 * h / BOHR)
    rho = O.probe(model, xyz, p, q, mu, pts)["rho"]
    assert np.allclose(div, 4 * np.pi * rho, rtol=1e-5, atol=1e-7 * np.abs(rho).max())


@pytest.mark.parametrize("model", [0, 1])
def test_probe_density_moments(model):
    """The density integrates to the total charge and its first moment to
    sum q_i r_i + sum mu_i (midpoint rule on a fine grid, spectrally accurate
    for Gaussians)."""
    xyz, p, q, mu = _probe_case(model, n=3)
    lo, hi = xyz.min(0) - 6.0, xyz.max(0) + 6.0
    hstep = 0.12
    axes = [np.arange(lo[a], hi[a], hstep) + hstep / 2 for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    rho = O.probe(model, xyz, p, q, mu, pts)["rho"]
    dv = (hstep / BOHR) ** 3
    assert abs(rho.sum() * dv - q.sum()) <= 1e-8 * np.abs(q).sum()
    dip = (rho[:, None] * (pts / BOHR)).sum(0) * dv
    ref = (q[None, :] * (xyz.T / BOHR)).sum(1)
    if model == 1:
        ref = ref + mu.sum(1)
    assert np.allclose(dip, ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


@pytest.mark.parametrize("model", [0, 1])
def test_probe_far_field_is_point_multipoles(model):
    """Far from the atoms the Gaussians act as point charges and point
    dipoles: phi = q / r + mu . d / r^3 and E = q d / r^3 + (3 (mu . d) d / r^2 - mu) / r^3."""
    xyz, p, q, mu = _probe_case(model)
    pts = np.array([[80.0, 10.0, -30.0], [-50.0, 60.0, 45.0]])
    r = O.probe(model, xyz, p, q, mu, pts)
    for t, pt in enumerate(pts / BOHR):
        d = pt[None, :] - xyz / BOHR
        rr = np.linalg.norm(d, axis=1)
        phi = (q / rr).sum()
        e = (q[:, None] * d / rr[:, None] ** 3).sum(0)
        if model == 1:
            md = (mu.T * d).sum(1)
            phi += (md / rr ** 3).sum()
            e += ((3 * md[:, None] * d / rr[:, None] ** 2 - mu.T) / rr[:, None] ** 3).sum(0)
        assert abs(r["phi"][t] - phi) <= 1e-13 * np.abs(q).sum()
        assert np.allclose(r["field"][t], e, rtol=1e-12, atol=1e-15)
        assert abs(r["rho"][t]) < 1e-300


def test_probe_at_an_atom_centre_and_series_boundary():
    """At a charge's own centre: zero field, potential 2 q / (sqrt(pi) R_q),
    density q / (pi^1.5 R_q^3); the series (x < 1/2) and the closed form agree
    across x = 1/2 for a charge and a dipole."""
    p = pv(AU)
    rq, rmu = M.load("au_wfqfmu")["r_q_bohr"], M.load("au_wfqfmu")["r_mu_bohr"]
    xyz = np.zeros((1, 3))
    r = O.probe(0, xyz, p, np.array([1.0 + 0.5j]), None, xyz)
    assert abs(r["field"]).max() == 0.0
    assert abs(r["phi"][0] - (1 + 0.5j) * 2 / (np.sqrt(np.pi) * rq)) < 1e-15
    assert abs(r["rho"][0] - (1 + 0.5j) / (np.pi ** 1.5 * rq ** 3)) < 1e-15
    for R, model, mu in ((rq, 0, None), (rmu, 1, np.array([[0.3], [-0.7], [0.4]], dtype=complex))):
        d = np.array([0.6, -0.3, 0.2])
        d = d / np.linalg.norm(d)
        x = 0.5 * R * BOHR
        lo = O.probe(model, xyz, p, np.array([0.8]), mu, (x * (1 - 1e-9)) * d[None, :])["field"]
        hi = O.probe(model, xyz, p, np.array([0.8]), mu, (x * (1 + 1e-9)) * d[None, :])["field"]
        assert np.allclose(lo, hi, rtol=1e-8)


# ---------------------------------------------------------------- BEM (DPCM)
# Section 2.3, Eq. (bem-dpcm), "approximate" F, read for the tessera charges
# (oracle/px_oracle.c, or_bem_*).  Pinned to the textbook quasistatic sphere
# (Clausius-Mossotti polarizability, the Frohlich resonance, the eigenvalues
# 2 pi / (2l + 1) of the adjoint double-layer operator on a sphere), the
# depolarization-factor closed form of a spheroid, charge neutrality and the
# icosahedral isotropy of the mesh.
from workloads import mesh as ME  # noqa: E402

ANG3 = BOHR ** 3


def _bem_alpha(m, eps2, pol=0b100):
    om = np.linspace(2.0, 3.0, len(np.atleast_1d(eps2)))
    out = O.bem_solve_spectrum(m, om, np.atleast_1d(eps2), 1.0, pol, 1e-4)
    assert out["status"] == 0
    return out


@pytest.mark.parametrize("eps2", [-1.5 + 0.3j, 5.0 + 0.0j])
def test_bem_sphere_converges_to_clausius_mossotti(eps2):
    """A meshed sphere's dipolar polarizability tends to R^3 (e2 - e1) / (e2 + 2 e1)
    as the mesh is refined (80, 320, 1280 tesserae), at second order."""
    R = 40.0
    exact = (R ** 3 / ANG3) * (eps2 - 1.0) / (eps2 + 2.0)
    errs = []
    for k in (1, 2, 3):
        a = _bem_alpha(ME.sphere(R, k), eps2)["alpha"][0, 2, 2]
        errs.append(abs(a - exact) / abs(exact))
    assert errs[0] > 2.5 * errs[1] > 2.5 * 2.5 * errs[2]
    assert errs[2] < 0.02


def test_bem_icosphere_is_isotropic_and_neutral():
    """The icosahedral mesh leaves no preferred axis (alpha = alpha_iso I), and
    the induced charges of a neutral body sum to zero."""
    out = _bem_alpha(ME.sphere(30.0, 2), -2.3 + 0.4j, pol=0b111)
    al = out["alpha"][0]
    iso = np.trace(al) / 3
    assert np.abs(al - iso * np.eye(3)).max() <= 1e-11 * abs(iso)
    for q in out["q"][0]:
        assert abs(q.sum()) <= 1e-12 * np.abs(q).sum()


def test_bem_operator_has_the_sphere_eigenvalues():
    """On a sphere the kernel A_i (s_i - s_j).n_i / r^3 is the adjoint double
    layer: charge patterns of degree l are eigenvectors with eigenvalue
    2 pi / (2l + 1) (l = 0: 2 pi; l = 1: 2 pi / 3; l = 2: 2 pi / 5)."""
    res = {}
    for k in (2, 3):
        m = ME.sphere(25.0, k)
        M_ = O.bem_matrix(m)
        c, a = m["cen"], m["area"]
        u = c / np.linalg.norm(c, axis=1)[:, None]
        for l, (q, lam) in enumerate(((a, 2 * np.pi), (a * u[:, 2], 2 * np.pi / 3),
                                      (a * (3 * u[:, 0] * u[:, 1]), 2 * np.pi / 5))):
            mq = M_ @ q
            res.setdefault(l, []).append(np.linalg.norm(mq - lam * q) / np.linalg.norm(lam * q))
            if k == 3:
                assert abs((q @ mq) / (q @ q) / lam - 1.0) <= 5e-3      # Rayleigh quotient
    for l in res:
        assert res[l][1] < res[l][0] and res[l][1] < 0.03


def test_bem_spheroid_approaches_depolarization_closed_form():
    """A prolate spheroid (semi-axes 15, 15, 45 Angstrom) against the textbook
    alpha_ll = (a a c / 3) (e2 - e1) / (e1 + L_l (e2 - e1)), L from the
    eccentricity: the error falls as the mesh is refined."""
    a_, c_ = 15.0, 45.0
    e = np.sqrt(1 - (a_ / c_) ** 2)
    Lz = (1 - e * e) / (e * e) * (np.log((1 + e) / (1 - e)) / (2 * e) - 1)
    Lx = (1 - Lz) / 2
    eps2 = -1.2 + 0.5j
    errs = {0: [], 2: []}
    for k in (2, 3):
        out = _bem_alpha(ME.spheroid(a_, c_, k), eps2, pol=0b101)
        for l, L in ((0, Lx), (2, Lz)):
            exact = (a_ * a_ * c_ / 3.0 / ANG3) * (eps2 - 1.0) / (1.0 + L * (eps2 - 1.0))
            errs[l].append(abs(out["alpha"][0, l, l] - exact) / abs(exact))
        for q in out["q"][0]:
            assert abs(q.sum()) <= 1e-3 * np.abs(q).sum()
    for l in (0, 2):
        assert errs[l][1] < errs[l][0] and errs[l][1] < 0.06


def test_bem_drude_sphere_resonates_at_the_frohlich_frequency():
    """A Drude sphere absorbs most where e2 = -2 e1, i.e. at w_p / sqrt(eps_inf + 2)."""
    p = M.load("ag_bem")
    b = p["bem"]
    wf = b["omega_p_ev"] / np.sqrt(b["eps_inf"] + 2.0)
    om = np.linspace(wf - 0.15, wf + 0.15, 61)
    out = O.bem_solve_spectrum(ME.sphere(20.0, 2), om, M.drude_permittivity(p, om), 1.0, 0b001, 1e-4)
    peak = om[int(np.argmax(out["sigma"]))]
    assert abs(peak - wf) <= 0.01 * wf


def test_bem_apply_rhs_and_direct_solution_agree():
    """The matrix-free apply is (M - z I) x with z = 2 pi (e2 + e1) / (e2 - e1);
    the right-hand side is -A E0 n_l; the dense LU solution satisfies the system."""
    m = ME.spheroid(12.0, 30.0, 2)
    n = len(m["area"])
    om = np.array([2.5, 3.1])
    eps2 = np.array([-3.0 + 0.7j, 2.0 + 0.1j])
    M_ = O.bem_matrix(m)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    y = O.bem_apply(m, eps2, 1.0, x)
    for c in range(2):
        z = 2 * np.pi * (eps2[c] + 1.0) / (eps2[c] - 1.0)
        ref = M_ @ x[c] - z * x[c]
        assert np.abs(y[c] - ref).max() <= 1e-12 * np.abs(ref).max()
    out = O.bem_solve_spectrum(m, om, eps2, 1.0, 0b011, 1e-4)
    for l in (0, 1):
        b = O.bem_rhs(m, l, 1e-4)
        assert np.abs(b + 1e-4 * m["area"] / BOHR ** 2 * m["nrm"][:, l]).max() <= 1e-15
        for w in range(2):
            r = O.bem_apply(m, eps2[w:w + 1], 1.0, out["q"][w, l][None, :])[0] - b
            assert np.abs(r).max() <= 1e-11 * np.abs(b).max()


# ---------------------------------------------------------------- BEM (IEFPCM)
# Section 2.3, Eq. (bem-iefpcm) with the paper's S and F (oracle/px_oracle.c,
# or_bem_ief_*; F's diagonal read as the double layer's self patch).  Pinned to
# the identities of the continuous operators (Gauss's solid angle: the double
# layer maps 1 to -2 pi on any closed surface; on a sphere S and the double
# layer have the eigenvalues 4 pi R / (2l + 1) and -2 pi / (2l + 1)), the
# Clausius-Mossotti sphere (also in a medium), the spheroid closed form, the
# Frohlich resonance, neutrality and isotropy.

def _ief(m, eps2, eps1=1.0, pol=0b100):
    om = np.linspace(2.0, 3.0, len(np.atleast_1d(eps2)))
    out = O.bem_ief_solve_spectrum(m, om, np.atleast_1d(eps2), eps1, pol, 1e-4)
    assert out["status"] == 0
    return out


@pytest.mark.parametrize("eps2,eps1", [(-1.5 + 0.3j, 1.0), (5.0 + 0.0j, 1.0), (-3.0 + 0.2j, 1.77)])
def test_bem_ief_sphere_converges_to_clausius_mossotti(eps2, eps1):
    """R^3 (e2 - e1) / (e2 + 2 e1) at second order under refinement (80, 320,
    1280 tesserae).  The printed positive diagonal of F misses this by O(1)
    near resonance (e2 = -1.5: 172 %, 139 %, 61 %)."""
    R = 40.0
    exact = (R ** 3 / ANG3) * (eps2 - eps1) / (eps2 + 2.0 * eps1)
    errs = []
    for k in (1, 2, 3):
        a = _ief(ME.sphere(R, k), eps2, eps1)["alpha"][0, 2, 2]
        errs.append(abs(a - exact) / abs(exact))
    assert errs[0] > 2.5 * errs[1] > 2.5 * 2.5 * errs[2]
    assert errs[2] < 0.02


def test_bem_ief_sphere_operator_identities():
    """Row sums of F tend to -2 pi (Gauss) and of S to 4 pi R (the potential of
    a unit density on a sphere); degree-l densities are eigenvectors of S and
    F with 4 pi R / (2l + 1) and -2 pi / (2l + 1).  All errors fall with
    refinement (320 -> 1280 tesserae)."""
    errs = []
    for k in (2, 3):
        m = ME.sphere(25.0, k)
        S, F = O.bem_ief_matrices(m)
        R = 25.0 / BOHR
        u = m["cen"] / np.linalg.norm(m["cen"], axis=1)[:, None]
        e = [np.abs(F.sum(1) + 2 * np.pi).max() / (2 * np.pi), np.abs(S.sum(1) / (4 * np.pi * R) - 1).max()]
        for l, y in ((1, u[:, 2]), (2, 3 * u[:, 0] * u[:, 1])):
            ls, lf = 4 * np.pi * R / (2 * l + 1), -2 * np.pi / (2 * l + 1)
            e.append(np.linalg.norm(S @ y - ls * y) / np.linalg.norm(ls * y))
            e.append(np.linalg.norm(F @ y - lf * y) / np.linalg.norm(lf * y))
        errs.append(np.array(e))
    assert np.all(errs[1] < errs[0])
    assert errs[1].max() < 0.015


def test_bem_ief_double_layer_normal_is_the_source_normal():
    """Gauss's identity holds for any closed surface, not only a sphere: on a
    prolate spheroid the row sums of F stay near -2 pi (rms 0.12 at 1280
    tesserae); F built with the row's normal instead misses it by 0.8."""
    m = ME.spheroid(15.0, 45.0, 3)
    S, F = O.bem_ief_matrices(m)
    rs = F.sum(1) + 2 * np.pi
    assert np.sqrt(np.mean(rs ** 2)) < 0.2
    assert np.all(np.diag(F) < 0)


def test_bem_ief_spheroid_approaches_depolarization_closed_form():
    """The spheroid of the DPCM pin (semi-axes 15, 15, 45 Angstrom): the error
    against the depolarization-factor closed form falls with refinement."""
    a_, c_ = 15.0, 45.0
    e = np.sqrt(1 - (a_ / c_) ** 2)
    Lz = (1 - e * e) / (e * e) * (np.log((1 + e) / (1 - e)) / (2 * e) - 1)
    Lx = (1 - Lz) / 2
    eps2 = -1.2 + 0.5j
    errs = {0: [], 2: []}
    for k in (2, 3):
        out = _ief(ME.spheroid(a_, c_, k), eps2, pol=0b101)
        for l, L in ((0, Lx), (2, Lz)):
            exact = (a_ * a_ * c_ / 3.0 / ANG3) * (eps2 - 1.0) / (1.0 + L * (eps2 - 1.0))
            errs[l].append(abs(out["alpha"][0, l, l] - exact) / abs(exact))
        for q in out["q"][0]:
            assert abs(q.sum()) <= 1e-10 * np.abs(q).sum()
    assert errs[0][1] < 0.6 * errs[0][0] and errs[0][1] < 0.05
    assert errs[2][1] < 0.75 * errs[2][0] and errs[2][1] < 0.2


def test_bem_ief_isotropic_neutral_and_resonant():
    """An icosphere leaves no preferred axis, the induced charges sum to zero,
    and a Drude sphere absorbs most at w_p / sqrt(eps_inf + 2)."""
    out = _ief(ME.sphere(30.0, 2), -2.3 + 0.4j, pol=0b111)
    al = out["alpha"][0]
    iso = np.trace(al) / 3
    assert np.abs(al - iso * np.eye(3)).max() <= 1e-11 * abs(iso)
    for q in out["q"][0]:
        assert abs(q.sum()) <= 1e-12 * np.abs(q).sum()
    p = M.load("ag_bem")
    b = p["bem"]
    wf = b["omega_p_ev"] / np.sqrt(b["eps_inf"] + 2.0)
    om = np.linspace(wf - 0.15, wf + 0.15, 61)
    out = O.bem_ief_solve_spectrum(ME.sphere(20.0, 2), om, M.drude_permittivity(p, om), 1.0, 0b001, 1e-4)
    assert abs(om[int(np.argmax(out["sigma"]))] - wf) <= 0.01 * wf


def test_bem_ief_apply_rhs_and_direct_solution_agree():
    """The apply is [2 pi f I + F] x, the right-hand side -(2 pi I + F) V with
    V = -E0 s_l, and the direct solution satisfies Eq. (bem-iefpcm)."""
    m = ME.spheroid(12.0, 30.0, 2)
    n = len(m["area"])
    S, F = O.bem_ief_matrices(m)
    a = m["area"] / BOHR ** 2
    s = m["cen"] / BOHR
    om = np.array([2.5, 3.1])
    eps2 = np.array([-3.0 + 0.7j, 2.0 + 0.1j])
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    y = O.bem_ief_apply(m, eps2, 1.3, x)
    for c in range(2):
        f = (eps2[c] + 1.3) / (eps2[c] - 1.3)
        ref = F @ x[c] + 2 * np.pi * f * x[c]
        assert np.abs(y[c] - ref).max() <= 1e-12 * np.abs(ref).max()
    out = O.bem_ief_solve_spectrum(m, om, eps2, 1.3, 0b011, 1e-4)
    c = (a[:, None] * s).sum(axis=0) / a.sum()
    for l in (0, 1):
        b = O.bem_ief_rhs(m, l, 1e-4)
        v = -1e-4 * (s[:, l] - c[l])
        assert np.abs(b + (2 * np.pi * v + F @ v)).max() <= 1e-12 * np.abs(b).max()
        for w in range(2):
            f = (eps2[w] + 1.3) / (eps2[w] - 1.3)
            lhs = (2 * np.pi * f * np.eye(n) + F) @ (S @ (out["q"][w, l] / a))
            assert np.abs(lhs - b).max() <= 1e-10 * np.abs(b).max()


def test_bem_ief_potential_is_the_single_layer_over_the_areas():
    """The matrix-free potential S A^-1 q of the oracle's IEFPCM charges: on a
    sphere a degree-1 charge pattern q = A u_z makes 4 pi R / 3 u_z (the
    single layer's eigenvalue), and the direct solution's potential solves
    the shifted double-layer system [2 pi f I + F] y = b."""
    m = ME.sphere(25.0, 3)
    R = 25.0 / BOHR
    a = m["area"] / BOHR ** 2
    u = m["cen"] / np.linalg.norm(m["cen"], axis=1)[:, None]
    y = O.bem_ief_potential(m, (a * u[:, 2]).astype(np.complex128))[0]
    lam = 4 * np.pi * R / 3
    assert np.linalg.norm(y - lam * u[:, 2]) / np.linalg.norm(lam * u[:, 2]) < 2e-3
    m = ME.sphere(20.0, 2)
    eps2 = np.array([-2.0 + 0.5j])
    out = O.bem_ief_solve_spectrum(m, np.array([3.0]), eps2, 1.0, 0b001, 1e-4)
    y = O.bem_ief_potential(m, out["q"][0, 0])[0]
    r = O.bem_ief_apply(m, eps2, 1.0, y[None, :])[0] - O.bem_ief_rhs(m, 0, 1e-4)
    assert np.abs(r).max() <= 1e-10 * np.abs(O.bem_ief_rhs(m, 0, 1e-4)).max()


def test_bem_ief_does_not_depend_on_where_the_mesh_sits():
    """A constant in V drops out of the continuous equation but not of the
    discrete one; with V and the dipole taken relative to the tesserae's
    area-weighted centroid, two unequal spheres (neutral only up to the
    discretization) give the same polarizability and charges wherever they
    sit (moved by 1000 Angstrom; an uncentred V changes alpha by ~80 %)."""
    s1, s2 = ME.sphere(20.0, 2), ME.sphere(30.0, 2)
    m = dict(cen=np.vstack([s1["cen"], s2["cen"] + np.array([60.0, 0.0, 0.0])]),
             nrm=np.vstack([s1["nrm"], s2["nrm"]]), area=np.concatenate([s1["area"], s2["area"]]), r_enc=60.0)
    eps2 = np.array([-3.0 + 0.3j])
    ref = O.bem_ief_solve_spectrum(m, np.array([3.0]), eps2, 1.0, 0b101, 1e-4)
    moved = O.bem_ief_solve_spectrum(dict(m, cen=m["cen"] + np.array([1000.0, -300.0, 50.0])), np.array([3.0]), eps2,
                                     1.0, 0b101, 1e-4)
    assert np.abs(moved["alpha"] - ref["alpha"]).max() <= 1e-9 * np.abs(ref["alpha"]).max()
    assert np.abs(moved["q"] - ref["q"]).max() <= 1e-9 * np.abs(ref["q"]).max()
    q = ref["q"][0, 0]
    assert 1e-6 < abs(q.sum()) / np.abs(q).sum() < 1e-2       # not neutral by symmetry here


def test_bem_dpcm_dipole_does_not_depend_on_where_the_mesh_sits():
    """DPCM's charges of two unequal spheres are neutral only to ~1e-4 of
    sum |q|; with the dipole taken from the tesserae's area-weighted centroid
    the polarizability is the same wherever the pair sits (an origin at the
    caller's zero changes it by 0.4 % at 1000 Angstrom)."""
    s1, s2 = ME.sphere(20.0, 2), ME.sphere(30.0, 2)
    m = dict(cen=np.vstack([s1["cen"], s2["cen"] + np.array([60.0, 0.0, 0.0])]),
             nrm=np.vstack([s1["nrm"], s2["nrm"]]), area=np.concatenate([s1["area"], s2["area"]]), r_enc=60.0)
    eps2 = np.array([-3.0 + 0.3j])
    ref = O.bem_solve_spectrum(m, np.array([3.0]), eps2, 1.0, 0b001, 1e-4)
    moved = O.bem_solve_spectrum(dict(m, cen=m["cen"] + np.array([1000.0, -300.0, 50.0])), np.array([3.0]), eps2,
                                 1.0, 0b001, 1e-4)
    assert np.abs(moved["alpha"] - ref["alpha"]).max() <= 1e-9 * np.abs(ref["alpha"]).max()
    q = ref["q"][0, 0]
    assert abs(q.sum()) / np.abs(q).sum() > 1e-6
