"""GPU parity of the BEM path in the IEFPCM form against the oracle (Section
2.3, Eq. bem-iefpcm, "approximate" F; oracle/px_oracle.c or_bem_ief_*).

The GPU solves [F - z I] y = b for the potentials y = S A^-1 q (z = -2 pi f)
and takes the dipole from y with the weights w = (S A^-1)^-1 s; the oracle
factors the printed product [2 pi f I + F] S A^-1 for the charges q.  Bounds:
operator apply max|dy| <= 1e-11 max|y| (FP64 sums over N terms); spectra at
rel_tol 1e-12 in FP64: sigma <= 1e-10, alpha <= 1e-9, charges <= 1e-8 (the
charges go through one more solve, S A^-1 q = y, to 1e-12); rel_tol 1e-8 in
PX_MIXED (the BEM apply is FP64 in both): sigma <= 1e-5.  Full size (the
20,480-tesserae sphere): the oracle residual of sampled columns' charges in
the printed equation <= rel_tol + 1e-9, and the polarizability within 1 % of
Clausius-Mossotti away from the resonance.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2510_12731_amd as px
from workloads import materials as M
from workloads import mesh as ME

pytestmark = pytest.mark.gpu

BOHR = 0.529177210903


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


@pytest.fixture(scope="module", autouse=True)
def lib():
    import torch
    assert torch.cuda.is_available()
    return px.load()


AG = M.load("ag_bem")
AU = M.load("au_bem")


def cases():
    om_s = np.linspace(3.0, 4.5, 24)
    om_r = np.linspace(1.5, 3.5, 6)
    om_d = np.linspace(3.2, 4.2, 8)
    return [
        dict(name="sphere 320", mesh=ME.sphere(30.0, 2), om=om_s, eps=M.drude_permittivity(AG, om_s), pol=0b111),
        dict(name="spheroid 1280", mesh=ME.spheroid(15.0, 45.0, 3), om=om_r, eps=M.drude_permittivity(AU, om_r),
             pol=0b100),
        dict(name="dimer 640", mesh=ME.sphere_dimer(20.0, 5.0, 2), om=om_d, eps=M.drude_permittivity(AG, om_d),
             pol=0b001),
    ]


def make(c, eps_env=1.0):
    s = px.Structure.bem(c["mesh"], eps_env, px.default_stream(), form="iefpcm")
    s.set_frequencies(c["om"], c["pol"], 1e-4, c["eps"])
    return s


@pytest.mark.parametrize("k,ncol,eps1", [(2, 1, 1.0), (2, 3, 1.0), (3, 2, 1.77), (3, 6, 1.0)])
def test_bem_ief_apply_matches_oracle(k, ncol, eps1):
    """y = [F + 2 pi f(eps2) I] x against the oracle's matrix-free apply,
    narrow blocks and a block wider than one launch (6 columns: 12 real)."""
    m = ME.spheroid(14.0, 28.0, k)
    n = len(m["area"])
    rng = np.random.default_rng(10 * k + ncol)
    x = rng.standard_normal((ncol, n)) + 1j * rng.standard_normal((ncol, n))
    om = np.linspace(2.0, 4.0, ncol)
    eps = M.drude_permittivity(AU, om)
    say(f"[bem ief apply] n={n} ncol={ncol} eps1={eps1}")
    s = px.Structure.bem(m, eps1, px.default_stream(), form="iefpcm")
    y = s.apply(px.PX_FP64, om, x, eps)
    ref = O.bem_ief_apply(m, eps, eps1, x)
    e = rel_err(y, ref)
    say(f"   {e:.1e}")
    assert e <= 1e-11
    s.close()


@pytest.mark.parametrize("shifted", [2, 1, 0])
def test_bem_ief_spectra_match_oracle(shifted):
    """Sphere (3 polarizations), spheroid (one) and gap dimer, FP64 and mixed,
    against the oracle's dense LU of the printed product; the shared phase
    (shifted 2: one block process, 1: one per polarization) and the blocked
    solver (0)."""
    for c in cases():
        ref = O.bem_ief_solve_spectrum(c["mesh"], c["om"], c["eps"], 1.0, c["pol"], 1e-4)
        for prec, tol, bound in ((px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)):
            say(f"[bem ief {c['name']}] shifted={shifted} prec={prec}")
            s = make(c)
            st = s.solve(precision=prec, rel_tol=tol, shifted=shifted)
            alpha, sigma = s.spectrum()
            it, cyc, rr = s.stats()
            e_s, e_a = rel_err(sigma, ref["sigma"]), rel_err(alpha, ref["alpha"])
            say(f"   status {st} steps max {it.max()} relres {rr.max():.1e} sigma {e_s:.1e} alpha {e_a:.1e}")
            assert st == px.PX_OK and rr.max() <= tol and e_s <= bound
            if prec == px.PX_FP64:
                assert e_a <= 1e-9
                pols = [l for l in range(3) if c["pol"] >> l & 1]
                for w in (0, len(c["om"]) - 1):
                    q = s.charges(w, pols[0])
                    e_q = rel_err(q, ref["q"][w, 0])
                    say(f"   charges w={w}: {e_q:.1e}")
                    assert e_q <= 1e-8
                    assert abs(q.sum()) <= 1e-8 * np.abs(q).sum()
            s.close()


def test_bem_ief_charges_give_the_spectrum_dipole():
    """The dipole from the charges (pxGetCharges: a single-layer solve per
    column) equals the one the spectrum takes from the potentials through the
    dipole weights, for every column of the sphere."""
    c = cases()[0]
    s = make(c)
    assert s.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    alpha = s.spectrum()[0]
    a = c["mesh"]["area"]
    cen = c["mesh"]["cen"]
    s_b = (cen - (a[:, None] * cen).sum(axis=0) / a.sum()) / BOHR   # relative to the area-weighted centroid
    worst = 0.0
    for w in range(0, len(c["om"]), 5):
        for l in range(3):
            d = s.charges(w, l) @ s_b
            worst = max(worst, float(np.abs(d / 1e-4 - alpha[w, :, l]).max() / np.abs(alpha[w]).max()))
    say(f"[bem ief dipole] charges vs weights {worst:.1e}")
    assert worst <= 1e-10
    s.close()


def test_bem_ief_medium_permittivity():
    """A sphere in a medium (eps1 = 1.77, water-like) against the oracle."""
    c = cases()[0]
    ref = O.bem_ief_solve_spectrum(c["mesh"], c["om"], c["eps"], 1.77, c["pol"], 1e-4)
    s = make(c, eps_env=1.77)
    assert s.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    e = rel_err(s.spectrum()[1], ref["sigma"])
    say(f"[bem ief medium] sigma {e:.1e}")
    assert e <= 1e-10
    s.close()


def test_bem_ief_edge_cases_and_no_alloc_apply():
    """Invalid meshes are refused as for DPCM; eps2 = eps1 and a missing eps2
    are refused; the no-allocation apply equals the allocating one; batch
    solves refuse stacking and solve the structure whole."""
    m = ME.sphere(10.0, 1)
    bad = dict(m, area=np.where(np.arange(len(m["area"])) == 3, 0.0, m["area"]))
    with pytest.raises(px.PxError) as e:
        px.Structure.bem(bad, form="iefpcm")
    assert e.value.status == px.PX_E_INVALID
    s = px.Structure.bem(m, form="iefpcm")
    with pytest.raises(px.PxError) as e:
        s.set_frequencies(np.array([2.0]), 0b001, 1e-4, np.array([1.0 + 0.0j]))
    assert e.value.status == px.PX_E_INVALID
    with pytest.raises(px.PxError):
        s.set_frequencies(np.array([2.0]), 0b001, 1e-4, None)
    s.close()
    import torch
    m = ME.sphere(25.0, 3)
    n = len(m["area"])
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    om = np.array([3.5, 3.8])
    eps = M.drude_permittivity(AG, om)
    s = px.Structure.bem(m, form="iefpcm")
    xd = torch.from_numpy(x.view(np.float64).copy()).to("cuda")
    yd = torch.zeros_like(xd)
    torch.cuda.synchronize()
    px.pxApplyOperatorNoAlloc(s.h, om, xd.data_ptr(), yd.data_ptr(), eps)
    y = yd.cpu().numpy().view(np.complex128).reshape(x.shape)
    assert rel_err(y, s.apply(px.PX_FP64, om, x, eps)) <= 1e-12
    assert rel_err(y, O.bem_ief_apply(m, eps, 1.0, x)) <= 1e-11
    s.close()
    c = cases()[2]
    s = make(c)
    with pytest.raises(px.PxError) as e:
        px.solve_batch([s], shifted=0)
    assert e.value.status == px.PX_E_INVALID
    assert px.solve_batch([s], precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    ref = O.bem_ief_solve_spectrum(c["mesh"], c["om"], c["eps"], 1.0, c["pol"], 1e-4)
    assert rel_err(s.spectrum()[1], ref["sigma"]) <= 1e-10
    s.close()


def test_bem_ief_sphere_full_size():
    """The BEM benchmark workload in the IEFPCM form: 20,480-tesserae Ag
    sphere (R = 80 Angstrom), 64 frequencies x 3 polarizations, rel_tol 1e-8:
    sampled columns' charges in the printed equation under the oracle's own
    matrix-free operators, neutrality, isotropy, passivity, and
    Clausius-Mossotti away from the resonance."""
    m = ME.sphere(80.0, 5)
    om = np.linspace(3.2, 4.4, 64)
    eps = M.drude_permittivity(AG, om)
    say(f"[bem ief full size] n={len(m['area'])}: create")
    s = px.Structure.bem(m, 1.0, px.default_stream(), form="iefpcm")
    s.set_frequencies(om, 0b111, 1e-4, eps)
    st = s.solve(precision=px.PX_MIXED, rel_tol=1e-8)
    it, cyc, rr = s.stats()
    alpha, sigma = s.spectrum()
    say(f"   status {st} steps max {it.max()} relres max {rr.max():.1e}")
    assert st == px.PX_OK and rr.max() <= 1e-8
    iso = np.trace(alpha, axis1=1, axis2=2) / 3
    assert np.abs(alpha - iso[:, None, None] * np.eye(3)).max() <= 1e-6 * np.abs(iso).max()
    assert np.all(sigma > 0)
    cm = (80.0 / BOHR) ** 3 * (eps - 1.0) / (eps + 2.0)
    off = np.abs(cm) < 0.5 * np.abs(cm).max()
    e_cm = float(np.max(np.abs(iso[off] - cm[off]) / np.abs(cm[off])))
    say(f"   Clausius-Mossotti off resonance: {e_cm:.1e}")
    assert e_cm <= 0.01
    w_peak = int(np.argmax(sigma))
    for w, pol in ((w_peak, 0), (5, 2)):
        q = s.charges(w, pol)
        assert abs(q.sum()) <= 1e-8 * np.abs(q).sum()
        b = O.bem_ief_rhs(m, pol, 1e-4)
        y = O.bem_ief_potential(m, q[None, :])
        r = b - O.bem_ief_apply(m, eps[w:w + 1], 1.0, y)[0]
        rel = np.linalg.norm(r) / np.linalg.norm(b)
        say(f"   column (w={om[w]:.3f} eV, pol {pol}): oracle residual {rel:.2e}")
        assert rel <= 1e-8 + 1e-9
    s.close()


@pytest.mark.parametrize("form", ["dpcm", "iefpcm"])
def test_bem_phase_true_residuals_and_short_phase(form):
    """The block phase checks every pair's true FP64 residual through one
    operator apply over its basis: with the default step cap no pair needs a
    blocked cycle (one cycle each, relres <= rel_tol); with the phase cut
    short (4 block steps) the blocked solver takes every pair above rel_tol,
    and both spectra match the oracle."""
    c = cases()[0]
    solve = O.bem_ief_solve_spectrum if form == "iefpcm" else O.bem_solve_spectrum
    ref = solve(c["mesh"], c["om"], c["eps"], 1.0, c["pol"], 1e-4)
    for cap in (400, 4):
        s = px.Structure.bem(c["mesh"], 1.0, px.default_stream(), form=form)
        s.set_frequencies(c["om"], c["pol"], 1e-4, c["eps"])
        st = s.solve(precision=px.PX_FP64, rel_tol=1e-12, shifted_max_steps=cap)
        it, cyc, rr = s.stats()
        e = rel_err(s.spectrum()[1], ref["sigma"])
        say(f"[bem {form} phase cap {cap}] status {st} cycles max {cyc.max()} relres {rr.max():.1e} sigma {e:.1e}")
        assert st == px.PX_OK and rr.max() <= 1e-12 and e <= 1e-10
        if cap == 400:
            assert cyc.max() == 1
        else:
            assert cyc.max() > 1
        s.close()


@pytest.mark.parametrize("form", ["dpcm", "iefpcm"])
def test_bem_four_tesserae(form):
    """The smallest closed mesh: the four faces of a regular tetrahedron (edge
    20 Angstrom), one tile of 256 rows with 252 ghosts, against the oracle."""
    a = 20.0
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float) * a / np.sqrt(8.0)
    faces = [(1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1)]
    cen = np.array([v[list(f)].mean(axis=0) for f in faces])
    nrm = cen / np.linalg.norm(cen, axis=1)[:, None]
    area = np.full(4, np.sqrt(3.0) / 4.0 * a * a)
    m = dict(cen=cen, nrm=nrm, area=area, r_enc=float(np.linalg.norm(v[0])))
    om = np.linspace(2.5, 4.0, 5)
    eps = M.drude_permittivity(AG, om)
    solve = O.bem_ief_solve_spectrum if form == "iefpcm" else O.bem_solve_spectrum
    ref = solve(m, om, eps, 1.0, 0b101, 1e-4)
    s = px.Structure.bem(m, 1.0, px.default_stream(), form=form)
    s.set_frequencies(om, 0b101, 1e-4, eps)
    assert s.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    e_s, e_a = rel_err(s.spectrum()[1], ref["sigma"]), rel_err(s.spectrum()[0], ref["alpha"])
    e_q = rel_err(s.charges(2, 2), ref["q"][2, 1])
    say(f"[bem {form} tetrahedron] sigma {e_s:.1e} alpha {e_a:.1e} charges {e_q:.1e}")
    assert e_s <= 1e-10 and e_a <= 1e-9 and e_q <= 1e-8
    s.close()


def test_bem_ief_does_not_depend_on_where_the_mesh_sits():
    """Two unequal spheres (not neutral by symmetry) and the same pair moved
    by 1000 Angstrom: the same spectrum and charges on the GPU, both against
    the oracle (V and the dipole are taken relative to the tesserae's
    area-weighted centroid)."""
    s1, s2 = ME.sphere(20.0, 2), ME.sphere(30.0, 2)
    m = dict(cen=np.vstack([s1["cen"], s2["cen"] + np.array([60.0, 0.0, 0.0])]),
             nrm=np.vstack([s1["nrm"], s2["nrm"]]), area=np.concatenate([s1["area"], s2["area"]]), r_enc=60.0)
    moved = dict(m, cen=m["cen"] + np.array([1000.0, -300.0, 50.0]))
    om = np.linspace(3.0, 4.0, 12)
    eps = M.drude_permittivity(AG, om)
    ref = O.bem_ief_solve_spectrum(m, om, eps, 1.0, 0b011, 1e-4)
    out = []
    for mesh in (m, moved):
        s = px.Structure.bem(mesh, 1.0, px.default_stream(), form="iefpcm")
        s.set_frequencies(om, 0b011, 1e-4, eps)
        assert s.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
        out.append((s.spectrum()[0], s.charges(4, 0)))
        s.close()
    e_move = rel_err(out[1][0], out[0][0])
    e_ref = rel_err(out[0][0], ref["alpha"])
    e_q = rel_err(out[1][1], ref["q"][4, 0])
    say(f"[bem ief moved] alpha moved vs not {e_move:.1e}, vs oracle {e_ref:.1e}, charges {e_q:.1e}")
    assert e_move <= 1e-9 and e_ref <= 1e-9 and e_q <= 1e-8
