"""GPU parity of the BEM (DPCM) path against the oracle (Section 2.3, Eq.
bem-dpcm, "approximate" F; oracle/px_oracle.c or_bem_*).

Bounds (as for the atomistic models): operator apply max|dy| <= 1e-11
max|y| (FP64 sums over N terms); spectra solved to rel_tol 1e-12 in FP64:
rel_err sigma <= 1e-10, alpha <= 1e-9, charges <= 1e-8; PX_MIXED at rel_tol
1e-8 (the BEM apply is FP64 in both): rel_err sigma <= 1e-5.  Full size (the
benchmark's 20,480-tesserae sphere): the oracle residual of sampled columns
<= rel_tol + 1e-10.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2510_12731_amd as px
from workloads import materials as M
from workloads import mesh as ME

pytestmark = pytest.mark.gpu


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
    s = px.Structure.bem(c["mesh"], eps_env, px.default_stream())
    s.set_frequencies(c["om"], c["pol"], 1e-4, c["eps"])
    return s


@pytest.mark.parametrize("k,ncol", [(2, 1), (2, 3), (3, 2), (3, 6)])
def test_bem_apply_matches_oracle(k, ncol):
    """y = [M - z(eps2) I] x against the oracle's matrix-free apply, narrow
    blocks and a block wider than one launch (6 columns: 12 real)."""
    m = ME.spheroid(14.0, 28.0, k)
    n = len(m["area"])
    rng = np.random.default_rng(10 * k + ncol)
    x = rng.standard_normal((ncol, n)) + 1j * rng.standard_normal((ncol, n))
    om = np.linspace(2.0, 4.0, ncol)
    eps = M.drude_permittivity(AU, om)
    s = px.Structure.bem(m, 1.0, px.default_stream())
    y = s.apply(px.PX_FP64, om, x, eps)
    ref = O.bem_apply(m, eps, 1.0, x)
    e = rel_err(y, ref)
    say(f"[bem apply] n={n} ncol={ncol}: {e:.1e}")
    assert e <= 1e-11
    s.close()


@pytest.mark.parametrize("shifted", [2, 1])
def test_bem_spectra_match_oracle(shifted):
    """Sphere (3 polarizations: the block phase with shifted = 2), spheroid
    (one polarization) and gap dimer, FP64 and mixed, against the oracle's
    dense LU spectra."""
    for c in cases():
        ref = O.bem_solve_spectrum(c["mesh"], c["om"], c["eps"], 1.0, c["pol"], 1e-4)
        for prec, tol, bound in ((px.PX_FP64, 1e-12, 1e-10), (px.PX_MIXED, 1e-8, 1e-5)):
            s = make(c)
            st = s.solve(precision=prec, rel_tol=tol, shifted=shifted)
            alpha, sigma = s.spectrum()
            it, cyc, rr = s.stats()
            e_s, e_a = rel_err(sigma, ref["sigma"]), rel_err(alpha, ref["alpha"])
            say(f"[bem {c['name']}] shifted={shifted} prec={prec}: status {st} steps max {it.max()} "
                f"relres {rr.max():.1e} sigma {e_s:.1e} alpha {e_a:.1e}")
            assert st == px.PX_OK and rr.max() <= tol and e_s <= bound
            if prec == px.PX_FP64:
                assert e_a <= 1e-9
                pols = [l for l in range(3) if c["pol"] >> l & 1]
                for w in (0, len(c["om"]) - 1):
                    q = s.charges(w, pols[0])
                    assert rel_err(q, ref["q"][w, 0]) <= 1e-8
                    assert abs(q.sum()) <= 1e-8 * np.abs(q).sum()
            s.close()


def test_bem_medium_permittivity():
    """A sphere in a medium (eps1 = 1.77, water-like) against the oracle."""
    c = cases()[0]
    ref = O.bem_solve_spectrum(c["mesh"], c["om"], c["eps"], 1.77, c["pol"], 1e-4)
    s = make(c, eps_env=1.77)
    assert s.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    e = rel_err(s.spectrum()[1], ref["sigma"])
    say(f"[bem medium] sigma {e:.1e}")
    assert e <= 1e-10
    s.close()


def test_bem_edge_cases():
    m = ME.sphere(10.0, 1)
    bad = dict(m, area=np.where(np.arange(len(m["area"])) == 3, 0.0, m["area"]))
    with pytest.raises(px.PxError) as e:
        px.Structure.bem(bad)
    assert e.value.status == px.PX_E_INVALID
    bad = dict(m, nrm=np.where(np.arange(len(m["area"]))[:, None] == 5, 0.0, m["nrm"]))
    with pytest.raises(px.PxError):
        px.Structure.bem(bad)
    s = px.Structure.bem(m)
    with pytest.raises(px.PxError) as e:                     # eps2 = eps1: no interface
        s.set_frequencies(np.array([2.0]), 0b001, 1e-4, np.array([1.0 + 0.0j]))
    assert e.value.status == px.PX_E_INVALID
    with pytest.raises(px.PxError):                           # eps2 is required
        s.set_frequencies(np.array([2.0]), 0b001, 1e-4, None)
    s.set_frequencies(np.array([2.0, 3.0]), 0b001, 1e-4, np.array([-2.5 + 0.3j, -1.0 + 0.2j]))
    with pytest.raises(px.PxError):                           # the atomistic probe fields
        s.probe_field(np.zeros(len(m["area"])), None, np.zeros((1, 3)))
    with pytest.raises(px.PxError):                           # no FP32 BEM apply
        s.apply(px.PX_MIXED, np.array([2.0]), np.ones((1, len(m["area"]))), np.array([-2.0 + 0.1j]))
    s.close()


def test_bem_batch_refuses_stacking_and_solves_whole():
    """pxSolveBatch refuses a BEM structure in the stacked block (shifted = 0)
    and solves it whole beside an omegaFQ structure otherwise, each as alone."""
    c = cases()[2]
    s = make(c)
    with pytest.raises(px.PxError) as e:
        px.solve_batch([s], shifted=0)
    assert e.value.status == px.PX_E_INVALID
    from workloads import geometry as G
    ag = M.load("ag_wfq")
    a = px.Structure(0, G.fcc_sphere_n(500, seed=9), ag, px.default_stream())
    a.set_frequencies(np.linspace(2.5, 4.5, 16), 0b001)
    assert px.solve_batch([s, a], precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    sig_b = s.spectrum()[1]
    solo = make(c)
    assert solo.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    e = rel_err(sig_b, solo.spectrum()[1])
    say(f"[bem batch] vs alone {e:.1e}")
    assert e <= 1e-10
    for x in (s, a, solo):
        x.close()


def test_bem_no_alloc_apply_matches():
    import torch
    m = ME.sphere(25.0, 3)
    n = len(m["area"])
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    om = np.array([3.5, 3.8])
    eps = M.drude_permittivity(AG, om)
    s = px.Structure.bem(m)
    xd = torch.from_numpy(x.view(np.float64).copy()).to("cuda")
    yd = torch.zeros_like(xd)
    torch.cuda.synchronize()
    px.pxApplyOperatorNoAlloc(s.h, om, xd.data_ptr(), yd.data_ptr(), eps)
    y = yd.cpu().numpy().view(np.complex128).reshape(x.shape)
    assert rel_err(y, s.apply(px.PX_FP64, om, x, eps)) <= 1e-12
    s.close()


def test_bem_sphere_full_size():
    """The benchmark's BEM workload: 20,480-tesserae Ag sphere (R = 80
    Angstrom), 64 frequencies x 3 polarizations, rel_tol 1e-8: sampled columns
    (one at the Frohlich resonance) under the oracle's own operator, charge
    neutrality, isotropy and passivity on every frequency."""
    m = ME.sphere(80.0, 5)
    om = np.linspace(3.2, 4.4, 64)
    eps = M.drude_permittivity(AG, om)
    s = px.Structure.bem(m, 1.0, px.default_stream())
    s.set_frequencies(om, 0b111, 1e-4, eps)
    st = s.solve(precision=px.PX_MIXED, rel_tol=1e-8)
    it, cyc, rr = s.stats()
    alpha, sigma = s.spectrum()
    say(f"[bem full size] n={len(m['area'])}: status {st} steps max {it.max()} relres max {rr.max():.1e}")
    assert st == px.PX_OK and rr.max() <= 1e-8
    iso = np.trace(alpha, axis1=1, axis2=2) / 3
    assert np.abs(alpha - iso[:, None, None] * np.eye(3)).max() <= 1e-6 * np.abs(iso).max()
    assert np.all(sigma > 0)
    w_peak = int(np.argmax(sigma))
    for w, pol in ((w_peak, 0), (5, 2)):
        q = s.charges(w, pol)
        assert abs(q.sum()) <= 1e-8 * np.abs(q).sum()
        b = O.bem_rhs(m, pol, 1e-4)
        r = b - O.bem_apply(m, eps[w:w + 1], 1.0, q[None, :])[0]
        rel = np.linalg.norm(r) / np.linalg.norm(b)
        say(f"   column (w={om[w]:.3f} eV, pol {pol}): oracle residual {rel:.2e}")
        assert rel <= 1e-8 + 1e-10
    s.close()


def test_bem_dipole_does_not_depend_on_where_the_mesh_sits():
    """Two unequal spheres (charges neutral only to ~1e-4 of sum |q|) and the
    same pair moved by 1000 Angstrom: the same polarizability on the GPU (the
    dipole is taken from the tesserae's area-weighted centroid), and the
    oracle's."""
    s1, s2 = ME.sphere(20.0, 2), ME.sphere(30.0, 2)
    m = dict(cen=np.vstack([s1["cen"], s2["cen"] + np.array([60.0, 0.0, 0.0])]),
             nrm=np.vstack([s1["nrm"], s2["nrm"]]), area=np.concatenate([s1["area"], s2["area"]]), r_enc=60.0)
    moved = dict(m, cen=m["cen"] + np.array([1000.0, -300.0, 50.0]))
    om = np.linspace(3.0, 4.0, 12)
    eps = M.drude_permittivity(AG, om)
    ref = O.bem_solve_spectrum(m, om, eps, 1.0, 0b011, 1e-4)
    al = []
    for mesh in (m, moved):
        s = px.Structure.bem(mesh, 1.0, px.default_stream())
        s.set_frequencies(om, 0b011, 1e-4, eps)
        assert s.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
        al.append(s.spectrum()[0])
        s.close()
    e_move, e_ref = rel_err(al[1], al[0]), rel_err(al[0], ref["alpha"])
    say(f"[bem moved] alpha moved vs not {e_move:.1e}, vs oracle {e_ref:.1e}")
    assert e_move <= 1e-9 and e_ref <= 1e-9
