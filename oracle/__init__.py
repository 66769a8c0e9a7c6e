"""Reference oracle (plain single-threaded FP64 C, loaded through ctypes).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library and its Python
binding never do.  The C source, px_oracle.c, follows the paper's equations
step by step (Sections 2.1, 2.2, 2.3, 6 and 7) with a dense build and its own LU.

Conventions of this wrapper:
  * coordinates in Angstrom, frequencies in eV, parameters as the flat vector
    ``workloads.materials.param_vector`` builds (units in the parameter names);
  * complex arrays are numpy complex128;
  * unknown order for the dipole model is [q | mu_x | mu_y | mu_z] (each N long).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "px_oracle.c")
_LIB = os.path.join(_HERE, "libpxoracle.so")

_lib = None


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lp = ctypes.POINTER(ctypes.c_int64)
    lib.or_build_kbar.argtypes = [i64, dp, dp, dp]
    lib.or_build_tqq.argtypes = [i64, dp, dp, dp]
    lib.or_build_tfull.argtypes = [i64, dp, dp, dp]
    lib.or_drude_weight.argtypes = [dp]
    lib.or_drude_weight.restype = ctypes.c_double
    lib.or_zq.argtypes = [dp, ctypes.c_double, dp]
    lib.or_lu_factor.argtypes = [i64, dp, lp]
    lib.or_lu_factor.restype = i64
    lib.or_lu_factor_partial.argtypes = [i64, dp, lp, i64]
    lib.or_lu_factor_partial.restype = i64
    lib.or_lu_solve.argtypes = [i64, dp, lp, dp]
    lib.or_solve_spectrum.argtypes = [ctypes.c_int, i64, dp, dp, i64, dp, ctypes.c_uint32, ctypes.c_double,
                                      dp, dp, dp, dp]
    lib.or_solve_spectrum.restype = i64
    lib.or_apply.argtypes = [ctypes.c_int, i64, dp, dp, i64, dp, dp, dp, dp]
    lib.or_rhs.argtypes = [ctypes.c_int, i64, dp, dp, ctypes.c_int, ctypes.c_double, dp]
    lib.or_tapply_rows.argtypes = [ctypes.c_int, i64, dp, dp, i64, lp, i64, dp, dp]
    lib.or_assemble.argtypes = [ctypes.c_int, i64, dp, dp, ctypes.c_double, dp, dp]
    lib.or_constants.argtypes = [dp]
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.or_solve_spectrum_het.argtypes = [ctypes.c_int, i64, dp, ip, dp, dp, i64, dp, ctypes.c_uint32,
                                          ctypes.c_double, dp, dp, dp, dp, dp]
    lib.or_solve_spectrum_het.restype = i64
    lib.or_apply_het.argtypes = [ctypes.c_int, i64, dp, ip, dp, dp, i64, dp, dp, dp, dp, dp]
    lib.or_rhs_het.argtypes = [ctypes.c_int, i64, dp, ip, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                               dp]
    lib.or_probe.argtypes = [ctypes.c_int, i64, dp, dp, dp, dp, i64, dp, dp, dp, dp]
    lib.or_bem_matrix.argtypes = [i64, dp, dp, dp, ctypes.c_double, dp]
    lib.or_bem_rhs.argtypes = [i64, dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double, dp]
    lib.or_bem_apply.argtypes = [i64, dp, dp, dp, ctypes.c_double, i64, dp, dp, dp, dp]
    lib.or_bem_solve_spectrum.argtypes = [i64, dp, dp, dp, ctypes.c_double, i64, dp, dp, dp, ctypes.c_uint32,
                                          ctypes.c_double, dp, dp, dp]
    lib.or_bem_solve_spectrum.restype = i64
    lib.or_bem_ief_matrices.argtypes = [i64, dp, dp, dp, ctypes.c_double, dp, dp]
    lib.or_bem_ief_rhs.argtypes = [i64, dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double, dp]
    lib.or_bem_ief_apply.argtypes = [i64, dp, dp, dp, ctypes.c_double, i64, dp, dp, dp, dp]
    lib.or_bem_ief_potential.argtypes = [i64, dp, dp, dp, ctypes.c_double, i64, dp, dp]
    lib.or_bem_ief_solve_spectrum.argtypes = [i64, dp, dp, dp, ctypes.c_double, i64, dp, dp, dp, ctypes.c_uint32,
                                              ctypes.c_double, dp, dp, dp]
    lib.or_bem_ief_solve_spectrum.restype = i64
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _l(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _xyz(xyz):
    return np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)


def _pv(p):
    from_dict = isinstance(p, dict)
    if from_dict:
        raise TypeError("pass the flat parameter vector (workloads.materials.param_vector)")
    return np.ascontiguousarray(p, dtype=np.float64)


def constants():
    out = np.zeros(3)
    _load().or_constants(_d(out))
    return dict(ang_per_bohr=out[0], ev_per_hartree=out[1], c_au=out[2])


def kbar(xyz, p):
    xyz = _xyz(xyz)
    n = len(xyz)
    out = np.zeros((n, n))
    _load().or_build_kbar(n, _d(xyz), _d(_pv(p)), _d(out))
    return out


def tqq(xyz, p):
    xyz = _xyz(xyz)
    n = len(xyz)
    out = np.zeros((n, n))
    _load().or_build_tqq(n, _d(xyz), _d(_pv(p)), _d(out))
    return out


def tfull(xyz, p):
    xyz = _xyz(xyz)
    n = len(xyz)
    out = np.zeros((4 * n, 4 * n))
    _load().or_build_tfull(n, _d(xyz), _d(_pv(p)), _d(out))
    return out


def drude_weight(p):
    return _load().or_drude_weight(_d(_pv(p)))


def zq(p, omega_hartree):
    out = np.zeros(2)
    _load().or_zq(_d(_pv(p)), float(omega_hartree), _d(out))
    return complex(out[0], out[1])


def lu_solve(a, b):
    """Solve a x = b with the oracle's own LU (a: n x n complex, b: n or n x k)."""
    a = np.ascontiguousarray(a, dtype=np.complex128).copy()
    n = a.shape[0]
    piv = np.zeros(n, dtype=np.int64)
    rc = _load().or_lu_factor(n, _d(a.view(np.float64)), _l(piv))
    if rc != 0:
        raise np.linalg.LinAlgError(f"zero pivot at step {rc - 1}")
    b2 = np.array(b, dtype=np.complex128, copy=True)
    cols = b2.reshape(n, -1).T.copy()
    for c in range(cols.shape[0]):
        col = np.ascontiguousarray(cols[c])
        _load().or_lu_solve(n, _d(a.view(np.float64)), _l(piv), _d(col.view(np.float64)))
        cols[c] = col
    return cols.T.reshape(b2.shape)


def lu_factor_partial(a, kmax):
    """Run the first kmax elimination steps in place (timing samples only)."""
    n = a.shape[0]
    piv = np.zeros(n, dtype=np.int64)
    return _load().or_lu_factor_partial(n, _d(a.view(np.float64)), _l(piv), int(kmax))


def _alpha_ib_arr(alpha_ib, n):
    if alpha_ib is None:
        return np.zeros(2 * max(n, 1))
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha_ib, dtype=np.complex128), (n,)))
    return a.view(np.float64).copy()


def solve_spectrum(model, xyz, p, omega_ev, pol_mask, e0, alpha_ib=None):
    """Direct-solve spectrum.  Returns dict(q=[n_omega, n_pol, nu] complex,
    alpha=[n_omega, 3, 3] complex, sigma=[n_omega] bohr^2, status=int)."""
    xyz = _xyz(xyz)
    n = len(xyz)
    nu = 4 * n if model == 1 else n
    om = np.ascontiguousarray(omega_ev, dtype=np.float64)
    nw = len(om)
    npol = bin(pol_mask & 7).count("1")
    q = np.zeros((nw, npol, nu), dtype=np.complex128)
    alpha = np.zeros((nw, 3, 3), dtype=np.complex128)
    sigma = np.zeros(nw)
    aib = _alpha_ib_arr(alpha_ib, nw)
    st = _load().or_solve_spectrum(int(model), n, _d(xyz), _d(_pv(p)), nw, _d(om), int(pol_mask), float(e0),
                                   _d(aib), _d(q.view(np.float64)), _d(alpha.view(np.float64)), _d(sigma))
    return dict(q=q, alpha=alpha, sigma=sigma, status=int(st))


def apply(model, xyz, p, omega_ev, x, alpha_ib=None):
    """y = A(w_c) x_c for each column; x: [ncol, nu] complex, omega_ev: [ncol]."""
    xyz = _xyz(xyz)
    n = len(xyz)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    ncol = x.shape[0]
    om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega_ev, dtype=np.float64), (ncol,)))
    y = np.zeros_like(x)
    aib = _alpha_ib_arr(alpha_ib, ncol)
    _load().or_apply(int(model), n, _d(xyz), _d(_pv(p)), ncol, _d(om), _d(aib), _d(x.view(np.float64)),
                     _d(y.view(np.float64)))
    return y


def rhs(model, xyz, p, pol, e0):
    xyz = _xyz(xyz)
    n = len(xyz)
    nu = 4 * n if model == 1 else n
    b = np.zeros(nu, dtype=np.complex128)
    _load().or_rhs(int(model), n, _d(xyz), _d(_pv(p)), int(pol), float(e0), _d(b.view(np.float64)))
    return b


def _types(types, n):
    t = np.ascontiguousarray(types, dtype=np.int32)
    assert t.shape == (n,) and np.all((t == 0) | (t == 1))
    return t


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def solve_spectrum_het(model, xyz, types, pa, pb, omega_ev, pol_mask, e0, alpha_ib_a=None, alpha_ib_b=None):
    """Direct-solve spectrum of a two-type structure (Eq. wfqfmu-leghe; model 0
    is its charge block).  types[i] in {0: A, 1: B}; returns as solve_spectrum."""
    xyz = _xyz(xyz)
    n = len(xyz)
    t = _types(types, n)
    nu = 4 * n if model == 1 else n
    om = np.ascontiguousarray(omega_ev, dtype=np.float64)
    nw = len(om)
    npol = bin(pol_mask & 7).count("1")
    q = np.zeros((nw, npol, nu), dtype=np.complex128)
    alpha = np.zeros((nw, 3, 3), dtype=np.complex128)
    sigma = np.zeros(nw)
    aa, ab = _alpha_ib_arr(alpha_ib_a, nw), _alpha_ib_arr(alpha_ib_b, nw)
    st = _load().or_solve_spectrum_het(int(model), n, _d(xyz), _i(t), _d(_pv(pa)), _d(_pv(pb)), nw, _d(om),
                                       int(pol_mask), float(e0), _d(aa), _d(ab), _d(q.view(np.float64)),
                                       _d(alpha.view(np.float64)), _d(sigma))
    return dict(q=q, alpha=alpha, sigma=sigma, status=int(st))


def apply_het(model, xyz, types, pa, pb, omega_ev, x, alpha_ib_a=None, alpha_ib_b=None):
    """y = A(w_c) x_c of a two-type structure; x: [ncol, nu] complex."""
    xyz = _xyz(xyz)
    n = len(xyz)
    t = _types(types, n)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    ncol = x.shape[0]
    om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega_ev, dtype=np.float64), (ncol,)))
    y = np.zeros_like(x)
    aa, ab = _alpha_ib_arr(alpha_ib_a, ncol), _alpha_ib_arr(alpha_ib_b, ncol)
    _load().or_apply_het(int(model), n, _d(xyz), _i(t), _d(_pv(pa)), _d(_pv(pb)), ncol, _d(om), _d(aa), _d(ab),
                         _d(x.view(np.float64)), _d(y.view(np.float64)))
    return y


def rhs_het(model, xyz, types, pa, pb, omega_ev, pol, e0):
    xyz = _xyz(xyz)
    n = len(xyz)
    t = _types(types, n)
    nu = 4 * n if model == 1 else n
    b = np.zeros(nu, dtype=np.complex128)
    _load().or_rhs_het(int(model), n, _d(xyz), _i(t), _d(_pv(pa)), _d(_pv(pb)), float(omega_ev), int(pol),
                       float(e0), _d(b.view(np.float64)))
    return b


def tapply_rows(model, xyz, p, rows, x):
    """Sampled rows of T X for real X [ncol, nu]; returns [ncol, len(rows)]."""
    xyz = _xyz(xyz)
    n = len(xyz)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    y = np.zeros((x.shape[0], len(rows)))
    _load().or_tapply_rows(int(model), n, _d(xyz), _d(_pv(p)), len(rows), _l(rows), x.shape[0], _d(x), _d(y))
    return y


def assemble(model, xyz, p, omega_ev, alpha_ib=None):
    xyz = _xyz(xyz)
    n = len(xyz)
    nu = 4 * n if model == 1 else n
    a = np.zeros((nu, nu), dtype=np.complex128)
    aib = _alpha_ib_arr(alpha_ib, 1)
    _load().or_assemble(int(model), n, _d(xyz), _d(_pv(p)), float(omega_ev), _d(aib), _d(a.view(np.float64)))
    return a


def probe(model, xyz, p, q, mu, pts):
    """Potential, field and density of Gaussian charges q [n] (and dipoles mu
    [3, n], model 1) on the atoms at points pts [npts, 3] (Angstrom).  Returns
    dict(phi=[npts], field=[npts, 3], rho=[npts]) complex, atomic units."""
    xyz = _xyz(xyz)
    n = len(xyz)
    q = np.ascontiguousarray(q, dtype=np.complex128).reshape(n)
    mu_arr = None
    if model == 1 and mu is not None:
        mu_arr = np.ascontiguousarray(mu, dtype=np.complex128).reshape(3 * n)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    npts = len(pts)
    phi = np.zeros(npts, dtype=np.complex128)
    field = np.zeros((npts, 3), dtype=np.complex128)
    rho = np.zeros(npts, dtype=np.complex128)
    _load().or_probe(int(model), n, _d(xyz), _d(_pv(p)), _d(q.view(np.float64)),
                     _d(mu_arr.view(np.float64)) if mu_arr is not None else None, npts, _d(pts),
                     _d(phi.view(np.float64)), _d(field.view(np.float64)), _d(rho.view(np.float64)))
    return dict(phi=phi, field=field, rho=rho)


# ---- BEM (Section 2.3, Eq. bem-dpcm) ---------------------------------------
# mesh: a dict from workloads.mesh (cen, nrm, area in Angstrom units, r_enc);
# eps2: complex metal permittivity per frequency (or per column); eps1: the
# medium's (complex scalar).

def _mesh(m):
    cen = np.ascontiguousarray(m["cen"], dtype=np.float64).reshape(-1, 3)
    nrm = np.ascontiguousarray(m["nrm"], dtype=np.float64).reshape(-1, 3)
    area = np.ascontiguousarray(m["area"], dtype=np.float64).reshape(-1)
    return len(area), cen, nrm, area, float(m["r_enc"])


def _cplx(a, n):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.complex128), (n,))).view(np.float64).copy()


def bem_matrix(m):
    n, cen, nrm, area, r = _mesh(m)
    out = np.zeros((n, n))
    _load().or_bem_matrix(n, _d(cen), _d(nrm), _d(area), r, _d(out))
    return out


def bem_rhs(m, pol, e0):
    n, cen, nrm, area, r = _mesh(m)
    b = np.zeros(n, dtype=np.complex128)
    _load().or_bem_rhs(n, _d(cen), _d(nrm), _d(area), r, int(pol), float(e0), _d(b.view(np.float64)))
    return b


def bem_apply(m, eps2, eps1, x):
    """y_c = [M - z(eps2_c) I] x_c; x: [ncol, n] complex, eps2: [ncol]."""
    n, cen, nrm, area, r = _mesh(m)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    ncol = x.shape[0]
    y = np.zeros_like(x)
    _load().or_bem_apply(n, _d(cen), _d(nrm), _d(area), r, ncol, _d(_cplx(eps2, ncol)), _d(_cplx(eps1, 1)),
                         _d(x.view(np.float64)), _d(y.view(np.float64)))
    return y


def bem_solve_spectrum(m, omega_ev, eps2, eps1, pol_mask, e0):
    """Direct-solve BEM spectrum.  Returns dict(q=[n_omega, n_pol, n] tessera
    charges, alpha=[n_omega, 3, 3], sigma=[n_omega] bohr^2, status)."""
    n, cen, nrm, area, r = _mesh(m)
    om = np.ascontiguousarray(omega_ev, dtype=np.float64)
    nw = len(om)
    npol = bin(pol_mask & 7).count("1")
    q = np.zeros((nw, npol, n), dtype=np.complex128)
    alpha = np.zeros((nw, 3, 3), dtype=np.complex128)
    sigma = np.zeros(nw)
    st = _load().or_bem_solve_spectrum(n, _d(cen), _d(nrm), _d(area), r, nw, _d(om), _d(_cplx(eps2, nw)),
                                       _d(_cplx(eps1, 1)), int(pol_mask), float(e0), _d(q.view(np.float64)),
                                       _d(alpha.view(np.float64)), _d(sigma))
    return dict(q=q, alpha=alpha, sigma=sigma, status=int(st))


# ---- BEM, IEFPCM (Section 2.3, Eq. bem-iefpcm) -------------------------------
# The same mesh dicts; S (bohr) and F (dimensionless) are the paper's matrices
# (F's diagonal read as the double layer's self patch, -S_ii / 2R).

def bem_ief_matrices(m):
    """(S, F) as dense [n, n] arrays."""
    n, cen, nrm, area, r = _mesh(m)
    s = np.zeros((n, n))
    f = np.zeros((n, n))
    _load().or_bem_ief_matrices(n, _d(cen), _d(nrm), _d(area), r, _d(s), _d(f))
    return s, f


def bem_ief_rhs(m, pol, e0):
    """-(2 pi I + F) V with V_i = -E0 (s_i - c)_pol, c the area-weighted
    centroid of the tesserae: [n] complex."""
    n, cen, nrm, area, r = _mesh(m)
    b = np.zeros(n, dtype=np.complex128)
    _load().or_bem_ief_rhs(n, _d(cen), _d(nrm), _d(area), r, int(pol), float(e0), _d(b.view(np.float64)))
    return b


def bem_ief_apply(m, eps2, eps1, x):
    """y_c = [2 pi f(eps2_c) I + F] x_c; x: [ncol, n] complex, eps2: [ncol]."""
    n, cen, nrm, area, r = _mesh(m)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    ncol = x.shape[0]
    y = np.zeros_like(x)
    _load().or_bem_ief_apply(n, _d(cen), _d(nrm), _d(area), r, ncol, _d(_cplx(eps2, ncol)), _d(_cplx(eps1, 1)),
                             _d(x.view(np.float64)), _d(y.view(np.float64)))
    return y


def bem_ief_potential(m, q):
    """y_c = S A^-1 q_c, the potential of the charges at the barycentres;
    q: [ncol, n] complex."""
    n, cen, nrm, area, r = _mesh(m)
    q = np.ascontiguousarray(np.atleast_2d(q), dtype=np.complex128)
    y = np.zeros_like(q)
    _load().or_bem_ief_potential(n, _d(cen), _d(nrm), _d(area), r, q.shape[0], _d(q.view(np.float64)),
                                 _d(y.view(np.float64)))
    return y


def bem_ief_solve_spectrum(m, omega_ev, eps2, eps1, pol_mask, e0):
    """Direct-solve IEFPCM spectrum.  Returns dict(q=[n_omega, n_pol, n]
    tessera charges, alpha=[n_omega, 3, 3], sigma=[n_omega] bohr^2, status)."""
    n, cen, nrm, area, r = _mesh(m)
    om = np.ascontiguousarray(omega_ev, dtype=np.float64)
    nw = len(om)
    npol = bin(pol_mask & 7).count("1")
    q = np.zeros((nw, npol, n), dtype=np.complex128)
    alpha = np.zeros((nw, 3, 3), dtype=np.complex128)
    sigma = np.zeros(nw)
    st = _load().or_bem_ief_solve_spectrum(n, _d(cen), _d(nrm), _d(area), r, nw, _d(om), _d(_cplx(eps2, nw)),
                                           _d(_cplx(eps1, 1)), int(pol_mask), float(e0), _d(q.view(np.float64)),
                                           _d(alpha.view(np.float64)), _d(sigma))
    return dict(q=q, alpha=alpha, sigma=sigma, status=int(st))
