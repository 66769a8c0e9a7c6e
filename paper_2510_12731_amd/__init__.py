"""Python binding of the MI355X omegaFQ / omegaFQFmu solver library.

Argument marshalling only: every step of the solve runs in the HIP library
``libplasmonx_hip.so`` built from ``csrc/``.  The functions carry the names of
the C entry points declared in ``include/plasmonx.h``; ``Structure`` wraps them
for convenience.  Importing this package never builds anything and never
falls back to another implementation: if the library is missing, ``load()``
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplasmonx_hip.so")

PX_OK, PX_E_INVALID, PX_E_OOM, PX_E_NOTCONV, PX_E_DEVICE, PX_E_STATE = range(6)
PX_WFQ, PX_WFQFMU, PX_BEM = 0, 1, 2
PX_FP64, PX_MIXED = 0, 1
PX_ORTHO_CGS2, PX_ORTHO_DCGS2 = 0, 1
PX_TAPPLY_AUTO, PX_TAPPLY_ON_THE_FLY, PX_TAPPLY_STORED = 0, 1, 2
STATUS_NAMES = {0: "PX_OK", 1: "PX_E_INVALID", 2: "PX_E_OOM", 3: "PX_E_NOTCONV", 4: "PX_E_DEVICE", 5: "PX_E_STATE"}

EXPORTED = ["pxDefaultSolveOptions", "pxCreateStructure", "pxCreateStructureHetero", "pxSetFrequencies", "pxSolveSpectrum", "pxSolveBatch",
            "pxGetCharges", "pxGetSpectrum", "pxGetSolveStats", "pxApplyOperator", "pxGetSize", "pxGetTimings", "pxGetWork", "pxGetTApplyStats",
            "pxDestroyStructure", "pxLastError", "pxServerCreate", "pxServerSubmit", "pxServerStep",
            "pxServerQuery", "pxServerDestroy", "pxInducedField", "pxProbeField", "pxGetProbeStats",
            "pxServerMemory", "pxSolveFootprint", "pxGetSolveStatus", "pxApplyOperatorNoAlloc", "pxCreateBem",
            "pxCreateBemIefpcm", "pxSetAllocator", "pxReleaseCache", "pxSolveSpectrumAsync", "pxSolveProgress",
            "pxSolveWait"]


class PxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class pxMaterial(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("a_eff", "r_q", "r_mu", "tau", "density", "eff_mass", "fermi_d",
                                               "fermi_s", "r0_ang", "cutoff_ang", "fermi_energy_ev",
                                               "sheet_thickness")]


class pxSolveOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("restart_m", ctypes.c_int32), ("rel_tol", ctypes.c_double),
                ("max_cycles", ctypes.c_int32), ("max_block_cols", ctypes.c_int32),
                ("inner_reduction", ctypes.c_double), ("timings", ctypes.c_int32), ("stall_cycles", ctypes.c_int32),
                ("max_restart_m", ctypes.c_int32), ("block_cols", ctypes.c_int32), ("ortho", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("t_apply", ctypes.c_int32), ("shifted", ctypes.c_int32),
                ("shifted_max_steps", ctypes.c_int32)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
# pxDeviceAllocFn / pxDeviceFreeFn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run python -m paper_2510_12731_amd.build)")
    # torch bundles its own HIP runtime under the same soname as ROCm's
    # (libamdhip64.so.7); whichever is loaded first serves the whole process.
    # Import torch first so that the library and torch's streams share one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.pxDefaultSolveOptions.argtypes = [ctypes.POINTER(pxSolveOptions)]
    lib.pxDefaultSolveOptions.restype = None
    lib.pxCreateStructure.argtypes = [ctypes.c_int, i64, _dp, ctypes.POINTER(pxMaterial), _vp, ctypes.POINTER(_vp)]
    lib.pxCreateStructureHetero.argtypes = [ctypes.c_int, i64, _dp, ctypes.POINTER(ctypes.c_uint8),
                                            ctypes.POINTER(pxMaterial), ctypes.POINTER(pxMaterial), _vp,
                                            ctypes.POINTER(_vp)]
    lib.pxSetFrequencies.argtypes = [_vp, i32, _dp, u32, ctypes.c_double, _dp]
    lib.pxSolveSpectrum.argtypes = [_vp, ctypes.POINTER(pxSolveOptions)]
    lib.pxSolveSpectrumAsync.argtypes = [_vp, ctypes.POINTER(pxSolveOptions)]
    lib.pxSolveProgress.argtypes = [_vp, ctypes.POINTER(i32)]
    lib.pxSolveWait.argtypes = [_vp]
    lib.pxSolveBatch.argtypes = [ctypes.POINTER(_vp), i32, ctypes.POINTER(pxSolveOptions)]
    lib.pxGetCharges.argtypes = [_vp, i32, i32, _dp, _dp]
    lib.pxGetSpectrum.argtypes = [_vp, _dp, _dp]
    lib.pxGetSolveStats.argtypes = [_vp, ctypes.POINTER(i32), ctypes.POINTER(i32), _dp]
    lib.pxApplyOperator.argtypes = [_vp, i32, i32, _dp, _dp, _dp, _dp]
    lib.pxGetSize.argtypes = [_vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.pxGetTimings.argtypes = [_vp, _dp, ctypes.POINTER(i64)]
    lib.pxGetWork.argtypes = [_vp, _dp]
    lib.pxGetTApplyStats.argtypes = [_vp, ctypes.POINTER(i64), _dp, _dp]
    lib.pxInducedField.argtypes = [_vp, i32, i32, i64, _dp, _dp, _dp]
    lib.pxProbeField.argtypes = [_vp, _dp, _dp, i64, _dp, _dp, _dp]
    lib.pxGetProbeStats.argtypes = [_vp, _dp]
    lib.pxServerCreate.argtypes = [ctypes.c_double, ctypes.POINTER(pxSolveOptions), _vp, ctypes.POINTER(_vp)]
    lib.pxServerSubmit.argtypes = [_vp, _vp]
    lib.pxServerStep.argtypes = [_vp, ctypes.POINTER(_vp), i32, ctypes.POINTER(i32)]
    lib.pxServerQuery.argtypes = [_vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                  ctypes.POINTER(i64)]
    lib.pxCreateBem.argtypes = [i64, _dp, _dp, _dp, ctypes.c_double, _dp, _vp, ctypes.POINTER(_vp)]
    lib.pxCreateBemIefpcm.argtypes = [i64, _dp, _dp, _dp, ctypes.c_double, _dp, _vp, ctypes.POINTER(_vp)]
    lib.pxApplyOperatorNoAlloc.argtypes = [_vp, i32, _dp, _dp, _vp, _vp]
    lib.pxServerMemory.argtypes = [_vp, _dp, _dp, ctypes.POINTER(i32)]
    lib.pxSolveFootprint.argtypes = [_vp, ctypes.POINTER(pxSolveOptions), _dp]
    lib.pxGetSolveStatus.argtypes = [_vp, ctypes.POINTER(i32), ctypes.c_char_p, i32]
    lib.pxSetAllocator.argtypes = [ALLOC_FN, FREE_FN, _vp]
    lib.pxReleaseCache.argtypes = []
    lib.pxServerDestroy.argtypes = [_vp]
    lib.pxServerDestroy.restype = None
    lib.pxDestroyStructure.argtypes = [_vp]
    lib.pxDestroyStructure.restype = None
    lib.pxLastError.argtypes = []
    lib.pxLastError.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("pxDefaultSolveOptions", "pxDestroyStructure", "pxLastError", "pxServerDestroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


_allocator = None   # the installed callbacks (kept alive while installed)


def pxSetAllocator(alloc, free, user=None):
    """pxSetAllocator with ctypes callbacks (ALLOC_FN, FREE_FN), or None, None."""
    global _allocator
    lib = load()
    if alloc is None and free is None:
        _check(lib.pxSetAllocator(ALLOC_FN(), FREE_FN(), user))
    else:
        _check(lib.pxSetAllocator(alloc, free, user))
    # blocks made by earlier callbacks still go back through them
    _allocator = (alloc, free, _allocator)


def pxReleaseCache():
    _check(load().pxReleaseCache())


def use_torch_allocator():
    """Route the library's device memory through torch's caching allocator:
    torch.cuda.memory_allocated() then counts it, and torch reuses it after
    pxDestroyStructure."""
    import torch

    def alloc(nbytes, device, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), int(device))
        except Exception:   # out of memory: the library reports PX_E_OOM
            return None

    def free(ptr, device, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:   # interpreter shutting down: the block is leaked
            pass

    pxSetAllocator(ALLOC_FN(alloc), FREE_FN(free))


def use_hip_allocator():
    """Back to hipMalloc/hipFree (blocks made by torch still go back to it)."""
    pxSetAllocator(None, None)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _check(st, allow=(PX_OK,)):
    if st not in allow:
        raise PxError(st, load().pxLastError().decode())
    return st


def material(params) -> pxMaterial:
    """pxMaterial from a parameter dict (workload parameter files) or vector."""
    if isinstance(params, dict):
        keys = ("a_eff_bohr2", "r_q_bohr", "r_mu_bohr", "tau_au", "density_au", "eff_mass_au", "fermi_d", "fermi_s",
                "r0_ang", "cutoff_ang", "fermi_energy_ev", "sheet_thickness_bohr")
        vals = [float(params[k]) for k in keys]
    else:
        vals = [float(v) for v in params]
    return pxMaterial(*vals)


def default_stream():
    """The current torch stream (HIP) if torch sees a GPU, else None."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


# ---- same-name wrappers of the C entry points -------------------------------

def pxDefaultSolveOptions() -> pxSolveOptions:
    o = pxSolveOptions()
    load().pxDefaultSolveOptions(ctypes.byref(o))
    return o


def pxCreateStructure(model, xyz_ang, mat, hip_stream=None):
    xyz = np.ascontiguousarray(xyz_ang, dtype=np.float64).reshape(-1, 3)
    h = _vp()
    m = mat if isinstance(mat, pxMaterial) else material(mat)
    _check(load().pxCreateStructure(int(model), len(xyz), _ptr(xyz), ctypes.byref(m), hip_stream, ctypes.byref(h)))
    return h


def pxCreateStructureHetero(model, xyz_ang, types, mat_a, mat_b, hip_stream=None):
    """Two atom types: types[i] = 0 for mat_a, 1 for mat_b."""
    xyz = np.ascontiguousarray(xyz_ang, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
    if len(t) != len(xyz):
        raise PxError(PX_E_INVALID, "types and coordinates differ in length")
    h = _vp()
    ma = mat_a if isinstance(mat_a, pxMaterial) else material(mat_a)
    mb = mat_b if isinstance(mat_b, pxMaterial) else material(mat_b)
    _check(load().pxCreateStructureHetero(int(model), len(xyz), _ptr(xyz), t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                          ctypes.byref(ma), ctypes.byref(mb), hip_stream, ctypes.byref(h)))
    return h


def _bem_args(mesh, eps_env):
    cen = np.ascontiguousarray(mesh["cen"], dtype=np.float64).reshape(-1, 3)
    nrm = np.ascontiguousarray(mesh["nrm"], dtype=np.float64).reshape(-1, 3)
    area = np.ascontiguousarray(mesh["area"], dtype=np.float64).reshape(-1)
    e1 = np.array([complex(eps_env).real, complex(eps_env).imag])
    return cen, nrm, area, e1


def pxCreateBem(mesh, eps_env=1.0, hip_stream=None):
    """BEM (DPCM) structure from a mesh dict (cen, nrm, area in Angstrom
    units, r_enc)."""
    cen, nrm, area, e1 = _bem_args(mesh, eps_env)
    h = _vp()
    _check(load().pxCreateBem(len(area), _ptr(cen), _ptr(nrm), _ptr(area), float(mesh["r_enc"]), _ptr(e1), hip_stream,
                              ctypes.byref(h)))
    return h


def pxCreateBemIefpcm(mesh, eps_env=1.0, hip_stream=None):
    """BEM (IEFPCM) structure from a mesh dict, as pxCreateBem."""
    cen, nrm, area, e1 = _bem_args(mesh, eps_env)
    h = _vp()
    _check(load().pxCreateBemIefpcm(len(area), _ptr(cen), _ptr(nrm), _ptr(area), float(mesh["r_enc"]), _ptr(e1),
                                    hip_stream, ctypes.byref(h)))
    return h


def pxSetFrequencies(h, omega_ev, pol_mask, e0_au, alpha_ib=None):
    om = np.ascontiguousarray(omega_ev, dtype=np.float64)
    aib = None if alpha_ib is None else np.ascontiguousarray(np.asarray(alpha_ib, dtype=np.complex128)).view(np.float64)
    _check(load().pxSetFrequencies(h, len(om), _ptr(om), int(pol_mask), float(e0_au), _ptr(aib)))


def pxSolveSpectrum(h, opt: pxSolveOptions | None = None):
    return _check(load().pxSolveSpectrum(h, None if opt is None else ctypes.byref(opt)), (PX_OK, PX_E_NOTCONV))


def pxSolveSpectrumAsync(h, opt: pxSolveOptions | None = None):
    return _check(load().pxSolveSpectrumAsync(h, None if opt is None else ctypes.byref(opt)))


def pxSolveProgress(h):
    done = ctypes.c_int32()
    _check(load().pxSolveProgress(h, ctypes.byref(done)))
    return bool(done.value)


def pxSolveWait(h):
    return _check(load().pxSolveWait(h), (PX_OK, PX_E_NOTCONV))


def pxSolveBatch(handles, opt: pxSolveOptions | None = None):
    arr = (_vp * len(handles))(*[h.value if isinstance(h, _vp) else h for h in handles])
    return _check(load().pxSolveBatch(arr, len(handles), None if opt is None else ctypes.byref(opt)),
                  (PX_OK, PX_E_NOTCONV))


def pxApplyOperatorNoAlloc(h, omega_ev, x_dev_ptr, y_dev_ptr, alpha_ib=None):
    """FP64 y = A(w) x with x, y given as device addresses ([ncol][nu] complex
    interleaved); the library allocates nothing for the call."""
    om = np.ascontiguousarray(np.atleast_1d(omega_ev), dtype=np.float64)
    aib = None
    if alpha_ib is not None:
        aib = np.ascontiguousarray(np.asarray(alpha_ib, dtype=np.complex128).reshape(len(om), -1)).view(np.float64)
    _check(load().pxApplyOperatorNoAlloc(h, len(om), _ptr(om), _ptr(aib), ctypes.c_void_p(int(x_dev_ptr)),
                                         ctypes.c_void_p(int(y_dev_ptr))))


def pxGetSize(h):
    n, nu = ctypes.c_int64(), ctypes.c_int64()
    _check(load().pxGetSize(h, ctypes.byref(n), ctypes.byref(nu)))
    return n.value, nu.value


def pxGetCharges(h, i_omega, pol, with_dipoles=False):
    n, nu = pxGetSize(h)
    q = np.zeros(n, dtype=np.complex128)
    mu = np.zeros((3, n), dtype=np.complex128) if with_dipoles else None
    _check(load().pxGetCharges(h, int(i_omega), int(pol), _ptr(q.view(np.float64)),
                               None if mu is None else _ptr(mu.view(np.float64))))
    return (q, mu) if with_dipoles else q


def _probe_out(pts):
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    field = np.zeros((len(pts), 3), dtype=np.complex128)
    rho = np.zeros(len(pts), dtype=np.complex128)
    return pts, field, rho


def pxInducedField(h, i_omega, pol, pts):
    """Field [npts, 3] and density [npts] (complex, atomic units) of the solved
    column (i_omega, pol) at points pts [npts, 3] (Angstrom)."""
    pts, field, rho = _probe_out(pts)
    _check(load().pxInducedField(h, int(i_omega), int(pol), len(pts), _ptr(pts), _ptr(field.view(np.float64)),
                                 _ptr(rho.view(np.float64))))
    return field, rho


def pxProbeField(h, q, mu, pts):
    """Field and density of caller-given charges q [n] (and dipoles mu [3, n])
    on the structure's atoms (caller's atom order) at points pts (Angstrom)."""
    pts, field, rho = _probe_out(pts)
    q = np.ascontiguousarray(q, dtype=np.complex128).ravel()
    mu_a = None if mu is None else np.ascontiguousarray(mu, dtype=np.complex128).ravel()
    _check(load().pxProbeField(h, _ptr(q.view(np.float64)), None if mu_a is None else _ptr(mu_a.view(np.float64)),
                               len(pts), _ptr(pts), _ptr(field.view(np.float64)), _ptr(rho.view(np.float64))))
    return field, rho


def pxGetProbeStats(h):
    out = np.zeros(2)
    _check(load().pxGetProbeStats(h, _ptr(out)))
    return dict(ms_kernel=out[0], pairs=out[1])


def pxGetSpectrum(h, n_omega):
    alpha = np.zeros((n_omega, 3, 3), dtype=np.complex128)
    sigma = np.zeros(n_omega)
    _check(load().pxGetSpectrum(h, _ptr(alpha.view(np.float64)), _ptr(sigma)))
    return alpha, sigma


def pxGetSolveStats(h, ncol):
    it = (ctypes.c_int32 * ncol)()
    cy = (ctypes.c_int32 * ncol)()
    rr = np.zeros(ncol)
    _check(load().pxGetSolveStats(h, it, cy, _ptr(rr)))
    return np.array(it[:]), np.array(cy[:]), rr


def pxApplyOperator(h, precision, omega_ev, x, alpha_ib=None, het=False):
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    ncol = x.shape[0]
    om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega_ev, dtype=np.float64), (ncol,)))
    aib = None
    if alpha_ib is not None:
        a = np.asarray(alpha_ib, dtype=np.complex128)
        # two-type structures: alpha_IB of type A and of type B per column
        aib = np.ascontiguousarray(np.broadcast_to(a, (ncol, 2) if het else (ncol,))).view(np.float64)
    y = np.zeros_like(x)
    _check(load().pxApplyOperator(h, int(precision), ncol, _ptr(om), _ptr(aib), _ptr(x.view(np.float64)),
                                  _ptr(y.view(np.float64))))
    return y


def pxGetWork(h):
    """Algorithmic work of the last solve: FP32 T-apply FLOP, FP64 T-apply FLOP, HBM bytes."""
    w = np.zeros(3)
    _check(load().pxGetWork(h, _ptr(w)))
    return dict(flop_f32=float(w[0]), flop_f64=float(w[1]), hbm_bytes=float(w[2]))


def pxGetTApplyStats(h):
    """T-apply launches (and their timed milliseconds) of the last solve by method."""
    st = (ctypes.c_int64 * 4)()
    ms = np.zeros(4)
    fl = np.zeros(4)
    _check(load().pxGetTApplyStats(h, st, _ptr(ms), _ptr(fl)))
    names = ("f32_on_the_fly", "f32_stored", "f64_on_the_fly", "f64_stored")
    out = {nm: int(st[k]) for k, nm in enumerate(names)}
    out.update({"ms_" + nm: float(ms[k]) for k, nm in enumerate(names)})
    out.update({"flop_" + nm: float(fl[k]) for k, nm in enumerate(names)})
    return out


def pxGetTimings(h):
    ms = np.zeros(6)
    cnt = (ctypes.c_int64 * 6)()
    _check(load().pxGetTimings(h, _ptr(ms), cnt))
    return dict(ms_total=ms[0], ms_tapply_f32=ms[1], ms_tapply_f64_cycles=ms[2], ms_spmm=ms[3], ms_arnoldi=ms[4],
                ms_other=ms[5], n_tapply_f32=cnt[0], cols_f32_padded=cnt[1], cols_f32=cnt[2],
                n_tapply_f64=cnt[3], cols_f64_padded=cnt[4], cols_f64=cnt[5])


def pxDestroyStructure(h):
    if h is not None:
        load().pxDestroyStructure(h)


def pxLastError():
    return load().pxLastError().decode()


def solve_options(precision=None, restart_m=None, rel_tol=None, max_cycles=None, max_block_cols=None,
                  inner_reduction=None, timings=None, stall_cycles=None, max_restart_m=None, block_cols=None,
                  ortho=None, graph_steps=None, t_apply=None, shifted=None, shifted_max_steps=None):
    """pxSolveOptions: pxDefaultSolveOptions with the given fields replaced."""
    o = pxDefaultSolveOptions()
    given = dict(precision=precision, restart_m=restart_m, max_cycles=max_cycles, max_block_cols=max_block_cols,
                 stall_cycles=stall_cycles, max_restart_m=max_restart_m, block_cols=block_cols, ortho=ortho,
                 graph_steps=graph_steps, t_apply=t_apply, shifted=shifted, shifted_max_steps=shifted_max_steps)
    for name, v in given.items():
        if v is not None:
            setattr(o, name, int(v))
    if rel_tol is not None:
        o.rel_tol = float(rel_tol)
    if inner_reduction is not None:
        o.inner_reduction = float(inner_reduction)
    if timings is not None:
        o.timings = int(bool(timings))
    return o


def pxServerCreate(memory_budget_bytes, opt=None, hip_stream=None):
    h = _vp()
    _check(load().pxServerCreate(float(memory_budget_bytes), None if opt is None else ctypes.byref(opt), hip_stream,
                                 ctypes.byref(h)))
    return h


def pxServerSubmit(sv, h):
    _check(load().pxServerSubmit(sv, h))


def pxServerStep(sv, max_finished=64):
    arr = (_vp * max_finished)()
    n = ctypes.c_int32()
    _check(load().pxServerStep(sv, arr, max_finished, ctypes.byref(n)))
    return [arr[k] for k in range(n.value)]


def pxServerQuery(sv):
    q, a = ctypes.c_int32(), ctypes.c_int32()
    r, c = ctypes.c_int64(), ctypes.c_int64()
    _check(load().pxServerQuery(sv, ctypes.byref(q), ctypes.byref(a), ctypes.byref(r), ctypes.byref(c)))
    return dict(queued=q.value, active=a.value, rows_in_use=r.value, rows_capacity=c.value)


def pxServerMemory(sv):
    used, budget, nw = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _check(load().pxServerMemory(sv, ctypes.byref(used), ctypes.byref(budget), ctypes.byref(nw)))
    return dict(bytes_in_use=used.value, budget=budget.value, whole_solves=nw.value)


def pxSolveFootprint(h, opt: pxSolveOptions | None = None):
    b = ctypes.c_double()
    _check(load().pxSolveFootprint(h, None if opt is None else ctypes.byref(opt), ctypes.byref(b)))
    return b.value


def pxGetSolveStatus(h):
    st = ctypes.c_int32()
    buf = ctypes.create_string_buffer(512)
    _check(load().pxGetSolveStatus(h, ctypes.byref(st), buf, len(buf)))
    return st.value, buf.value.decode()


def pxServerDestroy(sv):
    if sv is not None:
        load().pxServerDestroy(sv)


# ---- convenience wrapper ---------------------------------------------------

def solve_batch(structures, **kw):
    """pxSolveBatch over Structure objects (keyword options as solve_options)."""
    return pxSolveBatch([st.h for st in structures], solve_options(**kw))


class Server:
    """Continuous-batching server (pxServerCreate ...)."""

    def __init__(self, memory_budget_bytes, hip_stream=None, **kw):
        self.h = pxServerCreate(memory_budget_bytes, solve_options(**kw), hip_stream)

    def submit(self, structure):
        pxServerSubmit(self.h, structure.h)

    def step(self, max_finished=64):
        return pxServerStep(self.h, max_finished)

    def query(self):
        return pxServerQuery(self.h)

    def memory(self):
        return pxServerMemory(self.h)

    def close(self):
        if self.h is not None:
            pxServerDestroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Structure:
    """One nanostructure on the GPU (see include/plasmonx.h).  With `types`
    and `params_b` it is a two-type structure (pxCreateStructureHetero); its
    alpha_ib arguments then hold (alpha_IB of A, alpha_IB of B) per frequency
    or column, shape (n, 2)."""

    def __init__(self, model, xyz_ang, params, hip_stream=None, types=None, params_b=None, mesh=None, eps_env=1.0,
                 bem_form="dpcm"):
        self.model = int(model)
        self.het = types is not None
        if self.model == PX_BEM:
            if bem_form not in ("dpcm", "iefpcm"):
                raise ValueError("bem_form is 'dpcm' or 'iefpcm'")
            create = pxCreateBemIefpcm if bem_form == "iefpcm" else pxCreateBem
            self.h = create(mesh, eps_env, hip_stream)
        elif self.het:
            self.h = pxCreateStructureHetero(model, xyz_ang, types, params, params_b, hip_stream)
        else:
            self.h = pxCreateStructure(model, xyz_ang, params, hip_stream)
        self.n, self.nu = pxGetSize(self.h)
        self.n_omega = 0
        self.ncol = 0

    @classmethod
    def bem(cls, mesh, eps_env=1.0, hip_stream=None, form="dpcm"):
        """A BEM structure on a mesh dict (workloads.mesh) in the DPCM or the
        IEFPCM form; its set_frequencies takes eps2(w) per frequency as
        alpha_ib."""
        return cls(PX_BEM, None, None, hip_stream, mesh=mesh, eps_env=eps_env, bem_form=form)

    def set_frequencies(self, omega_ev, pol_mask, e0_au=1e-4, alpha_ib=None):
        pxSetFrequencies(self.h, omega_ev, pol_mask, e0_au, alpha_ib)
        self.n_omega = len(np.atleast_1d(omega_ev))
        self.pol_mask = int(pol_mask)
        self.ncol = self.n_omega * bin(pol_mask & 7).count("1")

    def solve(self, **kw):
        return pxSolveSpectrum(self.h, solve_options(**kw))

    def solve_async(self, **kw):
        """Starts the solve (pxSolveSpectrumAsync); progress() advances it,
        wait() completes it."""
        return pxSolveSpectrumAsync(self.h, solve_options(**kw))

    def progress(self):
        return pxSolveProgress(self.h)

    def wait(self):
        return pxSolveWait(self.h)

    def spectrum(self):
        return pxGetSpectrum(self.h, self.n_omega)

    def charges(self, i_omega, pol, with_dipoles=False):
        return pxGetCharges(self.h, i_omega, pol, with_dipoles)

    def stats(self):
        return pxGetSolveStats(self.h, self.ncol)

    def status(self):
        """(status, message) of the last solve."""
        return pxGetSolveStatus(self.h)

    def footprint(self, **kw):
        return pxSolveFootprint(self.h, solve_options(**kw))

    def induced_field(self, i_omega, pol, pts):
        return pxInducedField(self.h, i_omega, pol, pts)

    def probe_field(self, q, mu, pts):
        return pxProbeField(self.h, q, mu, pts)

    def probe_stats(self):
        return pxGetProbeStats(self.h)

    def apply(self, precision, omega_ev, x, alpha_ib=None):
        return pxApplyOperator(self.h, precision, omega_ev, x, alpha_ib, self.het)

    def timings(self):
        return pxGetTimings(self.h)

    def work(self):
        return pxGetWork(self.h)

    def tapply_stats(self):
        return pxGetTApplyStats(self.h)

    def close(self):
        if self.h is not None:
            pxDestroyStructure(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
