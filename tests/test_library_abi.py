"""The C-ABI library builds for gfx950, loads, exports every declared entry
point, agrees with the binding on struct layouts, and validates arguments on
the host before touching a device (no compute call is made here)."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2510_12731_amd as px

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plasmonx.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(px.LIB_PATH):
        from paper_2510_12731_amd import build
        build.build(verbose=False)
    return px.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(px[A-Z]\w*)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(px.EXPORTED) == names


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "plasmonx.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(pxMaterial), sizeof(pxSolveOptions),'
                   ' offsetof(pxSolveOptions, inner_reduction), offsetof(pxSolveOptions, timings));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert int(out[0]) == ctypes.sizeof(px.pxMaterial)
    assert int(out[1]) == ctypes.sizeof(px.pxSolveOptions)
    assert int(out[2]) == px.pxSolveOptions.inner_reduction.offset
    assert int(out[3]) == px.pxSolveOptions.timings.offset


def test_default_options(lib):
    o = px.pxDefaultSolveOptions()
    assert (o.precision, o.restart_m, o.rel_tol, o.max_cycles, o.max_block_cols) == (px.PX_FP64, 100, 1e-8, 400, 0)
    assert o.shifted == 2 and o.shifted_max_steps == 2000
    assert o.inner_reduction == 1e-5 and o.timings == 0 and o.stall_cycles == 8
    assert o.max_restart_m == 200 and o.block_cols == 0 and o.ortho == px.PX_ORTHO_DCGS2 and o.graph_steps == 8 and o.t_apply == px.PX_TAPPLY_AUTO


def test_set_allocator_argument_errors(lib):
    """alloc and free come together; NULL/NULL restores hipMalloc (no device
    call is made)."""
    a = px.ALLOC_FN(lambda n, d, u: None)
    assert lib.pxSetAllocator(a, px.FREE_FN(), None) == px.PX_E_INVALID
    assert b"both" in lib.pxLastError()
    assert lib.pxSetAllocator(px.ALLOC_FN(), px.FREE_FN(lambda p, d, u: None), None) == px.PX_E_INVALID
    assert lib.pxSetAllocator(px.ALLOC_FN(), px.FREE_FN(), None) == px.PX_OK
    assert lib.pxReleaseCache() == px.PX_OK


def _mat():
    from workloads import materials as M
    return px.material(M.load("ag_wfq"))


@pytest.mark.parametrize("case", ["empty", "nan", "inf", "bad_model", "bad_tau", "bad_area", "bad_rmu_dipole"])
def test_invalid_inputs_rejected_on_host(lib, case):
    xyz = np.zeros((3, 3))
    xyz[1, 0] = 2.9
    xyz[2, 1] = 2.9
    m = _mat()
    model, n = px.PX_WFQ, 3
    if case == "empty":
        n = 0
    elif case == "nan":
        xyz[1, 2] = math.nan
    elif case == "inf":
        xyz[0, 0] = math.inf
    elif case == "bad_model":
        model = 7
    elif case == "bad_tau":
        m.tau = 0.0
    elif case == "bad_area":
        m.a_eff = -1.0
    elif case == "bad_rmu_dipole":
        model = px.PX_WFQFMU
        m.r_mu = 0.0
    h = ctypes.c_void_p()
    xp = np.ascontiguousarray(xyz)
    st = lib.pxCreateStructure(model, n, xp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(m), None,
                               ctypes.byref(h))
    assert st == px.PX_E_INVALID
    assert h.value is None
    assert len(px.pxLastError()) > 0


def test_null_handles_rejected(lib):
    assert lib.pxSolveSpectrum(None, None) == px.PX_E_INVALID
    assert lib.pxGetSpectrum(None, None, None) == px.PX_E_INVALID
    assert lib.pxGetSize(None, None, None) == px.PX_E_INVALID
    lib.pxDestroyStructure(None)


@pytest.mark.parametrize("case", ["null_types", "null_mat_b", "bad_type", "r_q_differs", "r_mu_differs",
                                  "bad_tau_b"])
def test_invalid_two_type_inputs_rejected_on_host(lib, case):
    from workloads import materials as M
    xyz = np.zeros((3, 3))
    xyz[1, 0] = 2.9
    xyz[2, 1] = 2.9
    ma, mb = px.material(M.load("ag_wfqfmu")), px.material(M.load("au_wfqfmu"))
    types = np.array([0, 1, 0], dtype=np.uint8)
    model = px.PX_WFQFMU
    tp = types.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    mbp = ctypes.byref(mb)
    if case == "null_types":
        tp = None
    elif case == "null_mat_b":
        mbp = None
    elif case == "bad_type":
        types[2] = 2
    elif case == "r_q_differs":
        mb.r_q = 1.01 * ma.r_q
    elif case == "r_mu_differs":
        mb.r_mu = 0.9 * ma.r_mu
    elif case == "bad_tau_b":
        mb.tau = -1.0
    h = ctypes.c_void_p()
    xp = np.ascontiguousarray(xyz)
    st = lib.pxCreateStructureHetero(model, 3, xp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), tp,
                                     ctypes.byref(ma), mbp, None, ctypes.byref(h))
    assert st == px.PX_E_INVALID
    assert h.value is None
    assert len(px.pxLastError()) > 0


def test_probe_rejections_on_host(lib):
    """Invalid probe calls fail on the host before any GPU work."""
    assert lib.pxInducedField(None, 0, 0, 0, None, None, None) == px.PX_E_INVALID
    assert lib.pxProbeField(None, None, None, 0, None, None, None) == px.PX_E_INVALID
    assert lib.pxGetProbeStats(None, None) == px.PX_E_INVALID
