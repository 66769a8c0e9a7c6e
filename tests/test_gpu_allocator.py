"""The library's device memory through the caller's allocator (pxSetAllocator):
torch's caching allocator counts what a structure and its solves hold, gets
all of it back at pxDestroyStructure, and the results do not depend on where
the memory came from.  An allocator that refuses turns into PX_E_OOM with
nothing left allocated."""
import sys

import numpy as np
import pytest

import paper_2510_12731_amd as px
from workloads import geometry as G
from workloads import materials as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def lib():
    import torch
    assert torch.cuda.is_available()
    return px.load()


AG = M.load("ag_wfq")
OM = np.linspace(3.0, 4.2, 12)


def _solve(xyz, **kw):
    s = px.Structure(0, xyz, AG, px.default_stream())
    s.set_frequencies(OM, 0b011)
    st = s.solve(rel_tol=1e-10, **kw)
    return s, st


@pytest.mark.parametrize("kw", [dict(precision=px.PX_FP64),
                                dict(precision=px.PX_MIXED, shifted=0, t_apply=px.PX_TAPPLY_STORED)],
                         ids=["shared_phase_fp64", "blocked_mixed_stored_T"])
def test_torch_allocator_holds_the_library_memory(kw):
    import torch
    xyz = G.fcc_sphere_n(1500, seed=4)
    ref, st = _solve(xyz, **kw)
    assert st == px.PX_OK
    sig_ref = ref.spectrum()[1]
    ref.close()
    px.use_torch_allocator()
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        s = px.Structure(0, xyz, AG, px.default_stream())
        held = torch.cuda.memory_allocated() - base
        s.set_frequencies(OM, 0b011)
        torch.cuda.reset_peak_memory_stats()
        st = s.solve(rel_tol=1e-10, **kw)
        peak = torch.cuda.max_memory_allocated() - base
        sig = s.spectrum()[1]
        say(f"[allocator {kw}] structure {held / 2**20:.1f} MiB, peak in the solve {peak / 2**20:.1f} MiB")
        assert st == px.PX_OK
        assert held > 0 and peak > held
        # same kernels on the same inputs wherever the memory lives
        e = float(np.max(np.abs(sig - sig_ref)) / np.max(np.abs(sig_ref)))
        say(f"   sigma vs the hipMalloc run: {e:.1e}")
        assert e <= 1e-12
        s.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        px.use_hip_allocator()


def test_refusing_allocator_gives_oom_and_leaks_nothing():
    """A budgeted allocator over torch's: too small for the structure ->
    PX_E_OOM from pxCreateStructure and every block given back; large enough
    for the structure but not for the solve -> PX_E_OOM from the solve, the
    structure still usable once the budget grows."""
    import torch
    state = dict(limit=0, used=0, sizes={})

    def alloc(nbytes, device, user):
        if state["used"] + nbytes > state["limit"]:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), int(device))
        state["used"] += nbytes
        state["sizes"][p] = nbytes
        return p

    def free(ptr, device, user):
        state["used"] -= state["sizes"].pop(ptr)
        torch.cuda.caching_allocator_delete(int(ptr))

    xyz = G.fcc_sphere_n(1500, seed=4)
    px.pxSetAllocator(px.ALLOC_FN(alloc), px.FREE_FN(free))
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        state["limit"] = 64 << 10
        with pytest.raises(px.PxError) as e:
            px.Structure(0, xyz, AG, px.default_stream())
        assert e.value.status == px.PX_E_OOM
        assert state["used"] == 0 and torch.cuda.memory_allocated() == base
        state["limit"] = 1 << 40
        s = px.Structure(0, xyz, AG, px.default_stream())
        s.set_frequencies(OM, 0b011)
        state["limit"] = state["used"] + (64 << 10)
        with pytest.raises(px.PxError) as e:
            s.solve(precision=px.PX_FP64, rel_tol=1e-10)
        assert e.value.status == px.PX_E_OOM
        say(f"[allocator budget] solve refused at {state['used'] / 2**20:.1f} MiB in use")
        state["limit"] = 1 << 40
        assert s.solve(precision=px.PX_FP64, rel_tol=1e-10) == px.PX_OK
        s.close()
        torch.cuda.synchronize()
        assert state["used"] == 0 and torch.cuda.memory_allocated() == base
    finally:
        px.use_hip_allocator()


@pytest.mark.parametrize("what", ["wfq_block_phase", "bem_iefpcm_block_phase"])
def test_solve_footprint_bounds_the_solve_peak(what):
    """pxSolveFootprint (the server's admission figure) is at least what a
    solve takes from the caller's allocator at its peak: the omegaFQ block
    phase, and the IEFPCM block phase whose true residuals go through its
    basis (the buffers of that route included)."""
    import torch
    from workloads import mesh as ME
    if what.startswith("wfq"):
        make = lambda: px.Structure(0, G.fcc_sphere_n(1500, seed=4), AG, px.default_stream())
        om, extra = OM, None
    else:
        m = ME.sphere(40.0, 3)
        make = lambda: px.Structure.bem(m, 1.0, px.default_stream(), form="iefpcm")
        om = np.linspace(3.0, 4.4, 48)
        extra = M.drude_permittivity(M.load("ag_bem"), om)
    px.use_torch_allocator()
    try:
        s = make()
        s.set_frequencies(om, 0b111, 1e-4, extra)
        fp = s.footprint(precision=px.PX_FP64, rel_tol=1e-10)
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        assert s.solve(precision=px.PX_FP64, rel_tol=1e-10) == px.PX_OK
        peak = torch.cuda.max_memory_allocated() - base
        say(f"[footprint {what}] solve peak {peak / 2**20:.1f} MiB, footprint {fp / 2**20:.1f} MiB")
        assert 0 < peak <= fp
        s.close()
    finally:
        px.use_hip_allocator()
