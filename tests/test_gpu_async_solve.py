"""pxSolveSpectrumAsync / pxSolveProgress / pxSolveWait: a solve started
without waiting returns before the spectrum is solved, advances in later
calls, and gives the spectrum of the synchronous solve bit for bit (the same
launches in the same order); any other call on the structure first completes
it, and destroying the structure abandons it safely."""
import sys
import time

import numpy as np
import pytest

import paper_2510_12731_amd as px
from workloads import geometry as G
from workloads import materials as M
from workloads import mesh as ME

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def lib():
    import torch
    assert torch.cuda.is_available()
    return px.load()


AG = M.load("ag_wfq")
OM = np.linspace(3.0, 4.2, 48)


def make(xyz):
    s = px.Structure(0, xyz, AG, px.default_stream())
    s.set_frequencies(OM, 0b111)
    return s


def test_async_solve_matches_the_synchronous_one():
    import torch
    xyz = G.fcc_sphere_n(6000, seed=5)
    ref = make(xyz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assert ref.solve(precision=px.PX_FP64, rel_tol=1e-10) == px.PX_OK
    t_sync = time.perf_counter() - t0
    alpha_ref, sigma_ref = ref.spectrum()
    it_ref = ref.stats()[0]
    ref.close()

    s = make(xyz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.solve_async(precision=px.PX_FP64, rel_tol=1e-10)
    t_call = time.perf_counter() - t0
    polls = 0
    while not s.progress():
        polls += 1
    t_all = time.perf_counter() - t0
    say(f"[async] 6000 atoms x 144 columns: synchronous {t_sync * 1e3:.1f} ms; async call returned after "
        f"{t_call * 1e3:.1f} ms, done after {polls} polls, {t_all * 1e3:.1f} ms")
    assert polls >= 1 and t_call < 0.5 * t_sync
    assert s.wait() == px.PX_OK
    assert s.status()[0] == px.PX_OK
    alpha, sigma = s.spectrum()
    assert np.array_equal(sigma, sigma_ref) and np.array_equal(alpha, alpha_ref)
    assert np.array_equal(s.stats()[0], it_ref)
    s.close()


def test_other_calls_complete_an_async_solve_first():
    xyz = G.fcc_sphere_n(3000, seed=6)
    ref = make(xyz)
    assert ref.solve(precision=px.PX_FP64, rel_tol=1e-10) == px.PX_OK
    sigma_ref = ref.spectrum()[1]
    ref.close()
    # a read completes the solve
    s = make(xyz)
    s.solve_async(precision=px.PX_FP64, rel_tol=1e-10)
    assert np.array_equal(s.spectrum()[1], sigma_ref)
    assert s.progress()
    # new frequencies complete it, then discard its results
    s.solve_async(precision=px.PX_FP64, rel_tol=1e-10)
    s.set_frequencies(OM[:8], 0b001)
    with pytest.raises(px.PxError) as e:
        s.spectrum()
    assert e.value.status == px.PX_E_STATE
    # a second solve after the first one's frequencies were replaced
    s.solve_async(precision=px.PX_FP64, rel_tol=1e-10)
    assert s.wait() == px.PX_OK
    s.close()
    # destroyed while in progress, then the library goes on
    d = make(xyz)
    d.solve_async(precision=px.PX_FP64, rel_tol=1e-10)
    d.close()
    again = make(xyz)
    assert again.solve(precision=px.PX_FP64, rel_tol=1e-10) == px.PX_OK
    assert np.array_equal(again.spectrum()[1], sigma_ref)
    again.close()


def test_async_bem_solve_and_argument_errors():
    m = ME.sphere(30.0, 2)
    om = np.linspace(3.0, 4.5, 24)
    eps = M.drude_permittivity(M.load("ag_bem"), om)
    ref = px.Structure.bem(m, 1.0, px.default_stream(), form="iefpcm")
    ref.set_frequencies(om, 0b111, 1e-4, eps)
    assert ref.solve(precision=px.PX_FP64, rel_tol=1e-12) == px.PX_OK
    s = px.Structure.bem(m, 1.0, px.default_stream(), form="iefpcm")
    s.set_frequencies(om, 0b111, 1e-4, eps)
    s.solve_async(precision=px.PX_FP64, rel_tol=1e-12)
    assert s.wait() == px.PX_OK
    assert np.array_equal(s.spectrum()[1], ref.spectrum()[1])
    assert np.array_equal(s.charges(3, 1), ref.charges(3, 1))
    ref.close()
    s.close()
    fresh = px.Structure(0, G.fcc_sphere_n(300, seed=2), AG, px.default_stream())
    with pytest.raises(px.PxError) as e:                       # no frequencies yet
        fresh.solve_async()
    assert e.value.status == px.PX_E_STATE
    assert fresh.progress()                                    # nothing in progress
    fresh.set_frequencies(OM[:4], 0b001)
    with pytest.raises(px.PxError) as e:                       # invalid options
        fresh.solve_async(rel_tol=-1.0)
    assert e.value.status == px.PX_E_INVALID
    fresh.close()
