"""The entry point that allocates nothing (pxApplyOperatorNoAlloc) against the
one it is a variant of (pxApplyOperator, FP64) and against the oracle.

Bars: against pxApplyOperator max|dy| <= 1e-12 max|y| (the same kernels on
the same inputs); against the oracle max|dy| <= 1e-11 max|y| (the FP64
operator-apply bound of the parity tests).  Two calls in a row, the second
with a smaller input, so that a value left in the shared scratch array by
the first call would show in the second; then a structure whose scratch
exceeds the fixed array is refused with PX_E_OOM, and a later call still
works.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2510_12731_amd as px
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


def no_alloc_apply(s, om, x, aib=None):
    """x [ncol, nu] complex on the host -> device tensors -> the entry point."""
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x).view(np.float64).copy()).to("cuda")
    yd = torch.full_like(xd, float("nan"))
    torch.cuda.synchronize()
    px.pxApplyOperatorNoAlloc(s.h, om, xd.data_ptr(), yd.data_ptr(), aib)
    return yd.cpu().numpy().view(np.complex128).reshape(x.shape)


def case(model, n, ncol, seed):
    params = M.load("ag_wfq" if model == 0 else "au_wfqfmu")
    xyz = G.fcc_sphere_n(n, seed=seed) if model == 0 else G.fcc_rod_n(n, seed=seed)
    nu = 4 * n if model else n
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((ncol, nu)) + 1j * rng.standard_normal((ncol, nu))
    om = np.linspace(1.7, 4.3, ncol)
    aib = M.interband_alpha(params, om) if model else None
    return params, xyz, x, om, aib


@pytest.mark.parametrize("model,sizes", [(0, ((1000, 4), (300, 1))), (1, ((700, 3), (240, 2)))])
def test_no_alloc_apply_matches_the_allocating_entry_point(model, sizes):
    for k, (n, ncol) in enumerate(sizes):
        params, xyz, x, om, aib = case(model, n, ncol, seed=50 + 7 * k + model)
        say(f"[no-alloc] call {k + 1}: model={model} n={n} ncol={ncol}")
        s = px.Structure(model, xyz, params, px.default_stream())
        y0 = no_alloc_apply(s, om, x, aib)
        y1 = s.apply(px.PX_FP64, om, x, aib)
        ref = O.apply(model, xyz, M.param_vector(params), om, x, aib)
        e1, e_ref = rel_err(y0, y1), rel_err(y0, ref)
        say(f"   vs pxApplyOperator {e1:.1e}, vs oracle {e_ref:.1e}")
        assert np.all(np.isfinite(y0))
        assert e1 <= 1e-12 and e_ref <= 1e-11
        s.close()


def test_no_alloc_refuses_more_than_its_array_and_keeps_working():
    au = M.load("au_wfqfmu")
    big = px.Structure(1, G.fcc_sphere_n(20000, seed=61), au, px.default_stream())
    om = np.linspace(2.0, 3.0, 4)
    aib = M.interband_alpha(au, om)
    import torch
    xd = torch.zeros(4 * 4 * 20000 * 2, dtype=torch.float64, device="cuda")
    yd = torch.zeros_like(xd)
    with pytest.raises(px.PxError) as e:
        px.pxApplyOperatorNoAlloc(big.h, om, xd.data_ptr(), yd.data_ptr(), aib)
    say(f"[no-alloc] refused: {e.value}")
    assert e.value.status == px.PX_E_OOM and "bytes of scratch" in str(e.value)
    big.close()
    params, xyz, x, om, aib = case(0, 500, 2, seed=62)
    s = px.Structure(0, xyz, params, px.default_stream())
    assert rel_err(no_alloc_apply(s, om, x), s.apply(px.PX_FP64, om, x)) <= 1e-12
    s.close()
