"""The allocation-free forces entry point (coulomb_forces_noalloc) against
coulomb_forces through the C ABI: two calls in a row on each path, the
second smaller, and the CD_MIXED call at N = 1e5, whose partial sums are
batched to fit the fixed scratch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_24722_amd import FP64, MIXED, ops, workloads as W

pytestmark = pytest.mark.gpu

_vp = ctypes.c_void_p


def _noalloc():
    L = ops.lib()
    f = L.coulomb_forces_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp]
    return f


def _call(x, y, prec):
    n = x.numel()
    fx = torch.full((n,), float("nan"), dtype=torch.float64, device=x.device)
    fy = torch.full((n,), float("nan"), dtype=torch.float64, device=x.device)
    E = torch.full((1,), float("nan"), dtype=torch.float64, device=x.device)
    print(f"coulomb_forces_noalloc n={n} precision={prec}", flush=True)
    rc = _noalloc()(x.data_ptr(), y.data_ptr(), n, prec, fx.data_ptr(), fy.data_ptr(),
                    E.data_ptr(), ops.stream_ptr(x.device))
    assert rc == 0, ops.lib().coulomb_status_string(rc)
    torch.cuda.synchronize()
    return fx.cpu().numpy(), fy.cpu().numpy(), E.item()


def _rel_rms(ax, ay, bx, by):
    return np.sqrt(np.sum((ax - bx) ** 2 + (ay - by) ** 2) / np.sum(bx ** 2 + by ** 2))


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_noalloc_matches_forces_two_calls(dev, prec):
    # first call large (N = 1e5: on CD_MIXED its partial sums exceed the fixed
    # scratch and run in batches), second smaller, ragged (N = 4097)
    for n, seed in ((100000, 1003), (4097, 1001)):
        if n == 100000:
            x, y = W.warped_lattice(n, 0.02, seed)
        else:
            x, y = W.uniform_disk(n, seed)
        xt = torch.tensor(x, device=dev)
        yt = torch.tensor(y, device=dev)
        fx, fy, E = _call(xt, yt, prec)
        gx, gy, gE = ops.forces(xt, yt, prec)
        torch.cuda.synchronize()
        gx, gy, gE = gx.cpu().numpy(), gy.cpu().numpy(), gE.item()
        assert np.all(np.isfinite(fx)) and np.all(np.isfinite(fy))
        if prec == FP64 or n < 20000:
            # the same plan as coulomb_forces: identical results
            assert np.array_equal(fx, gx) and np.array_equal(fy, gy) and E == gE
        else:
            # batched reductions sum the same partials in another order
            assert _rel_rms(fx, fy, gx, gy) <= 1e-13
            assert abs(E - gE) <= 1e-14 * abs(gE)
        if n <= 5000:
            ox, oy = O.forces(x, y)
            oE = O.energy(x, y)
            ftol, etol = (1e-11, 1e-13) if prec == FP64 else (1e-5, 1e-7)
            assert _rel_rms(fx, fy, ox, oy) <= ftol
            assert abs(E - oE) <= etol * oE


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_noalloc_smallest_sizes(dev, prec):
    # one charge (no pair: zero force and energy), two, and one ragged block
    for n in (1, 2, 65):
        x, y = W.uniform_disk(n, 2000 + n)
        xt = torch.tensor(x, device=dev)
        yt = torch.tensor(y, device=dev)
        fx, fy, E = _call(xt, yt, prec)
        if n == 1:
            assert fx[0] == 0.0 and fy[0] == 0.0 and E == 0.0
            continue
        ox, oy = O.forces(x, y)
        oE = O.energy(x, y)
        ftol, etol = (1e-11, 1e-13) if prec == FP64 else (1e-5, 1e-7)
        assert _rel_rms(fx, fy, ox, oy) <= ftol and abs(E - oE) <= etol * oE


def test_noalloc_refuses_sizes_beyond_scratch(dev):
    x = torch.zeros(1, dtype=torch.float64, device=dev)
    rc = _noalloc()(x.data_ptr(), x.data_ptr(), 706305, MIXED, x.data_ptr(), x.data_ptr(), None,
                    ops.stream_ptr(dev))
    assert rc == -6
