"""Truncated-Newton polish of relax_subdomains (Sec. II.C step 4; Newton steps
solved by CG on the tangent-space Hessian through Hessian-vector products)
against the CPU oracle.

Every Newton-polished endpoint is re-checked by the oracle (E_sub to 1e-13,
the reduced gradient below the tolerance, the exact energy change, held
charges pushed outward); from a common near-minimum start the GPU's Newton
endpoints and the oracle's own Newton-CG relax reach the same minimum (E_sub
to 1e-12 relative, positions within 1e-3 h); Newton forced from rough starts
(indefinite Hessians: CG stops at negative curvature, failed line searches
fall back to L-BFGS) still ends in oracle-checked minima; and the rounds
replayed from HIP graphs match one-by-one launches bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_24722_amd import FP64, MIXED, workloads as W
from paper_2609_24722_amd import relax as R
from test_gpu_relax import check_endpoints, t

pytestmark = pytest.mark.gpu

ALWAYS = 1e300  # newton_tol that puts every patch in Newton mode from its start


def near_minimum_start(x, y, ptr, idx, dev, gtol, seed, h):
    base = R.relax_subdomains(t(x, dev), t(y, dev), ptr, idx, precision=FP64, gtol=gtol,
                              polish=R.POLISH_LBFGS)
    rng = np.random.default_rng(seed)
    n = int(ptr[-1])
    sx = base.x.cpu().numpy() + rng.normal(0, 1e-3 * h, n)
    sy = base.y.cpu().numpy() + rng.normal(0, 1e-3 * h, n)
    rr = np.hypot(sx, sy)
    return np.where(rr > 1, sx / rr, sx), np.where(rr > 1, sy / rr, sy)


@pytest.mark.parametrize("prec", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("switch", ["default", "always"])
def test_newton_endpoints_small_batch(dev, prec, switch):
    # patches of 1 to 400 actives (ragged against the 64-active blocks and the
    # 1024-thread update), warped lattice sigma 0.1 h, start = snapshot
    x, y = W.warped_lattice(3000, 0.1, 7)
    centres, _ = W.patch_draws(3000, 6, 10, 20, 8)
    sizes = np.array([1, 37, 64, 65, 200, 400], dtype=np.int32)
    xt, yt = t(x, dev), t(y, dev)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    kw = dict(newton_tol=ALWAYS) if switch == "always" else {}
    print(f"[case] newton small batch prec={prec} switch={switch}", flush=True)
    res = R.relax_subdomains(xt, yt, ptr, idx, precision=prec, gtol=1e-6,
                             polish=R.POLISH_NEWTON, **kw)
    torch.cuda.synchronize()
    ps = res.polish.cpu().numpy()
    print(f"[newton] steps={ps[:, 0]} cg={ps[:, 1]} iters={res.iters.cpu().numpy()[:, 0]}")
    check_endpoints(x, y, ptr, idx.cpu().numpy(), res, 1e-6, f"newton-{prec}-{switch}")
    # the polish ran: every patch of more than one charge took Newton steps
    assert (ps[1:, 0] > 0).all() and (ps[1:, 1] > 0).all()


def test_newton_same_basin_as_oracle_newton(dev):
    # from a common near-minimum start, Newton from the first iteration on the
    # GPU (both paths) and in the oracle's relax: the same minimum
    n = 20000
    x, y = W.warped_lattice(n, 0.05, 11)
    h = W.spacing(n)
    centres, sizes = W.patch_draws(n, 8, 150, 800, 12)
    xt, yt = t(x, dev), t(y, dev)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    idx_np = idx.cpu().numpy()
    print("[case] newton same basin", flush=True)
    sx, sy = near_minimum_start(x, y, ptr, idx, dev, 1e-6, 13, h)
    res = {prec: R.relax_subdomains(xt, yt, ptr, idx, t(sx, dev), t(sy, dev), precision=prec,
                                    gtol=1e-6, polish=R.POLISH_NEWTON, newton_tol=ALWAYS)
           for prec in (FP64, MIXED)}
    torch.cuda.synchronize()
    for prec in (FP64, MIXED):
        check_endpoints(x, y, ptr, idx_np, res[prec], 1e-6, f"newton-basin-{prec}")
        assert (res[prec].polish.cpu().numpy()[:, 0] > 0).all()
    for p in range(ptr.size - 1):
        sl = slice(ptr[p], ptr[p + 1])
        xo, yo, st = O.relax(x, y, idx_np[sl], sx[sl], sy[sl], gtol=1e-6, newton_tol=ALWAYS)
        Eo = O.esub(x, y, idx_np[sl], xo, yo)
        assert st["newton_steps"] > 0
        for prec in (FP64, MIXED):
            e = res[prec].e_sub.cpu().numpy()[p]
            d = np.hypot(res[prec].x.cpu().numpy()[sl] - xo, res[prec].y.cpu().numpy()[sl] - yo).max()
            print(f"[newton-basin] p{p} prec={prec} gpu={e:.15e} oracle-newton={Eo:.15e} disp={d / h:.1e} h")
            assert abs(e - Eo) <= 1e-12 * abs(Eo)
            assert d <= 1e-3 * h


@pytest.mark.parametrize("prec", [FP64, MIXED], ids=["fp64", "mixed"])
def test_newton_from_kicked_starts(dev, prec):
    # kicks of 0.3 h (config 5): Newton forced from the start meets indefinite
    # Hessians (CG stops at negative curvature; line searches that fail fall
    # back to L-BFGS), and the endpoints still pass the oracle's checks
    n = 40000
    x, y = W.workload(5, n)
    h = W.spacing(n)
    centres, sizes = W.patch_draws(n, 8, 200, 900, 1105)
    xt, yt = t(x, dev), t(y, dev)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    idx_np = idx.cpu().numpy()
    kx, ky = W.kicks(idx_np.size, 0.3 * h, 2105)
    print(f"[case] newton kicked prec={prec}", flush=True)
    res = R.relax_subdomains(xt, yt, ptr, idx, t(x[idx_np] + kx, dev), t(y[idx_np] + ky, dev),
                             precision=prec, gtol=1e-3, polish=R.POLISH_NEWTON, newton_tol=ALWAYS)
    torch.cuda.synchronize()
    print(f"[newton-kicked] polish={res.polish.cpu().numpy().tolist()}")
    check_endpoints(x, y, ptr, idx_np, res, 1e-3, f"newton-kicked-{prec}")


@pytest.mark.parametrize("prec", [FP64, MIXED], ids=["fp64", "mixed"])
def test_newton_graph_rounds_match_plain_launches(dev, prec):
    """Newton rounds (Hessian products, CG updates, line searches) replayed from
    captured HIP graphs equal the same kernels launched one by one, bit for
    bit, over three calls in a row."""
    x, y = W.warped_lattice(3000, 0.1, 17)
    centres, _ = W.patch_draws(3000, 6, 10, 20, 18)
    sizes = np.array([1, 50, 64, 130, 300, 700], dtype=np.int32)
    xt, yt = t(x, dev), t(y, dev)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    fields = ("x", "y", "dE", "e_sub", "gtan_inf", "iters", "status", "polish")
    runs = []
    for launch in (R.LAUNCH_GRAPH, R.LAUNCH_PLAIN, R.LAUNCH_GRAPH):
        res = R.relax_subdomains(xt, yt, ptr, idx, precision=prec, gtol=1e-6,
                                 polish=R.POLISH_NEWTON, newton_tol=ALWAYS, launch=launch)
        torch.cuda.synchronize()
        runs.append([getattr(res, f).clone() for f in fields])
    for a, b, c, f in zip(*runs, fields):
        assert torch.equal(a, b) and torch.equal(a, c), f
    assert (runs[0][6] == 0).all() and (runs[0][7][1:, 0] > 0).all()
