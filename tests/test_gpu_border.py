"""Border-interior split on the GPU (Sec. II.B) against the oracle: the
boundary split bit-exact, relaxations under pinned boundary charges and an
interior wall reaching closed-form minima, and same-basin energy parity with
the oracle's own border-interior relax on patches that touch the boundary."""
import math

import mpmath
import numpy as np
import pytest
import torch

import oracle as O
from oracle import border as OB
from paper_2609_24722_amd import FP64, MIXED, border as B, workloads as W
from paper_2609_24722_amd import relax as R

pytestmark = pytest.mark.gpu


def t(a, dev, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), device=dev, dtype=dtype)


def ngon_energy(n):
    mpmath.mp.dps = 40
    return float(mpmath.mpf(n) / 2 * mpmath.fsum(1 / (2 * mpmath.sin(mpmath.pi * k / n)) for k in range(1, n)))


def check_endpoints_bi(x, y, ptr, idx_np, res, gtol, flags, sigma, label):
    xo, yo = res.x.cpu().numpy(), res.y.cpu().numpy()
    es, gt, st = res.e_sub.cpu().numpy(), res.gtan_inf.cpu().numpy(), res.status.cpu().numpy()
    for p in range(ptr.size - 1):
        sl = slice(ptr[p], ptr[p + 1])
        ip = idx_np[sl]
        pin = flags[ip]
        Eo, gx, gy = O.esub(x, y, ip, xo[sl], yo[sl], grad=True)
        _, _, held, m = O.reduce_grad(xo[sl], yo[sl], gx, gy, pin=pin, sigma=sigma)
        r = np.hypot(xo[sl], yo[sl])
        print(f"[{label}] p{p} n={ip.size} pinned={pin.sum()} status={st[p]} gtan={gt[p]:.2e} "
              f"oracle gtan={m:.2e} E_sub rel={abs(es[p] - Eo) / Eo:.1e}", flush=True)
        assert st[p] == 0 and gt[p] <= gtol
        assert m <= 1.01 * gtol + 1e-12
        assert abs(es[p] - Eo) <= 1e-13 * Eo
        assert np.all(np.abs(r[pin == 1] - 1.0) <= 1e-15)
        assert np.all(r[pin == 0] <= sigma * (1 + 1e-15))
        wall = (pin == 0) & (held == 1)
        if wall.any():  # interior charges held by the wall are pushed outward
            assert np.all(-(gx * xo[sl] + gy * yo[sl])[wall] > 0)


def test_border_split_bit_exact(dev):
    n = 20000
    x, y = W.warped_lattice(n, 0.05, 1102)
    # exact ties in x*x + y*y at the cut and elsewhere
    x[100], y[100] = 0.6, 0.8
    x[200], y[200] = 0.8, 0.6
    x[300], y[300] = -0.6, 0.8
    xt, yt = t(x, dev), t(y, dev)
    r2 = x * x + y * y
    order = np.lexsort((np.arange(n), -r2))
    k_tie = int(np.nonzero(order == 200)[0][0])  # put the cut inside the tie group
    for nb in (0, 1, B.boundary_count(n), k_tie, k_tie + 1, n - 1, n):
        f = B.border_split(xt, yt, nb).cpu().numpy()
        assert np.array_equal(f, OB.border_split(x, y, nb)), nb


def _one_patch(n, dev):
    ptr = np.array([0, n], dtype=np.int32)
    return ptr, t(np.arange(n, dtype=np.int32), dev)


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_relax_bi_closed_forms(dev, prec):
    """Six pinned charges around one interior charge (sigma = 0.5): hexagon
    plus centre, E = E_6 + 6.  Three interior charges (sigma = 0.5): an
    equilateral triangle on the sigma circle, E = sqrt(3)/sigma.  Nine pinned
    charges: the regular 9-gon."""
    cases = []
    a = np.arange(6) * (2 * np.pi / 6) + np.array([0.1, -0.05, 0.08, 0.0, -0.1, 0.03])
    cases.append((np.append(0.9 * np.cos(a), 0.2), np.append(0.9 * np.sin(a), -0.1),
                  np.array([1] * 6 + [0], np.int32), 0.5, ngon_energy(6) + 6.0))
    cases.append((np.array([0.1, -0.2, 0.05]), np.array([0.1, 0.0, -0.3]), np.zeros(3, np.int32), 0.5,
                  math.sqrt(3.0) / 0.5))
    a = np.sort(np.random.default_rng(9).uniform(0, 2 * np.pi, 9))
    cases.append((0.7 * np.cos(a), 0.7 * np.sin(a), np.ones(9, np.int32), 0.3, ngon_energy(9)))
    for x, y, pin, sigma, E in cases:
        n = x.size
        xt, yt = t(x, dev), t(y, dev)
        ptr, idx = _one_patch(n, dev)
        print(f"[case] closed form n={n} sigma={sigma} prec={prec}", flush=True)
        res = R.relax_subdomains(xt, yt, ptr, idx, precision=prec, gtol=1e-9, sigma=sigma,
                                 boundary=t(pin, dev, torch.int32))
        assert res.status.cpu().numpy()[0] == 0
        xo, yo = res.x.cpu().numpy(), res.y.cpu().numpy()
        assert abs(O.energy(xo, yo) - E) <= 1e-12 * E
        assert abs(res.e_sub.cpu().numpy()[0] - E) <= 1e-12 * E
        check_endpoints_bi(x, y, ptr, np.arange(n), res, 1e-9, pin, sigma, f"closed-{prec}")


def test_relax_bi_same_basin(dev):
    """Patches of the N = 20000 lattice that contain boundary charges, with
    N_b of Eq. 4 pinned and the interior wall at sigma0 of Eq. 5: from a common
    near-minimum start both GPU paths and the oracle's border-interior relax
    reach the same minimum (E_sub to 1e-12)."""
    n = 20000
    x, y = W.warped_lattice(n, 0.05, 31)
    h = W.spacing(n)
    nb = B.boundary_count(n)
    sigma = B.sigma0(n)
    xt, yt = t(x, dev), t(y, dev)
    flags_t = B.border_split(xt, yt, nb)
    flags = flags_t.cpu().numpy()
    far = np.argsort(-(x * x + y * y), kind="stable")
    centres = np.array([far[0], far[5000 % n], 123], dtype=np.int32)  # two at the edge, one inside
    sizes = np.array([400, 250, 300], dtype=np.int32)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    idx_np = idx.cpu().numpy()
    print(f"[case] bi same basin nb={nb} sigma={sigma} pinned per patch "
          f"{[int(flags[idx_np[ptr[p]:ptr[p + 1]]].sum()) for p in range(3)]}", flush=True)
    base = R.relax_subdomains(xt, yt, ptr, idx, precision=FP64, gtol=1e-5, sigma=sigma, boundary=flags_t)
    rng = np.random.default_rng(32)
    sx = base.x.cpu().numpy() + rng.normal(0, 1e-3 * h, idx_np.size)
    sy = base.y.cpu().numpy() + rng.normal(0, 1e-3 * h, idx_np.size)
    res = {prec: R.relax_subdomains(xt, yt, ptr, idx, t(sx, dev), t(sy, dev), precision=prec, gtol=1e-6,
                                    sigma=sigma, boundary=flags_t) for prec in (FP64, MIXED)}
    torch.cuda.synchronize()
    for prec in (FP64, MIXED):
        check_endpoints_bi(x, y, ptr, idx_np, res[prec], 1e-6, flags, sigma, f"bi-basin-{prec}")
    e64, e32 = res[FP64].e_sub.cpu().numpy(), res[MIXED].e_sub.cpu().numpy()
    for p in range(ptr.size - 1):
        sl = slice(ptr[p], ptr[p + 1])
        pin = flags[idx_np[sl]]
        xo, yo, st = O.relax(x, y, idx_np[sl], sx[sl], sy[sl], gtol=1e-6, pin=pin, sigma=sigma)
        Eo = O.esub(x, y, idx_np[sl], xo, yo)
        print(f"[bi-basin] p{p} plain={e64[p]:.15e} mixed={e32[p]:.15e} oracle-relax={Eo:.15e}", flush=True)
        assert st["status"] == 0
        assert abs(e32[p] - e64[p]) <= 1e-12 * abs(e64[p])
        assert abs(Eo - e64[p]) <= 1e-12 * abs(e64[p])
        for r in (res[FP64], res[MIXED]):
            d = np.hypot(r.x.cpu().numpy()[sl] - xo, r.y.cpu().numpy()[sl] - yo).max()
            assert d <= 1e-3 * h
    assert sum(int(flags[idx_np[ptr[p]:ptr[p + 1]]].sum()) for p in range(2)) > 0


def test_border_project_bit_exact(dev):
    x, y = W.uniform_disk(5000, 41)
    x[0], y[0] = 0.0, 0.0  # a boundary charge at the centre stays
    flags = OB.border_split(x, y, 400)
    flags[0] = 1
    for sigma in (0.3, 0.95, 1.0):
        xt, yt = t(x, dev), t(y, dev)
        B.border_project(xt, yt, t(flags, dev, torch.int32), sigma)
        px, py = OB.border_project(x, y, flags, sigma)
        assert np.array_equal(xt.cpu().numpy(), px) and np.array_equal(yt.cpu().numpy(), py)
        xt, yt = t(x, dev), t(y, dev)
        B.border_project(xt, yt, None, sigma)
        px, py = OB.border_project(x, y, None, sigma)
        assert np.array_equal(xt.cpu().numpy(), px) and np.array_equal(yt.cpu().numpy(), py)


@pytest.mark.parametrize("n", [1, 2, 700, 6000, 100000])
def test_border_spread_parity(dev, n):
    # the boundary charges of the split (Eq. 4's count, the farthest ones)
    # spread along the circle: the same charge at the same angle slot as the
    # oracle (slot order exact), positions to rounding, the rest untouched
    x, y = W.warped_lattice(n, 0.02, 1301) if n > 2 else W.uniform_disk(n, 1301)
    nb = max(1, B.boundary_count(n)) if n > 1 else 1
    flags = OB.border_split(x, y, nb)
    xt, yt = t(x, dev), t(y, dev)
    B.border_spread(xt, yt, t(flags, dev, torch.int32))
    gx, gy = xt.cpu().numpy(), yt.cpu().numpy()
    ox, oy = OB.border_spread(x, y, flags)
    f = flags == 1
    assert np.array_equal(gx[~f], x[~f]) and np.array_equal(gy[~f], y[~f])
    assert np.max(np.abs(gx - ox)) <= 2e-15 and np.max(np.abs(gy - oy)) <= 2e-15  # atan2, cos, sin: device vs host libm
    assert np.all(np.abs(np.hypot(gx[f], gy[f]) - 1.0) <= 1e-15)
    if f.sum() > 2:  # slot order: consecutive angles are 2 pi / nb apart in the oracle's order
        ang = np.mod(np.arctan2(gy[f], gx[f]) - np.arctan2(oy[f], ox[f]), 2 * np.pi)
        assert np.all(np.minimum(ang, 2 * np.pi - ang) <= 1e-12)


def test_defect_cycle_border_interior_small(dev):
    """A small defect-targeted cycle under the split with the sigma ramp:
    boundary charges stay on the circle, interior ones within the final
    sigma, the energy falls, and the tracked energy equals a fresh oracle
    evaluation."""
    from paper_2609_24722_amd import cycle
    n = 6000
    x, y = W.warped_lattice(n, 0.1, 1107)
    xt, yt = t(x, dev), t(y, dev)
    nb = B.boundary_count(n)
    flags = OB.border_split(x, y, nb)
    out = cycle.defect_cycle(xt, yt, T=96, cap=32, n_lo=50, n_hi=400, period=24, seed=1209, precision=MIXED,
                             border_nb=nb)
    xs, ys = xt.cpu().numpy(), yt.cpu().numpy()
    r = np.hypot(xs, ys)
    print(f"[bi-cycle] nb={nb} batches={out['batches']} committed={out['committed']} "
          f"E {out['E_start']:.10e} -> {out['E_end']:.10e} relax_status={out['relax_status']}", flush=True)
    assert out["E_end"] < out["E_start"]
    assert abs(out["tracked_energy"] - out["E_end"]) <= 1e-12 * out["E_end"]
    assert abs(out["E_end"] - O.energy(xs, ys)) <= 1e-13 * out["E_end"]
    assert np.all(np.abs(r[flags == 1] - 1.0) <= 1e-15)
    assert np.all(r[flags == 0] <= 1.0 + 1e-15)
    # the spread start leaves no near-coincident boundary charges: every zone converges
    assert out["committed"] >= 48 and out["relax_status"] == [96, 0, 0, 0]
