"""Riesz-s energy and forces on the GPU against the Riesz oracle: sizes that
span several tiles with ragged tails, several exponents, both precisions;
the Coulomb case against coulomb_forces; at N = 1e5 in the benchmark's
launch configuration, Euler's identity sum r.F = s E and the n-gon closed
form."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_24722_amd import FP64, MIXED, ops, workloads as W

pytestmark = pytest.mark.gpu

# Tolerances.  FP64: pow and FP64 sums, as for the 1/r path.  Mixed: the
# pair term 2^(t), t = (-s/2 - 1) log2 r2, is formed in FP32: t is rounded to
# about |t| 2^-23 and the log2 adds about one ulp of it, so the term carries
# up to about ln2 |t| 2^-22 relative error (the exp2 adds ~2 ulp).  The
# closest pair sets the largest |t|; the energy and forces of the near pairs
# dominate for larger s, so the bound is used unreduced (forces: twice it).
TOL = {FP64: (1e-13, 1e-11)}


def mixed_tol(x, y, s):
    from scipy.spatial import cKDTree
    d, _ = cKDTree(np.stack([x, y], 1)).query(np.stack([x, y], 1), k=2)
    r2min = float(np.min(d[:, 1])) ** 2
    t = (s / 2 + 1) * abs(np.log2(r2min)) + 2.0
    b = np.log(2.0) * t * 2.0 ** -22
    return 1.5 * b, 3.0 * b


def tol(prec, x, y, s):
    return TOL[prec] if prec == FP64 else mixed_tol(x, y, s)


def rel_rms(a, b):
    return np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2))


@pytest.mark.parametrize("prec", [FP64, MIXED])
@pytest.mark.parametrize("n", [2, 3, 17, 64, 65, 127, 700, 4097])
def test_riesz_parity(dev, prec, n):
    x, y = W.uniform_disk(n, 5000 + n) if n < 700 else W.warped_lattice(n, 0.1, 5000 + n)
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    # 2s integer (FP64: powers of the refined 1/r) and not (FP64: pow)
    for s in (0.5, 1.0, 1.7, 2.0, 3.5):
        etol, ftol = tol(prec, x, y, s) if n > 1 else (0, 0)
        print(f"[case] riesz n={n} s={s} prec={prec} tol {etol:.1e} {ftol:.1e}", flush=True)
        fx, fy, E = ops.riesz(xt, yt, s, prec)
        E0, gx, gy = O.riesz(x, y, s)
        e = abs(E.item() - E0) / E0
        f = rel_rms(np.concatenate([fx.cpu().numpy(), fy.cpu().numpy()]), np.concatenate([gx, gy]))
        assert e <= etol and f <= ftol, (s, e, f)


def test_riesz_one_charge(dev):
    xt = torch.tensor([0.3], dtype=torch.float64, device=dev)
    yt = torch.tensor([-0.2], dtype=torch.float64, device=dev)
    for prec in (FP64, MIXED):
        fx, fy, E = ops.riesz(xt, yt, 2.0, prec)
        assert E.item() == 0.0 and fx.item() == 0.0 and fy.item() == 0.0


def test_riesz_coulomb_case(dev):
    x, y = W.warped_lattice(20000, 0.05, 77)
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    for prec in (FP64, MIXED):
        etol, ftol = tol(prec, x, y, 1.0)
        fx, fy, E = ops.riesz(xt, yt, 1.0, prec)
        gx, gy, E1 = ops.forces(xt, yt, prec)
        assert abs(E.item() - E1.item()) <= etol * E1.item()
        d = rel_rms(torch.cat([fx, fy]).cpu().numpy(), torch.cat([gx, gy]).cpu().numpy())
        assert d <= ftol, d


def test_riesz_full_oracle_n20000(dev):
    x, y = W.warped_lattice(20000, 0.05, 78)
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    for sv in (2.0, 2.3):
        E0, gx, gy = O.riesz(x, y, sv)
        for prec in (FP64, MIXED):
            etol, ftol = tol(prec, x, y, sv)
            fx, fy, E = ops.riesz(xt, yt, sv, prec)
            assert abs(E.item() - E0) <= etol * E0
            assert rel_rms(np.concatenate([fx.cpu().numpy(), fy.cpu().numpy()]), np.concatenate([gx, gy])) <= ftol


def test_riesz_n100000_properties(dev):
    """At the benchmark's size and launch configuration: Euler's identity for
    a homogeneous energy of degree -s, FP64 against mixed, and a regular
    100000-gon against the closed form n (n^2 - 1) / 24 (s = 2)."""
    x, y = W.workload(3)
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    for s in (2.0, 3.0):
        out = {}
        for prec in (FP64, MIXED):
            fx, fy, E = ops.riesz(xt, yt, s, prec)
            rf = xt * fx + yt * fy
            vir, scale = float(torch.sum(rf).item()), float(torch.sum(torch.abs(rf)).item())
            print(f"[riesz-1e5] s={s} prec={prec} E={E.item():.15e} virial/sE-1={vir / (s * E.item()) - 1:.2e} "
                  f"sum|r.F|/sE={scale / (s * E.item()):.1f}", flush=True)
            # the virial sum cancels (sum |r.F| is up to ~1e4 s E at s = 3), so its error is
            # measured against sum |r.F|: FP64 rounding, or the mixed force bound
            assert abs(vir - s * E.item()) <= (1e-14 if prec == FP64 else mixed_tol(x, y, s)[1]) * scale
            out[prec] = (E.item(), torch.cat([fx, fy]).cpu().numpy())
        etol, ftol = mixed_tol(x, y, s)
        de, df = abs(out[MIXED][0] - out[FP64][0]) / out[FP64][0], rel_rms(out[MIXED][1], out[FP64][1])
        print(f"[riesz-1e5] s={s} mixed vs FP64: E {de:.2e} (tol {etol:.1e}) F {df:.2e} (tol {ftol:.1e})", flush=True)
        assert de <= etol and df <= ftol
    n = 100000
    t = 0.1 + 2 * np.pi * np.arange(n) / n
    xt, yt = torch.tensor(np.cos(t), device=dev), torch.tensor(np.sin(t), device=dev)
    want = n * (n * n - 1) / 24
    _, _, E = ops.riesz(xt, yt, 2.0, FP64)
    assert abs(E.item() - want) <= 1e-11 * want
