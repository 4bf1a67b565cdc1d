"""Greedy commit of relaxed candidates against a plain greedy loop on the
oracle; candidates are oracle-relaxed patches, partly overlapping."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_24722_amd import workloads as W
from paper_2609_24722_amd import relax as R

pytestmark = pytest.mark.gpu


def test_commit_matches_oracle_greedy(dev):
    n = 3000
    x, y = W.warped_lattice(n, 0.1, 41)
    h = W.spacing(n)
    centres, sizes = W.patch_draws(n, 10, 20, 120, 42)
    idx = O.patches(x, y, centres, sizes)
    ptr = np.zeros(sizes.size + 1, dtype=np.int32)
    ptr[1:] = np.cumsum(sizes)
    # candidates: oracle relax of kicked actives (some lower the energy, some not)
    kx, ky = W.kicks(idx.size, 0.3 * h, 43)
    xr = np.empty(idx.size)
    yr = np.empty(idx.size)
    key = np.empty(sizes.size)
    for p in range(sizes.size):
        sl = slice(ptr[p], ptr[p + 1])
        if p % 3 == 2:  # an unrelaxed kicked candidate (energy change usually positive)
            xa, ya = x[idx[sl]] + kx[sl], y[idx[sl]] + ky[sl]
            rr = np.hypot(xa, ya)
            xa, ya = np.where(rr > 1, xa / rr, xa), np.where(rr > 1, ya / rr, ya)
        else:
            xa, ya, _ = O.relax(x, y, idx[sl], x[idx[sl]] + kx[sl], y[idx[sl]] + ky[sl], gtol=1e-6)
        xr[sl], yr[sl] = xa, ya
        key[p] = O.esub_delta(x, y, idx[sl], xa, ya)
    # oracle greedy
    X, Y = x.copy(), y.copy()
    taken = np.zeros(n, bool)
    ref_c = np.zeros(sizes.size, np.int32)
    ref_d = np.zeros(sizes.size)
    for p in sorted([p for p in range(sizes.size) if key[p] < 0], key=lambda p: (key[p], p)):
        sl = slice(ptr[p], ptr[p + 1])
        if taken[idx[sl]].any():
            continue
        d = O.esub_delta(X, Y, idx[sl], xr[sl], yr[sl])
        ref_d[p] = d
        if d < 0:
            X[idx[sl]], Y[idx[sl]] = xr[sl], yr[sl]
            taken[idx[sl]] = True
            ref_c[p] = 1
    xt = torch.tensor(x, device=dev)
    yt = torch.tensor(y, device=dev)
    E0 = O.energy(x, y)
    c, d = R.commit_patches(xt, yt, ptr, torch.tensor(idx, device=dev), torch.tensor(xr, device=dev),
                            torch.tensor(yr, device=dev), key)
    torch.cuda.synchronize()
    print(f"[commit] committed {c.tolist()} ref {ref_c.tolist()}")
    assert np.array_equal(c, ref_c) and ref_c.sum() >= 2
    np.testing.assert_allclose(d, ref_d, rtol=1e-9, atol=1e-12 * E0)
    assert np.array_equal(xt.cpu().numpy(), X) and np.array_equal(yt.cpu().numpy(), Y)
    # tracked energy vs a from-scratch evaluation (drift check)
    assert abs((E0 + d[c == 1].sum()) - O.energy(X, Y)) <= 1e-12 * E0


def test_commit_patch_sizes_across_block_boundary(dev):
    # patches of 127 and 128 charges: the scratch sized for the largest patch
    # must hold the evaluation of every smaller one
    n = 4000
    x, y = W.warped_lattice(n, 0.1, 51)
    h = W.spacing(n)
    sizes = np.array([128, 127, 63, 65], dtype=np.int32)
    centres = np.array([100, 1500, 2500, 3500], dtype=np.int32)
    idx = O.patches(x, y, centres, sizes)
    ptr = np.zeros(sizes.size + 1, dtype=np.int32)
    ptr[1:] = np.cumsum(sizes)
    kx, ky = W.kicks(idx.size, 0.05 * h, 52)
    xr, yr = x[idx] + kx, y[idx] + ky
    rr = np.hypot(xr, yr)
    xr, yr = np.where(rr > 1, xr / rr, xr), np.where(rr > 1, yr / rr, yr)
    key = -np.arange(1.0, sizes.size + 1)  # every candidate is tried, largest first
    xt = torch.tensor(x, device=dev)
    yt = torch.tensor(y, device=dev)
    c, d = R.commit_patches(xt, yt, ptr, torch.tensor(idx, device=dev), torch.tensor(xr, device=dev),
                            torch.tensor(yr, device=dev), key)
    torch.cuda.synchronize()
    # reference: the same greedy order on the oracle (the patches are disjoint,
    # so every candidate is evaluated, against the configuration as committed)
    X, Y = x.copy(), y.copy()
    ref_d = np.zeros(sizes.size)
    for p in np.argsort(key, kind="stable"):
        sl = slice(ptr[p], ptr[p + 1])
        ref_d[p] = O.esub_delta(X, Y, idx[sl], xr[sl], yr[sl])
        if ref_d[p] < 0:
            X[idx[sl]], Y[idx[sl]] = xr[sl], yr[sl]
    assert np.array_equal(c, (ref_d < 0).astype(np.int32)) and 0 < c.sum() < sizes.size
    np.testing.assert_allclose(d, ref_d, rtol=1e-9, atol=1e-9)
