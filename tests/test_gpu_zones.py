"""Defect-targeted zones on the GPU against the zone oracle (Sec. II.C steps
1-4): defect statistics and list, zone centres and radii (bit-exact on the
same local energies), zone membership (bit-exact), and one small
defect-targeted cycle end to end."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import zones as Z
from paper_2609_24722_amd import FP64, MIXED, cycle, ops, workloads as W, zones

pytestmark = pytest.mark.gpu


def _t(a, dev, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=dev)


@pytest.fixture(scope="module")
def lattice():
    n = 20000
    x, y = W.warped_lattice(n, 0.1, 1102)
    _, e = O.energy(x, y, local=True)
    return x, y, e


@pytest.mark.parametrize("kappa", [-1.0, 1.0])
def test_defect_zones_match_oracle(dev, lattice, kappa):
    x, y, e = lattice
    n = x.size
    T, period, t0 = 300, 100, 37
    r_lo, r_hi = np.sqrt(200 / n), np.sqrt(4000 / n)
    draws = W.zone_draws(T, 1203)
    z = zones.defect_zones(_t(x, dev), _t(y, dev), _t(e, dev), _t(draws, dev), kappa, 0.8, r_lo, r_hi, t0,
                           period)
    mu, sg, thr, D = Z.defect_stats(e, kappa)
    st = z["stats"].cpu().numpy()
    assert abs(st[0] - mu) <= 1e-14 * abs(mu)
    assert abs(st[1] - sg) <= 1e-12 * sg
    assert abs(st[2] - thr) <= 1e-14 * abs(mu)
    # no local energy sits within rounding of the threshold, so the lists are unique
    assert np.min(np.abs(e - thr)) > 1e-9 * abs(thr)
    assert int(st[3]) == D.size
    assert np.array_equal(z["defects"][:D.size].cpu().numpy(), D)
    cx, cy, ci = Z.zone_centres(x, y, D, draws, 0.8)
    assert np.array_equal(z["centre_idx"].cpu().numpy(), ci)
    assert np.array_equal(z["cx"].cpu().numpy(), cx) and np.array_equal(z["cy"].cpu().numpy(), cy)
    rz = np.array([Z.zone_radius(t0 + t, period, r_lo, r_hi) for t in range(T)])
    assert np.array_equal(z["rz"].cpu().numpy(), rz)
    assert 0 < (ci >= 0).sum() < T


def test_defect_list_from_gpu_local_energies(dev, lattice):
    """Steps 1-2 on the GPU (FP64 local energies, then the list) against the
    oracle's local energies and list."""
    x, y, e = lattice
    xt, yt = _t(x, dev), _t(y, dev)
    _, eg = ops.energy(xt, yt, FP64, local=True)
    assert np.max(np.abs(eg.cpu().numpy() - e) / np.abs(e)) < 1e-13
    for kappa in (-1.0, 1.0):
        z = zones.defect_zones(xt, yt, eg, torch.zeros(0, dtype=torch.float64, device=dev), kappa)
        st = z["stats"].cpu().numpy()
        D = Z.defect_stats(e, kappa)[3]
        Dg = z["defects"][:int(st[3])].cpu().numpy()
        diff = np.setxor1d(D, Dg)
        assert np.all(np.abs(e[diff] - st[2]) < 1e-12 * abs(st[2])), diff


def test_defect_zones_edge_cases(dev):
    x, y = W.uniform_disk(1, 5)
    draws = W.zone_draws(6, 3)
    z = zones.defect_zones(_t(x, dev), _t(y, dev), _t([2.5], dev), _t(draws, dev), -1.0, 0.8, 0.1, 0.1, 5, 3)
    st = z["stats"].cpu().numpy()
    assert st.tolist() == [2.5, 0.0, 2.5, 0.0]  # one charge: no spread, nothing above
    assert (z["centre_idx"].cpu().numpy() == -1).all()
    assert np.array_equal(z["cx"].cpu().numpy(), draws[2::4])
    assert (z["rz"].cpu().numpy() == 0.1).all()
    n = 3000
    x, y = W.uniform_disk(n, 6)
    xt, yt = _t(x, dev), _t(y, dev)
    d = _t(W.zone_draws(200, 7), dev)
    z = zones.defect_zones(xt, yt, _t(np.full(n, 7.0), dev), d, 1.0, 0.8)  # constant energies
    assert z["stats"].cpu().numpy().tolist() == [7.0, 0.0, 7.0, 0.0]
    e = np.arange(n, dtype=np.float64)
    e[5] = np.nan  # a non-finite energy: no defects, every centre a disk point
    z = zones.defect_zones(xt, yt, _t(e, dev), d, 1.0, 0.8)
    assert z["stats"].cpu().numpy()[3] == 0 and (z["centre_idx"].cpu().numpy() == -1).all()
    e = np.arange(n, dtype=np.float64)
    for p, want in ((1.0, True), (0.0, False)):
        ci = zones.defect_zones(xt, yt, _t(e, dev), d, 0.0, p)["centre_idx"].cpu().numpy()
        assert ((ci >= 0) == want).all()
        if want:
            assert (ci > (n - 1) / 2).all()  # kappa = 0: the upper half of 0..n-1


def test_zone_patches_bit_exact(dev, lattice):
    x, y, _ = lattice
    n = x.size
    rng = np.random.default_rng(21)
    P = 40
    cx = rng.uniform(-1.0, 1.0, P)
    cy = rng.uniform(-1.0, 1.0, P)
    rz = rng.uniform(0.0, 0.3, P)
    cx[0], cy[0], rz[0] = x[17], y[17], 0.0      # radius 0 at a charge: that charge
    cx[1], cy[1], rz[1] = 0.0, 0.0, 3.0          # covers the disk
    cx[2], cy[2], rz[2] = 2.0, 2.0, 0.5          # outside the disk: empty
    cx[3], cy[3], rz[3] = x[5], y[5], np.sqrt((x[5] - x[6]) ** 2 + (y[5] - y[6]) ** 2)  # on a charge
    ptr0, idx0 = Z.zones(x, y, cx, cy, rz)
    xt, yt = _t(x, dev), _t(y, dev)
    for cap in (0, 1, int(ptr0[-1])):  # capacity too small, then exact
        ptr, idx = zones.zone_patches(xt, yt, _t(cx, dev), _t(cy, dev), _t(rz, dev), capacity=cap)
        assert np.array_equal(ptr, ptr0)
        assert np.array_equal(idx.cpu().numpy(), idx0)
    assert ptr0[1] - ptr0[0] == 1 and ptr0[2] - ptr0[1] == n and ptr0[3] == ptr0[2]


@pytest.mark.parametrize("precision", [MIXED, FP64])
def test_defect_cycle_small(dev, precision):
    n = 6000
    x, y = W.warped_lattice(n, 0.1, 1107)
    xt, yt = _t(x, dev), _t(y, dev)
    h = W.spacing(n)
    seen = []

    def inspect(b, sel, cx, cy, rz, ptr, idx):
        xs, ys = xt.cpu().numpy(), yt.cpu().numpy()
        p0, i0 = Z.zones(xs, ys, cx[sel], cy[sel], rz[sel])
        p0 = p0[np.concatenate([[True], np.diff(p0) > 0])]  # empty zones are dropped
        assert np.array_equal(ptr, p0) and np.array_equal(idx.cpu().numpy(), i0)
        for a in range(sel.size):  # zones of one batch are mutually apart
            for c in range(a):
                s, t = sel[c], sel[a]
                assert not Z.conflict(cx[s], cy[s], rz[s], cx[t], cy[t], rz[t], 2.0 * h)
        seen.append(b)

    out = cycle.defect_cycle(xt, yt, T=96, cap=32, n_lo=50, n_hi=400, period=24, seed=1208,
                             precision=precision, inspect=inspect)
    assert seen and out["zones_relaxed"] == 96
    assert out["E_end"] < out["E_start"]
    assert abs(out["tracked_energy"] - out["E_end"]) <= 1e-12 * out["E_end"]
    assert abs(out["E_end"] - O.energy(xt.cpu().numpy(), yt.cpu().numpy())) <= 1e-13 * out["E_end"]
    assert out["committed"] >= 48
    assert out["relax_status"] == [96, 0, 0, 0]  # every zone converges
    assert (np.hypot(xt.cpu().numpy(), yt.cpu().numpy()) <= 1.0 + 1e-15).all()
