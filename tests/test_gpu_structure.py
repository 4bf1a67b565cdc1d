"""Structure analysis on the GPU against the structure oracle (scipy's
Delaunay triangulation and convex hull): coordination numbers bit-exact,
hull charges marked, psi_6 to rounding, radial counts bit-exact; at
N = 1e5 on the benchmark's lattice as well."""
import numpy as np
import pytest
import torch

from oracle import structure as S
from paper_2609_24722_amd import structure as ST, workloads as W

pytestmark = pytest.mark.gpu


def _cmp(dev, x, y, label):
    import time
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z, psi = ST.voronoi(xt, yt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    st = ST.stats(z, psi)
    z = z.cpu().numpy()
    zo = S.voronoi_z(x, y)
    nb = S.voronoi_neighbours(x, y)
    po = S.psi6(x, y, nb)
    po[zo < 0] = 0
    bad = np.nonzero(z != zo)[0]
    print(f"[{label}] n={x.size} {ms:.1f} ms hull={int((zo == -2).sum())} P6={float((zo == 6).mean()):.4f} "
          f"mismatch={bad.size} {list(zip(bad[:5], z[bad[:5]], zo[bad[:5]]))}", flush=True)
    assert bad.size == 0
    assert np.max(np.abs(psi.cpu().numpy() - po)) < 1e-12
    # the statistics of Sec. III from the oracle's cells, by their definition
    ok = zo >= 0
    b = int(ok.sum())
    assert st["bounded_cells"] == b and st["hull"] == int((zo == -2).sum())
    assert st["unresolved"] == int((zo == -1).sum())
    for k in (4, 5, 6, 7, 8):
        assert abs(st["P_z"][k] - (zo == k).sum() / b) <= 2.3e-16 * max(1.0, st["P_z"][k] * 4)
    want = float(np.abs(po[ok]).mean())
    assert abs(st["mean_abs_psi6"] - want) <= 1e-12 * want


@pytest.mark.parametrize("case", ["lattice2000", "lattice20000", "uniform3000", "ring", "wall_ring"])
def test_voronoi_matches_oracle(dev, case):
    if case == "lattice2000":
        x, y = W.warped_lattice(2000, 0.1, 3)
    elif case == "lattice20000":
        x, y = W.warped_lattice(20000, 0.02, 4)
    elif case == "uniform3000":
        x, y = W.uniform_disk(3000, 5)
    elif case == "wall_ring":
        # a relaxed configuration's outer layer: charges on the unit circle
        # (all hull vertices) around a denser interior
        t = 2 * np.pi * (np.arange(800) + np.random.default_rng(6).uniform(-0.2, 0.2, 800)) / 800
        xi, yi = W.warped_lattice(8000, 0.02, 6)
        x, y = np.concatenate([np.cos(t), 0.995 * xi]), np.concatenate([np.sin(t), 0.995 * yi])
    else:
        t = 0.3 + 2 * np.pi * np.arange(7) / 7
        x, y = np.append(np.cos(t), 0.05), np.append(np.sin(t), -0.02)
    _cmp(dev, x, y, case)


def test_voronoi_n100000(dev):
    x, y = W.workload(3)
    _cmp(dev, x, y, "lattice1e5")


def test_radial_histogram_exact(dev):
    x, y = W.uniform_disk(20000, 9)
    r = np.array([0.0, 0.05, 0.1, 0.35, 0.5, 0.999, 1.0, 0.25])
    x = np.concatenate([x, r])
    y = np.concatenate([y, np.zeros(r.size)])
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    for nb in (1, 4, 50, 1000):
        c = ST.radial_histogram(xt, yt, nb).cpu().numpy()
        assert np.array_equal(c, S.radial_counts(x, y, nb)), nb


def test_voronoi_degenerate_inputs(dev):
    """One, two and three charges are all hull vertices (z = -2).  Charges
    strictly between two others on a line have unbounded strip cells though
    they are not hull vertices: z = -1 (the documented result for a cell the
    largest square cannot hold), psi_6 = 0."""
    cases = [
        (np.array([0.1]), np.array([-0.2]), [-2]),
        (np.array([0.1, -0.3]), np.array([0.2, 0.4]), [-2, -2]),
        (np.array([0.0, 0.5, -0.4]), np.array([0.0, 0.1, 0.3]), [-2, -2, -2]),
        (np.linspace(-0.8, 0.8, 5), 0.25 * np.linspace(-0.8, 0.8, 5), [-2, -1, -1, -1, -2]),
    ]
    for x, y, want in cases:
        z, psi = ST.voronoi(torch.tensor(x, device=dev), torch.tensor(y, device=dev))
        assert z.cpu().numpy().tolist() == want
        assert np.all(psi.cpu().numpy() == 0.0)
        # no bounded cell: fractions and the mean are 0, the counts exact
        st = ST.stats(z, psi)
        assert st["bounded_cells"] == 0 and st["mean_abs_psi6"] == 0.0
        assert all(v == 0.0 for v in st["P_z"].values())
        assert st["hull"] == want.count(-2) and st["unresolved"] == want.count(-1)
        st0 = ST.stats(z)  # without psi_6
        assert st0["hull"] == st["hull"] and st0["mean_abs_psi6"] == 0.0
