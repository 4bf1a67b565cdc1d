"""Host-side parts of the zone entry points (no GPU): the batch scheduler
zone_batches is host code and must give exactly the oracle's batches; the
device entry points reject bad arguments before anything is launched."""
import ctypes
import os

import numpy as np
import pytest

from oracle import zones as Z

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_24722_amd", "libcoulombdisk.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _zb():
    from paper_2609_24722_amd import zones
    return zones.zone_batches


def _random_zones(T, seed, r_lo=0.01, r_hi=0.2):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, size=(3 * T, 2))
    u = u[(u * u).sum(1) < 1][:T]
    return u[:, 0].copy(), u[:, 1].copy(), rng.uniform(r_lo, r_hi, T)


@pytest.mark.parametrize("keep_order", [True, False])
@pytest.mark.parametrize("T,gap,cap,seed", [(1, 0.0, 1, 1), (300, 0.0, 1000, 2), (300, 0.01, 16, 3),
                                            (500, 0.05, 1000, 4), (200, 0.0, 1, 5)])
def test_zone_batches_equal_oracle(T, gap, cap, seed, keep_order):
    cx, cy, rz = _random_zones(T, seed)
    b, nb = _zb()(cx, cy, rz, gap, cap, keep_order)
    want = Z.zone_batches(cx, cy, rz, gap, cap, keep_order)
    assert np.array_equal(b, want)
    assert nb == int(want.max()) + 1


def test_zone_batches_degenerate_inputs():
    zb = _zb()
    for order in (True, False):
        # identical centres conflict pairwise; zero radii with zero gap never conflict
        b, nb = zb(np.zeros(5), np.zeros(5), np.full(5, 0.1), 0.0, 100, order)
        assert b.tolist() == [0, 1, 2, 3, 4] and nb == 5
        b, nb = zb(np.zeros(5), np.zeros(5), np.zeros(5), 0.0, 100, order)
        assert b.tolist() == [0] * 5 and nb == 1
        # exact touching (distance == r_a + r_b + gap) is not a conflict
        b, _ = zb(np.array([0.0, 0.5]), np.zeros(2), np.array([0.25, 0.25]), 0.0, 10, order)
        assert b.tolist() == [0, 0]
        assert zb(np.zeros(0), np.zeros(0), np.zeros(0), 0.0, 4, order)[1] == 0
    # a chain a-b-c (a, c apart): ordered 0, 1, 2; first fit 0, 1, 0
    cx = np.array([0.0, 0.15, 0.3])
    assert zb(cx, np.zeros(3), np.full(3, 0.1), 0.0, 10, True)[0].tolist() == [0, 1, 2]
    assert zb(cx, np.zeros(3), np.full(3, 0.1), 0.0, 10, False)[0].tolist() == [0, 1, 0]


def test_zone_batches_grid_matches_brute_force_at_scale():
    """Many small zones: the grid path (many cells) must still find every
    conflict the brute-force oracle finds."""
    cx, cy, rz = _random_zones(1500, 9, 0.005, 0.03)
    for order in (True, False):
        b, _ = _zb()(cx, cy, rz, 0.002, 64, order)
        assert np.array_equal(b, Z.zone_batches(cx, cy, rz, 0.002, 64, order))


def test_zone_entry_points_reject_bad_arguments():
    L = ctypes.CDLL(LIB)
    from paper_2609_24722_amd import zones
    vp = ctypes.c_void_p
    L.zone_batches.restype = ctypes.c_int
    L.zone_batches.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                               vp, vp]
    a = np.zeros(3)
    out = np.zeros(3, dtype=np.int32)
    p = a.ctypes.data
    assert L.zone_batches(p, p, p, 3, 0.0, 0, 1, out.ctypes.data, None) == -1          # cap < 1
    assert L.zone_batches(p, p, p, 3, -1.0, 4, 1, out.ctypes.data, None) == -1         # negative gap
    bad = np.array([0.1, np.nan, 0.1])
    assert L.zone_batches(p, p, bad.ctypes.data, 3, 0.0, 4, 1, out.ctypes.data, None) == -1
    ws = L.coulomb_workspace_bytes
    ws.restype = ctypes.c_size_t
    ws.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int]
    assert ws(7, 1000, 0, 0, 0) >= 4000 and ws(7, 0, 0, 0, 0) == 0
    assert ws(8, 1000, 10, 0, 0) > 0 and ws(8, 1000, 0, 0, 0) == 0
    L.defect_zones.restype = ctypes.c_int
    L.defect_zones.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.POINTER(zones.ZoneOpts),
                               vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    fake = vp(256)
    good = zones.ZoneOpts(-1.0, 0.8, 0.01, 0.1, 0, 10, 0)
    big = ws(7, 1000, 0, 0, 0)
    call = lambda o, P=4, wsb=big: L.defect_zones(fake, fake, fake, 1000, P, fake, ctypes.byref(o), fake, fake,
                                                  fake, fake, None, None, fake, wsb, None)
    assert call(zones.ZoneOpts(-1.0, 0.8, 0.01, 0.1, 0, 0, 0)) == -1     # period < 1
    assert call(zones.ZoneOpts(-1.0, 0.8, 0.2, 0.1, 0, 10, 0)) == -1     # r_hi < r_lo
    assert call(zones.ZoneOpts(-1.0, 0.8, 0.01, 0.1, -1, 10, 0)) == -1   # t0 < 0
    assert call(good, P=-1) == -1
    assert call(good, wsb=16) == -2
    L.zone_patches.restype = ctypes.c_int
    L.zone_patches.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_int64, vp,
                               ctypes.c_size_t, vp]
    ptr = np.zeros(5, dtype=np.int32)
    zbig = ws(8, 1000, 4, 0, 0)
    assert L.zone_patches(fake, fake, 1000, 0, fake, fake, fake, ptr.ctypes.data, fake, 10, fake, zbig, None) == -1
    assert L.zone_patches(fake, fake, 1000, 4, fake, fake, fake, None, fake, 10, fake, zbig, None) == -1
    assert L.zone_patches(fake, fake, 1000, 4, fake, fake, fake, ptr.ctypes.data, None, 10, fake, zbig, None) == -1
    assert L.zone_patches(fake, fake, 1000, 4, fake, fake, fake, ptr.ctypes.data, fake, 10, fake, 8, None) == -2
    L.coulomb_status_string.restype = ctypes.c_char_p
    assert b"capacity" in L.coulomb_status_string(-5)
