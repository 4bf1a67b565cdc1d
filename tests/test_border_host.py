"""Host parts of the border-interior entry points (no GPU): Eq. 4's count and
Eq. 5's radius from the library equal the oracle's; argument errors."""
import ctypes
import os

import pytest

from oracle import border as OB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_24722_amd", "libcoulombdisk.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def test_border_count_and_sigma0_equal_oracle():
    from paper_2609_24722_amd import border as B
    for n in list(range(1, 3000)) + [10000, 40000, 100000, 123457, 1 << 26]:
        assert B.boundary_count(n) == min(n, OB.boundary_count(n)), n
        assert B.sigma0(n) == OB.sigma0(n), n
    assert B.boundary_count(100000) == 6099


def test_border_split_rejects_bad_arguments():
    L = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    L.border_split.restype = ctypes.c_int
    L.border_split.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp]
    fake = vp(256)
    assert L.border_split(fake, fake, 100, 101, fake, None) == -1
    assert L.border_split(fake, fake, 100, -1, fake, None) == -1
    assert L.border_split(None, fake, 100, 5, fake, None) == -1
    assert L.border_split(fake, fake, 0, 0, fake, None) == -1
