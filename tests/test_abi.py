"""The C-ABI library loads and exports every symbol its header declares;
argument errors are reported before anything touches a GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_24722_amd", "libcoulombdisk.so")
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            if m.group(1) not in ("if", "while", "defined"):
                names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["coulomb_energy", "coulomb_forces", "coulomb_hvp", "relax_subdomains", "build_patches",
              "coulomb_workspace_bytes", "coulomb_validate", "coulomb_status_string"]:
        assert n in names, n


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_workspace_sizes_are_host_computable(L):
    f = L.coulomb_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int]
    for op in (0, 1, 2, 3):
        for prec in (0, 1):
            a = f(op, 1000, 0, 0, prec)
            b = f(op, 100000, 0, 0, prec)
            assert 0 < a < b
    assert f(1, 0, 0, 0, 0) == 0          # n < 1
    assert f(1, 100, 0, 0, 7) == 0        # bad precision


def test_relax_workspace_grows_with_patch_size(L):
    # commit_patches sizes its scratch for the largest patch and evaluates
    # each patch in it, so a smaller patch must never need more (a 127-charge
    # patch once needed more than a 128-charge one).
    f = L.coulomb_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int]
    for n in (5000, 40000, 100000):
        for prec in (0, 1):
            sizes = [f(5, n, 1, k, prec) for k in range(1, 4097)]
            assert all(s > 0 for s in sizes)
            assert all(b >= a for a, b in zip(sizes, sizes[1:])), (n, prec)


def test_argument_errors_before_any_launch(L):
    vp = ctypes.c_void_p
    L.coulomb_forces.restype = ctypes.c_int
    L.coulomb_forces.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int, vp, vp, vp, vp, ctypes.c_size_t, vp]
    fake = vp(256)
    assert L.coulomb_forces(None, fake, 10, 0, fake, fake, None, fake, 1 << 30, None) == -1
    assert L.coulomb_forces(fake, fake, 10, 0, fake, fake, None, None, 0, None) == -2
    assert L.coulomb_forces(fake, fake, 10, 0, fake, fake, None, fake, 16, None) == -2
    assert L.coulomb_forces(fake, fake, 0, 0, fake, fake, None, fake, 1 << 30, None) == -1
    L.coulomb_status_string.restype = ctypes.c_char_p
    assert L.coulomb_status_string(-2) == b"workspace missing or too small"


def test_relax_argument_errors_before_any_launch(L):
    import numpy as np

    class Opts(ctypes.Structure):
        _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("lbfgs_m", ctypes.c_int32),
                    ("max_outer", ctypes.c_int32), ("gtol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                    ("halo_width", ctypes.c_double), ("step0", ctypes.c_double), ("sigma", ctypes.c_double),
                    ("boundary", ctypes.c_void_p), ("polish", ctypes.c_int32), ("max_polish_iter", ctypes.c_int32),
                    ("newton_tol", ctypes.c_double), ("cg_eta", ctypes.c_double), ("polish_stats", ctypes.c_void_p),
                    ("trust_radius", ctypes.c_double), ("coords", ctypes.c_int32),
                    ("launch", ctypes.c_int32), ("exterior_model", ctypes.c_int32)]
    vp = ctypes.c_void_p
    f = L.relax_subdomains
    f.restype = ctypes.c_int
    f.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp, ctypes.POINTER(Opts), vp, vp, vp, vp, vp,
                  vp, vp, vp, ctypes.c_size_t, vp]
    ws = L.coulomb_workspace_bytes
    ws.restype = ctypes.c_size_t
    ws.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int]
    ptr = np.array([0, 10, 30], dtype=np.int32)
    fake = vp(256)
    big = ws(5, 1000, 2, 30, 1)
    assert big > 0 and ws(5, 1000, 2, 30, 0) > 0
    o = Opts(1, 100, 8, 0, 1e-3, 0.0, 0.0, 0.0)
    call = lambda o, wsb, p=ptr: f(fake, fake, 1000, 2, p.ctypes.data, fake, None, None, ctypes.byref(o),
                                   fake, fake, None, None, None, None, None, fake, wsb, None)
    assert call(Opts(1, 100, 17, 0, 1e-3, 0.0, 0.0, 0.0), big) == -1   # memory above 16
    assert call(Opts(1, 100, 8, 0, 0.0, 0.0, 0.0, 0.0), big) == -1     # gtol must be > 0
    assert call(Opts(3, 100, 8, 0, 1e-3, 0.0, 0.0, 0.0), big) == -1    # bad precision
    assert call(Opts(1, 100, 8, 0, 1e-3, 0.0, 0.0, 0.0, 1.5), big) == -1   # interior wall beyond the disk
    assert call(Opts(1, 100, 8, 0, 1e-3, 0.0, 0.0, 0.0, -0.1), big) == -1  # negative interior wall
    def polished(**kw):
        q = Opts(1, 100, 8, 0, 1e-3, 0.0, 0.0, 0.0)
        for k, v in kw.items():
            setattr(q, k, v)
        return q
    assert call(polished(polish=3), big) == -1                          # unknown polish mode
    assert call(polished(max_polish_iter=-1), big) == -1                # negative CG cap
    assert call(polished(newton_tol=-1.0), big) == -1                   # negative switch
    assert call(polished(cg_eta=1.0), big) == -1                        # CG target not below 1
    assert call(polished(trust_radius=-1.0), big) == -1                 # negative trust radius
    assert call(polished(coords=2), big) == -1                          # unknown coordinates
    assert call(polished(launch=2), big) == -1                          # unknown launch mode
    assert call(polished(exterior_model=3), big) == -1                  # unknown exterior model
    assert call(polished(precision=1, exterior_model=1), big) == -1     # exact exterior needs FP64
    assert call(o, 1024) == -2                                          # workspace too small
    assert call(o, big, np.array([0, 10, 10], dtype=np.int32)) == -1    # empty patch
    assert call(o, big, np.array([1, 10, 30], dtype=np.int32)) == -1    # offsets must start at 0


def test_noalloc_refuses_sizes_beyond_its_scratch(L):
    # refused on the host before anything is enqueued (the first n past the fixed
    # scratch on each path); smaller sizes reach the GPU and are GPU tests
    f = L.coulomb_forces_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64, ctypes.c_int] + [ctypes.c_void_p] * 4
    d = ctypes.c_void_p(256)
    assert f(d, d, 706305, 1, d, d, None, None) == -6
    assert f(d, d, 830721, 0, d, d, None, None) == -6
    assert f(d, d, 1 << 27, 0, d, d, None, None) == -1   # beyond any plan
    assert f(None, d, 10, 0, d, d, None, None) == -1


def test_relax_autotune_argument_errors(L):
    vp = ctypes.c_void_p
    f = L.relax_autotune
    f.restype = ctypes.c_int
    f.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp, vp, vp]
    import numpy as np
    ptr = np.array([0, 10], dtype=np.int32)
    fake = vp(256)
    assert f(fake, fake, 100, 1, ptr.ctypes.data, fake, None, None, fake, fake, 1 << 20, None, None, None) == -1
    assert f(fake, fake, 100, 0, ptr.ctypes.data, fake, None, None, fake, fake, 1 << 20, None, fake, None) == -1


def test_host_functions_of_the_method(L):
    """The host-side arithmetic entry points against the oracle's own
    definitions (no GPU needed)."""
    import math
    from oracle import border as OB
    L.border_sigma_ramp.restype = ctypes.c_double
    L.border_sigma_ramp.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_double]
    L.zone_radius_holding.restype = ctypes.c_double
    L.zone_radius_holding.argtypes = [ctypes.c_int64, ctypes.c_int64]
    for n in (7, 1000, 100000):
        for stages in (1, 4, 44):
            for k in range(stages + 1):
                assert L.border_sigma_ramp(n, k, stages, 0.0, 1.0) == OB.sigma_ramp(k, stages, n)
        assert L.border_sigma_ramp(n, -3, 4, 0.0, 1.0) == OB.sigma0(n)
        assert L.border_sigma_ramp(n, 9, 4, 0.0, 1.0) == 1.0
        assert L.border_sigma_ramp(n, 0, 0, 0.5, 0.9) == 0.9
        # a zone of radius sqrt(c / n) holds c of n charges at density n / pi
        for c in (0, 200, 4000):
            r = L.zone_radius_holding(n, c)
            assert abs(math.pi * r * r * (n / math.pi) - c) <= 1e-12 * max(c, 1)
    assert L.zone_radius_holding(0, 5) == 0.0 and L.zone_radius_holding(5, -1) == 0.0
