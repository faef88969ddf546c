"""CPU-side checks of the C ABI: the library loads, every entry point declared
in include/*.h is exported, and the host-only quadrature routine is exact."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = ""
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            with open(os.path.join(ROOT, "include", name)) as f:
                text += f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2204_03575_amd import chm
    if not os.path.exists(chm.LIB_PATH):
        from paper_2204_03575_amd.build import build
        build()
    return chm.library()


def test_header_declares_the_binding_entry_points():
    from paper_2204_03575_amd.chm import ENTRY_POINTS
    assert _declared() == sorted(ENTRY_POINTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2204_03575_amd import chm
    monkeypatch.setattr(chm, "_lib", None)
    monkeypatch.setattr(chm, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        chm.library()


def test_create_rejects_bad_arguments_without_touching_the_gpu(lib):
    from paper_2204_03575_amd import chm
    import synthetic as S
    p = S.preset("square32", n=(2, 2))
    co, ce = S.make_mesh(p)
    ce = ce.copy()
    ce[0, 0] = 999                      # vertex index out of range: rejected on the host
    mesh = chm.chm_mesh_t(2, co.shape[0], co.ctypes.data_as(ctypes.c_void_p), ce.shape[0],
                          ce.ctypes.data_as(ctypes.c_void_p))
    prm = chm.params_from_dict(p)
    h = ctypes.c_void_p()
    rc = lib.chm_create(ctypes.byref(mesh), ctypes.byref(prm), None, ctypes.byref(h))
    assert rc == chm.CHM_EINVAL and not h.value
    assert b"out of range" in lib.chm_last_error(None)
    ce[0, 0] = 0
    prm.eps[1] = 2e-3                   # species with different eps are not supported
    rc = lib.chm_create(ctypes.byref(mesh), ctypes.byref(prm), None, ctypes.byref(h))
    assert rc == chm.CHM_EINVAL and b"share" in lib.chm_last_error(None)
    prm = chm.params_from_dict(dict(p, restart=65))
    rc = lib.chm_create(ctypes.byref(mesh), ctypes.byref(prm), None, ctypes.byref(h))
    assert rc == chm.CHM_EINVAL


@pytest.mark.parametrize("dim", [2, 3])
def test_library_quadrature_exact_on_barycentric_monomials(lib, dim):
    from paper_2204_03575_amd import chm_quadrature
    bary, w = chm_quadrature(dim)
    assert len(w) == 3 ** dim
    assert np.isclose(w.sum(), 1.0, rtol=1e-15)
    for deg in range(6):
        for alpha in itertools.product(range(deg + 1), repeat=dim + 1):
            if sum(alpha) != deg:
                continue
            num = np.sum(w * np.prod(bary ** np.array(alpha), axis=1))
            exact = (np.prod([math.factorial(a) for a in alpha]) * math.factorial(dim)
                     / math.factorial(deg + dim))
            assert abs(num - exact) < 2e-15, (alpha, num, exact)
