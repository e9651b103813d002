"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/fr.h, and rejects invalid descriptions before touching a
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fr.h")
LIB = os.path.join(ROOT, "paper_1910_03693_amd", "libfrx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libfrx():
    if not os.path.exists(LIB):
        from paper_1910_03693_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("fr_residual", "fr_jvp", "fr_vjp", "gmres_stage_solve", "esdirk_step", "spectral_decay_indicator"):
        assert n in names


def test_library_exports_every_declared_symbol(libfrx):
    missing = [n for n in declared_functions() if not hasattr(libfrx, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1910_03693_amd import frx
    for n in declared_functions():
        assert n in frx.EXPORTED, n


def _desc(frx, elem_xyz, elem_nbr, elem_p, physics=0):
    d = frx.fr_mesh_desc()
    d.n_elem = len(elem_p)
    d.elem_xyz = elem_xyz.ctypes.data_as(C.POINTER(C.c_double))
    d.elem_nbr = elem_nbr.ctypes.data_as(C.POINTER(C.c_int32))
    d.elem_p = elem_p.ctypes.data_as(C.POINTER(C.c_int8))
    d.physics, d.flux, d.gamma, d.mu, d.prandtl = physics, 0, 1.4, 0.0, 0.72
    return d


@pytest.mark.parametrize("bad", ["degree", "neighbour", "asymmetric", "nonconforming", "empty", "gamma"])
def test_create_rejects_invalid_descriptions(libfrx, bad):
    from paper_1910_03693_amd import frx
    from paper_1910_03693_amd import inputs as I
    m = I.box_mesh(2, 2, 1, (1.0, 1.0, 0.5))
    xyz = np.ascontiguousarray(m["elem_xyz"])
    nbr = np.ascontiguousarray(m["elem_nbr"])
    p = np.full(4, 2, np.int8)
    if bad == "degree":
        p[1] = 6
    elif bad == "neighbour":
        nbr[0, 1] = 17
    elif bad == "asymmetric":
        nbr[0, 1] = 0
    elif bad == "nonconforming":
        xyz[1, 0, 1] += 0.1  # moves a vertex of the face shared with element 0
    d = _desc(frx, xyz, nbr, p)
    if bad == "empty":
        d.n_elem = 0
    if bad == "gamma":
        d.gamma = 1.0
    L = frx.lib()
    h = C.c_void_p()
    st = L.fr_create(C.byref(d), C.byref(h))
    assert st == frx.FR_E_INVALID
    assert not h.value
    assert L.fr_last_error(None)
    with pytest.raises(frx.FrError):
        frx._check(st)
