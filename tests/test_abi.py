"""The C-ABI library loads and exports every symbol include/psf.h declares;
host-side argument checks fail cleanly without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1607_06170_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "psf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char\s*\*|const\s+char\s*\*)\s*\*?\s*(\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_symbols_exported():
    L = _lib.load()
    decl = _declared()
    assert len(decl) >= 13
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(_lib.SIGNATURES), set(decl) ^ set(_lib.SIGNATURES)


def test_status_strings():
    L = _lib.load()
    for code in range(-8, 1):
        assert L.psf_status_string(code)
    assert L.psf_status_string(-99) == b"unknown status"


def _geom(**kw):
    g = dict(n_blocks=16, n_cryst_t=8, n_cryst_z=1, n_block_rings=1, pitch_t=2.0, pitch_z=2.0, depth=15.0,
             radius_face=65.0, gap_z=0.0, mu=0.087, phi0=0.0)
    g.update(kw)
    return _lib.psf_geometry(**g)


def _img(**kw):
    d = dict(nx=64, ny=64, nz=1, pad=0, dx=1.0, dy=1.0, dz=1.0, cx=0.0, cy=0.0, cz=0.0)
    d.update(kw)
    return _lib.psf_image(**d)


@pytest.mark.parametrize("g,im,mode,code", [
    (dict(n_blocks=2), {}, 0, _lib.PSF_EINVAL),
    (dict(pitch_t=-1.0), {}, 0, _lib.PSF_EINVAL),
    (dict(radius_face=40.0), {}, 0, _lib.PSF_EGEOM),          # image corners outside the ring
    (dict(radius_face=20.0), dict(nx=4, ny=4), 0, _lib.PSF_EGEOM),  # blocks overlap
    ({}, dict(nz=2), 0, _lib.PSF_EINVAL),                      # 2D mode with a 3D image
    (dict(gap_z=1.0), {}, 0, _lib.PSF_EUNSUPPORTED),
    ({}, {}, 7, _lib.PSF_EINVAL),
])
def test_create_rejects_bad_geometry(g, im, mode, code):
    L = _lib.load()
    h = C.c_void_p(0)
    r = L.psf_create(C.byref(_geom(**g)), C.byref(_img(**im)), mode, C.byref(h))
    assert r == code
    assert not h.value


def test_null_arguments():
    L = _lib.load()
    h = C.c_void_p(0)
    assert L.psf_create(None, None, 0, C.byref(h)) == _lib.PSF_EINVAL
    assert L.psf_sizes(None, None, None, None) == _lib.PSF_EINVAL
    assert L.psf_workspace_size(None, None, None, 1, 0, None) == _lib.PSF_EINVAL
    assert L.build_psf_sysmat(None, None, None, None, 0, None, None) == _lib.PSF_EINVAL
    assert L.project_fwd(None, None, None, None, 1, None, 0, None, None, 0, None) == _lib.PSF_EINVAL
    assert L.project_adj(None, None, None, None, 1, None, 0, None, None, None, None, 0, None) == _lib.PSF_EINVAL
    assert L.psf_check(None, None, None) == _lib.PSF_EINVAL
    L.psf_destroy(None)
