"""CPU checks of the C ABI library: it loads, exports every symbol that
include/sme.h declares, validates meshes, and carries the basis tensors the
oracle computes independently (no GPU work is launched here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import tensors as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sme.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sme_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def sme():
    from paper_2601_04826_amd import sme as m

    return m


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("sme_init", "sme_step", "sme_run", "sme_eigmax", "sme_set_state", "sme_get_state",
                 "sme_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(sme):
    lib = ctypes.CDLL(sme.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(sme.EXPORTS) == declared_functions()


@pytest.mark.parametrize("level", range(0, 9))
def test_library_tensors_equal_exact_rationals(sme, level):
    got = sme.sme_basis_tensors(level)
    want = T.tensors(level)
    for key in ("M", "A", "B", "K"):
        np.testing.assert_allclose(got[key], want[key], rtol=2.3e-16, atol=0)


def test_layout_and_validation(sme):
    m, _ = sme.make_mesh(dict(kind="2d", nx=10, ny=7, x0=0, x1=1, y0=0, y1=1, bc=("wall",) * 4))
    assert sme.sme_layout(3, m) == (9, 70, 256)
    m1, _ = sme.make_mesh(dict(kind="1d", nx=12, x0=0, x1=1, bc=("extrap", "extrap")))
    assert sme.sme_layout(8, m1) == (10, 12, 256)
    with pytest.raises(sme.SmeError) as e:
        sme.sme_layout(9, m)
    assert e.value.code == sme.SME_EINVAL
    bad, _ = sme.make_mesh(dict(kind="1d", nx=12, x0=0, x1=1, bc=("periodic", "extrap")))
    with pytest.raises(sme.SmeError):
        sme.sme_layout(1, bad)
    vert = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    t, _ = sme.make_mesh(dict(kind="tri", vert=vert, tri=np.array([[0, 1, 2]], dtype=np.int32)))
    assert sme.sme_layout(2, t) == (7, 1, 256)
    # at most 2^28 triangles (the triangle kernel's 32-bit byte offsets within a
    # field); only the count is read when the layout is asked for
    t.n_tri = 1 << 28
    assert sme.sme_layout(0, t) == (3, 1 << 28, 1 << 28)
    t.n_tri = (1 << 28) + 1
    with pytest.raises(sme.SmeError) as e:
        sme.sme_layout(0, t)
    assert e.value.code == sme.SME_EINVAL


@pytest.mark.parametrize("mesh", [
    dict(kind="1d", nx=0, x0=0, x1=1, bc=("wall", "wall")),
    dict(kind="1d", nx=5, x0=1, x1=1, bc=("wall", "wall")),
    dict(kind="2d", nx=0, ny=4, x0=0, x1=1, y0=0, y1=1, bc=("wall",) * 4),
    dict(kind="2d", nx=4, ny=0, x0=0, x1=1, y0=0, y1=1, bc=("wall",) * 4),
    dict(kind="2d", nx=4, ny=4, x0=0, x1=1, y0=1, y1=0, bc=("wall",) * 4),
    dict(kind="2d", nx=4, ny=4, x0=0, x1=1, y0=0, y1=1, bc=("wall", "wall", "periodic", "wall")),
])
def test_layout_rejects_empty_and_invalid_meshes(sme, mesh):
    m, _ = sme.make_mesh(mesh)
    with pytest.raises(sme.SmeError) as e:
        sme.sme_layout(1, m)
    assert e.value.code == sme.SME_EINVAL


def test_workspace_size(sme):
    m, _ = sme.make_mesh(dict(kind="2d", nx=300, ny=7, x0=0, x1=1, y0=0, y1=1, bc=("wall",) * 4))
    nf, nc, st = sme.sme_layout(2, m)
    assert (nf, nc, st) == (7, 2100, 2304)
    ws = sme.sme_workspace_size(2, m)
    assert st * 8 <= ws < st * 8 + 16384          # bathymetry plus a few small tables
    vert = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    t, _ = sme.make_mesh(dict(kind="tri", vert=vert, tri=np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)))
    wt = sme.sme_workspace_size(3, t)
    assert wt >= 256 * 8 + 3 * 256 * (4 + 24) + 2 * 2 * 8
    # the second-order scheme on a structured grid computes its slopes inside
    # the stages up to level 6; above, it keeps 2 axes x (nfields + 1) of them
    w2 = sme.sme_workspace_size(2, m, sme.make_params(order=2))
    assert w2 == ws
    nf7, _, st7 = sme.sme_layout(7, m)
    w7 = sme.sme_workspace_size(7, m, sme.make_params(order=2)) - sme.sme_workspace_size(7, m)
    assert w7 == 2 * (nf7 + 1) * st7 * 8
    m1, _ = sme.make_mesh(dict(kind="1d", nx=1000, x0=0, x1=1, bc=("wall", "wall")))
    nf1, _, st1 = sme.sme_layout(3, m1)
    w1 = sme.sme_workspace_size(3, m1, sme.make_params(order=2)) - sme.sme_workspace_size(3, m1)
    assert w1 == (nf1 + 1) * st1 * 8


def test_strerror(sme):
    assert sme.lib().sme_strerror(sme.SME_ENONPHYS) == b"non-physical state"
    assert sme.lib().sme_strerror(0) == b"ok"
