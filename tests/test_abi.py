"""The C-ABI library loads and exports every symbol its header declares; the
host-side descriptor validation behaves as documented (no GPU work)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wcnst.h")


def _lib():
    from paper_1810_07806_amd import build, wcnst
    if not os.path.exists(build.LIB_PATH):
        build.build()
    return wcnst, wcnst.lib()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wcnst_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("wcnst_create", "wcnst_rhs", "wcnst_step", "wcnst_solve", "wcnst_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    wc, L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(wc.EXPORTS)


def test_struct_layout_matches_header():
    wc, L = _lib()
    d = wc.Desc()
    assert L.wcnst_desc_init(ctypes.byref(d)) == 0
    assert d.struct_size == ctypes.sizeof(wc.Desc)
    assert (d.q, d.CT, d.C, d.eps_teno, d.gamma) == (6, 1e-5, 1.0, 1e-40, 1.4)
    assert (d.z_q, d.eps_z) == (1, 1e-40)


def _ws(wc, L, **kw):
    base = dict(ndim=1, system="euler", nx=64)
    base.update(kw)
    d = wc.make_desc(base)
    n = ctypes.c_size_t(0)
    return L.wcnst_workspace_size(ctypes.byref(d), ctypes.byref(n)), n.value


def test_workspace_size_and_validation():
    wc, L = _lib()
    st, n = _ws(wc, L, nx=100)
    assert st == 0 and n >= 2 * 3 * 100 * 8
    st, n2 = _ws(wc, L, ndim=2, nx=2048, ny=2048)
    assert st == 0 and n2 >= 2 * 4 * 2048 * 2048 * 8
    st, _ = _ws(wc, L, nx=100, diff="md")
    assert st == 0
    st, _ = _ws(wc, L, nx=100, diff="md", scheme="z", z_q=2)
    assert st == 0
    bad = [dict(nx=4), dict(ndim=3), dict(ndim=2, system="advection", nx=8, ny=8),
           dict(ndim=2, nx=8, ny=4), dict(gamma=1.0), dict(CT=0.5), dict(q=0),
           dict(x0=1.0, x1=1.0), dict(ndim=2, nx=8, ny=8, diff="md"),
           dict(system="advection", flux="vanleer"), dict(ndim=2, nx=8, ny=8, diff="hwcns"),
           dict(system="advection", bc_x="reflect"), dict(gravity=1.0),
           dict(scheme="z", z_q=0), dict(scheme="z", z_q=5),
           dict(scheme="z", eps_z=0.0)]
    for kw in bad:
        st, _ = _ws(wc, L, **kw)
        assert st == wc.E_INVALID_ARG, kw
        assert L.wcnst_last_error()


def test_binding_refuses_a_missing_library(tmp_path):
    import importlib
    from paper_1810_07806_amd import wcnst
    saved = wcnst._lib
    try:
        wcnst._lib = None
        with pytest.raises(RuntimeError):
            wcnst.lib(str(tmp_path / "absent.so"))
    finally:
        wcnst._lib = saved
    importlib.reload  # keep the import used


def test_batches_and_pools_refuse_the_md_difference():
    """Batched and pooled solves run the MND stage kernels only; an MD
    descriptor is refused at sizing time with a message, before any device
    work."""
    wc, L = _lib()
    descs = (wc.Desc * 2)(*[wc.make_desc(dict(ndim=1, system="euler", nx=64, diff=df)) for df in ("mnd", "md")])
    n = ctypes.c_size_t(0)
    L.wcnst_batch_workspace_size.argtypes = [ctypes.POINTER(wc.Desc), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    assert L.wcnst_batch_workspace_size(descs, 1, ctypes.byref(n)) == 0
    assert L.wcnst_batch_workspace_size(descs, 2, ctypes.byref(n)) == wc.E_INVALID_ARG
    assert b"MND" in L.wcnst_last_error()
    # an empty batch is refused, not sized
    assert L.wcnst_batch_workspace_size(descs, 0, ctypes.byref(n)) == wc.E_INVALID_ARG
    assert L.wcnst_last_error()


def test_batches_and_pools_take_the_z_weights_with_one_scheme():
    """Batches take the WCNS-Z weights like the other schemes; a batch that
    mixes schemes, or Z powers, is refused at sizing time."""
    wc, L = _lib()
    n = ctypes.c_size_t(0)
    L.wcnst_batch_workspace_size.argtypes = [ctypes.POINTER(wc.Desc), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    same = (wc.Desc * 2)(*[wc.make_desc(dict(ndim=1, system="euler", nx=64, scheme="z")) for _ in range(2)])
    assert L.wcnst_batch_workspace_size(same, 2, ctypes.byref(n)) == 0 and n.value > 0
    mixed = (wc.Desc * 2)(*[wc.make_desc(dict(ndim=1, system="euler", nx=64, scheme=sc)) for sc in ("teno", "z")])
    assert L.wcnst_batch_workspace_size(mixed, 2, ctypes.byref(n)) == wc.E_INVALID_ARG
    assert b"differ" in L.wcnst_last_error()
    other_q = (wc.Desc * 2)(*[wc.make_desc(dict(ndim=1, system="euler", nx=64, scheme="z", z_q=zq)) for zq in (1, 2)])
    assert L.wcnst_batch_workspace_size(other_q, 2, ctypes.byref(n)) == wc.E_INVALID_ARG


def test_noalloc_solve_refuses_grids_beyond_its_scratch():
    """wcnst_solve_noalloc checks the grid against its static scratch before
    any device work: 1024 x 1024 2D Euler needs 2 x 32 MiB + 256 bytes,
    beyond the 64 MiB limit; a bad descriptor is refused the same way."""
    wc, L = _lib()
    d = wc.make_desc(dict(ndim=2, system="euler", nx=1024, ny=1024))
    U = ctypes.c_void_p(16)  # never dereferenced: the call fails first
    assert L.wcnst_solve_noalloc(ctypes.byref(d), None, U, 1.0, 0.5, 1, None, None) == wc.E_INVALID_ARG
    assert b"scratch" in L.wcnst_last_error()
    bad = wc.make_desc(dict(ndim=1, system="euler", nx=4))
    assert L.wcnst_solve_noalloc(ctypes.byref(bad), None, U, 1.0, 0.5, 1, None, None) == wc.E_INVALID_ARG
