"""ctypes binding of the plain FP64 CPU oracle (``wcnst_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP path; problem descriptors are plain dicts produced by the seeded
input generators in ``paper_1810_07806_amd.workloads``.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from .build import LIB_PATH, PLAIN_LIB_PATH, SRC as _SRC, build

ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, ZERO_GRADIENT = 0, 1
ROE, LF, VANLEER = 0, 1, 2
TENO, LINEAR, JS, Z = 0, 1, 2, 3
MND, MD, HWCNS = 0, 1, 2
OK, E_INVALID, E_NONPHYSICAL, E_MAX_STEPS = 0, 1, 2, 3

_SYSTEM = {"advection": ADVECTION, "burgers": BURGERS, "euler": EULER}
_BC = {"periodic": PERIODIC, "zero_gradient": ZERO_GRADIENT, "reflect": 2, "fixed": 3}
_FLUX = {"roe": ROE, "lf": LF, "vanleer": VANLEER}
_SCHEME = {"teno": TENO, "linear": LINEAR, "js": JS, "z": Z}
_DIFF = {"mnd": MND, "md": MD, "hwcns": HWCNS}


class Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("system", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
        ("flux", ctypes.c_int), ("scheme", ctypes.c_int), ("diff", ctypes.c_int),
        ("charwise", ctypes.c_int), ("q", ctypes.c_int),
        ("gamma", ctypes.c_double), ("adv_speed", ctypes.c_double),
        ("CT", ctypes.c_double), ("C", ctypes.c_double),
        ("eps_teno", ctypes.c_double), ("eps_js", ctypes.c_double),
        ("fixed_x", (ctypes.c_double * 4) * 2), ("fixed_y", (ctypes.c_double * 4) * 2),
        ("gravity", ctypes.c_double),
        ("z_q", ctypes.c_int), ("eps_z", ctypes.c_double),
    ]


_lib = None
_plain_lib = None


def _load(path: str, plain: bool):
    """Load a build of the oracle, compiling it first if it is absent or
    older than its source."""
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(plain=plain)
    return _configure(ctypes.CDLL(path))


def lib():
    """The oracle library."""
    global _lib
    if _lib is None:
        _lib = _load(LIB_PATH, plain=False)
    return _lib


def plain_lib():
    """The same source built with every explicit product-plus-sum rounded
    twice (``-DORC_PLAIN``): used only to show that the single rounding of
    the default build does not change results beyond the parity
    tolerances."""
    global _plain_lib
    if _plain_lib is None:
        _plain_lib = _load(PLAIN_LIB_PATH, plain=True)
    return _plain_lib


def _configure(L):
    """Argument and result types of the exported functions."""
    P = ctypes.POINTER(Problem)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.orc_nvar.argtypes = [P]
    L.orc_nfaces.argtypes = [P, ctypes.c_int]
    L.orc_flag_count.argtypes = [P]
    L.orc_flag_count.restype = ctypes.c_int64
    L.orc_interp_left.argtypes = [P, dp, dp, ctypes.POINTER(ctypes.c_int)]
    L.orc_interp_left.restype = ctypes.c_double
    L.orc_candidates.argtypes = [dp, dp, dp]
    L.orc_roe_eigen.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp, dp]
    L.orc_euler_flux.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
    L.orc_num_flux.argtypes = [P, dp, dp, dp]
    L.orc_rhs.argtypes = [P, dp, dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    L.orc_max_speed.argtypes = [P, dp]
    L.orc_max_speed.restype = ctypes.c_double
    L.orc_rk3_step.argtypes = [P, dp, ctypes.c_double, ctypes.c_int64, i64p, i64p, ctypes.c_int]
    L.orc_solve.argtypes = [P, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_int64, dp, i64p, i64p, i64p, ctypes.c_int]
    return L


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def problem(desc: dict) -> Problem:
    """Translate a problem descriptor dict into the oracle's struct."""
    ndim = int(desc.get("ndim", 1))
    nx = int(desc["nx"])
    ny = int(desc.get("ny", 1)) if ndim == 2 else 1
    x0, x1 = desc.get("x0", 0.0), desc.get("x1", 1.0)
    y0, y1 = desc.get("y0", 0.0), desc.get("y1", 1.0)
    return Problem(
        ndim=ndim, system=_SYSTEM[desc.get("system", "euler")], nx=nx, ny=ny,
        dx=(x1 - x0) / nx, dy=(y1 - y0) / ny if ndim == 2 else 1.0,
        bc_x=_BC[desc.get("bc_x", "zero_gradient")], bc_y=_BC[desc.get("bc_y", "zero_gradient")],
        flux=_FLUX[desc.get("flux", "roe")], scheme=_SCHEME[desc.get("scheme", "teno")],
        diff=_DIFF[desc.get("diff", "mnd")], charwise=int(desc.get("charwise", 1)),
        q=int(desc.get("q", 6)), gamma=float(desc.get("gamma", 1.4)),
        adv_speed=float(desc.get("adv_speed", 1.0)), CT=float(desc.get("CT", 1e-5)),
        C=float(desc.get("C", 1.0)), eps_teno=float(desc.get("eps_teno", 1e-40)),
        eps_js=float(desc.get("eps_js", 1e-6)),
        fixed_x=_fixed(desc.get("fixed_x")), fixed_y=_fixed(desc.get("fixed_y")),
        gravity=float(desc.get("gravity", 0.0)),
        z_q=int(desc.get("z_q", 1)), eps_z=float(desc.get("eps_z", 1e-40)),
    )


def _fixed(states):
    """Fixed-boundary ghost states ((lo), (hi)), conserved variables in
    storage order, as the struct's double[2][4]."""
    a = ((ctypes.c_double * 4) * 2)()
    if states is not None:
        for side in range(2):
            for v, val in enumerate(states[side]):
                a[side][v] = float(val)
    return a


def nvar(p: Problem) -> int:
    return lib().orc_nvar(ctypes.byref(p))


def nfaces(p: Problem, n: int) -> int:
    return lib().orc_nfaces(ctypes.byref(p), n)


def flag_shapes(p: Problem):
    """Shapes of the x- (and y-) direction flag blocks."""
    nv = nvar(p)
    shapes = [(nv, p.ny, nfaces(p, p.nx), 2)]
    if p.ndim == 2:
        shapes.append((nv, p.nx, nfaces(p, p.ny), 2))
    return shapes


def interp_left(p: Problem, s5):
    s = np.ascontiguousarray(s5, dtype=np.float64)
    chi = np.zeros(3)
    delta = (ctypes.c_int * 3)()
    val = lib().orc_interp_left(ctypes.byref(p), _dp(s), _dp(chi), delta)
    return val, chi, np.array(list(delta), dtype=np.int32)


def candidates(s5):
    s = np.ascontiguousarray(s5, dtype=np.float64)
    cand, beta = np.zeros(3), np.zeros(3)
    lib().orc_candidates(_dp(s), _dp(cand), _dp(beta))
    return cand, beta


def roe_eigen(nv: int, gamma: float, UA, UB):
    UA = np.ascontiguousarray(UA, dtype=np.float64)
    UB = np.ascontiguousarray(UB, dtype=np.float64)
    L, R, lam = np.zeros((nv, nv)), np.zeros((nv, nv)), np.zeros(nv)
    bad = lib().orc_roe_eigen(nv, gamma, _dp(UA), _dp(UB), _dp(L), _dp(R), _dp(lam))
    return L, R, lam, bad


def euler_flux(nv: int, gamma: float, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    F = np.zeros(nv)
    lib().orc_euler_flux(nv, gamma, _dp(U), _dp(F))
    return F


def num_flux(p: Problem, UL, UR):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    F = np.zeros(nvar(p))
    lib().orc_num_flux(ctypes.byref(p), _dp(UL), _dp(UR), _dp(F))
    return F


def rhs(p: Problem, U: np.ndarray, flags: bool = False, chi: bool = False, nthreads: int = 1,
        plain: bool = False):
    """R = -(dF/dx [+ dG/dy]); optionally the cut flags and chi values
    (``plain``: from the twice-rounded build, see ``plain_lib``).

    Returns (R, flag_blocks, chi_blocks); the block lists hold one array per
    direction (see ``flag_shapes``), or are None when not requested."""
    L = plain_lib() if plain else lib()
    U = np.ascontiguousarray(U, dtype=np.float64)
    R = np.empty_like(U)
    nfl = int(L.orc_flag_count(ctypes.byref(p)))
    fl = np.zeros(nfl, dtype=np.uint8) if flags else None
    ch = np.zeros(nfl * 3, dtype=np.float64) if chi else None
    st = L.orc_rhs(ctypes.byref(p), _dp(U), _dp(R),
                       fl.ctypes.data if fl is not None else None,
                       ch.ctypes.data if ch is not None else None, int(nthreads))
    if st:
        raise ValueError(f"oracle rejected the problem (status {st})")
    fb = cb = None
    shapes = flag_shapes(p)
    if flags:
        fb, off = [], 0
        for s in shapes:
            n = int(np.prod(s))
            fb.append(fl[off:off + n].reshape(s))
            off += n
    if chi:
        cb, off = [], 0
        for s in shapes:
            n = int(np.prod(s)) * 3
            cb.append(ch[off:off + n].reshape(s + (3,)))
            off += n
    return R, fb, cb


def max_speed(p: Problem, U: np.ndarray) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_max_speed(ctypes.byref(p), _dp(U))


def rk3_step(p: Problem, U: np.ndarray, dt: float, stage_base: int = 0, nthreads: int = 1):
    """One SSP-RK3 step on a copy of U.  Returns (U_new, status, bad_stage, bad_cell)."""
    V = np.array(U, dtype=np.float64, copy=True, order="C")
    bs, bc = ctypes.c_int64(-1), ctypes.c_int64(-1)
    st = lib().orc_rk3_step(ctypes.byref(p), _dp(V), float(dt), int(stage_base),
                            ctypes.byref(bs), ctypes.byref(bc), int(nthreads))
    return V, st, bs.value, bc.value


def solve(p: Problem, U: np.ndarray, t_final: float = math.inf, cfl: float = 0.5,
          max_steps: int = 1 << 40, t0: float = 0.0, nthreads: int = 1):
    """Advance a copy of U.  Returns dict(U, t, steps, status, bad_stage, bad_cell)."""
    V = np.array(U, dtype=np.float64, copy=True, order="C")
    t = ctypes.c_double(0.0)
    steps, bs, bc = ctypes.c_int64(0), ctypes.c_int64(-1), ctypes.c_int64(-1)
    st = lib().orc_solve(ctypes.byref(p), _dp(V), float(t0), float(t_final), float(cfl),
                         int(max_steps), ctypes.byref(t), ctypes.byref(steps),
                         ctypes.byref(bs), ctypes.byref(bc), int(nthreads))
    return dict(U=V, t=t.value, steps=steps.value, status=st,
                bad_stage=bs.value, bad_cell=bc.value)
