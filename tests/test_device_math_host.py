"""CPU check of the HIP path's arithmetic: the device header compiled for the
host (tests/hostcheck) against the oracle.  Flags must be identical and the
RHS within 1e-12 -- the same bar as the GPU parity tests, without a GPU --
and, since both evaluate every value in the order of its definition, the RHS
is identical bit for bit."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1810_07806_amd import workloads as W
from parity import assert_rhs_close

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "hostcheck", "wcnst_hostcheck.cpp")
LIB = os.path.join(HERE, "hostcheck", "libhostcheck.so")
_SYS = {"advection": 0, "burgers": 1, "euler": 2}


@pytest.fixture(scope="module")
def hc():
    dev = os.path.join(ROOT, "paper_1810_07806_amd", "csrc", "wcnst_device.hpp")
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(dev)):
        # a file of this process's own (parallel test workers may rebuild at once)
        tmp = f"{LIB}.tmp{os.getpid():x}"
        cmd = ["/opt/rocm/bin/hipcc", "--offload-host-only", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-ffp-contract=off", "-I", os.path.dirname(dev), "-o", tmp, SRC]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(tmp, LIB)
    L = ctypes.CDLL(LIB)
    dp = ctypes.c_void_p
    i, d = ctypes.c_int, ctypes.c_double
    L.hc_rhs.argtypes = [i, i, i, i, i, d, d, i, i, i, i, i, d, d, d, d, d, d, dp, dp, dp, i, d]
    return L


def _hc_rhs(hc, desc, U):
    from paper_1810_07806_amd.wcnst import flag_count, split_flags
    U = np.ascontiguousarray(U, dtype=np.float64)
    R = np.zeros_like(U)
    fl = np.zeros(flag_count(desc), dtype=np.uint8)
    ndim = desc["ndim"]
    nx, ny = desc["nx"], desc["ny"] if ndim == 2 else 1
    dx = (desc["x1"] - desc["x0"]) / nx
    dy = (desc["y1"] - desc["y0"]) / ny if ndim == 2 else 1.0
    bc = {"periodic": 0, "zero_gradient": 1}
    hc.hc_rhs(ndim, _SYS[desc["system"]], {"roe": 0, "lf": 1, "vanleer": 2}[desc["flux"]], nx, ny, dx, dy,
              bc[desc["bc_x"]], bc[desc["bc_y"]], {"teno": 0, "linear": 1, "js": 2, "z": 3}[desc["scheme"]],
              int(desc["charwise"]), int(desc["q"]), desc["gamma"], desc["adv_speed"], desc["CT"],
              desc["C"], desc["eps_teno"], desc["eps_js"], U.ctypes.data, R.ctypes.data, fl.ctypes.data,
              int(desc.get("z_q", 1)), float(desc.get("eps_z", 1e-40)))
    return R, [np.asarray(b) for b in split_flags(desc, fl)]


def _compare(orc, hc, desc, U):
    Rh, fh = _hc_rhs(hc, desc, U)
    Ro, fo, _ = orc.rhs(orc.problem(desc), U, flags=True)
    for a, b in zip(fh, fo):
        assert np.array_equal(a, b), f"{int((a != b).sum())} flags differ"
    assert_rhs_close(Rh, Ro)
    # the value arithmetic follows the definitions operation for operation
    assert np.array_equal(Rh, Ro, equal_nan=True), f"max diff {np.nanmax(np.abs(Rh - Ro))}"
    return fo


@pytest.mark.parametrize("flux", ["roe", "lf", "vanleer"])
@pytest.mark.parametrize("scheme", ["teno", "linear", "js", "z"])
@pytest.mark.parametrize("charwise", [1, 0])
def test_euler1d_lines(orc, hc, flux, scheme, charwise):
    rng = np.random.default_rng(31)
    for n in (5, 37, 128):
        for bc in ("zero_gradient", "periodic"):
            d, U = W.random_tube(rng, n)
            d.update(flux=flux, scheme=scheme, charwise=charwise, bc_x=bc)
            _compare(orc, hc, d, U)


def test_scalar_lines(orc, hc):
    d, U = W.advection_sine_square(200)
    fo = _compare(orc, hc, d, U)
    assert (fo[0] != 7).any()
    rng = np.random.default_rng(2)
    for flux in ("roe", "lf"):
        d = W.describe(ndim=1, system="burgers", nx=90, bc_x="periodic", flux=flux)
        _compare(orc, hc, d, rng.normal(size=(1, 1, 90)))


@pytest.mark.parametrize("flux", ["roe", "lf", "vanleer"])
def test_euler2d_planes(orc, hc, flux):
    rng = np.random.default_rng(41)
    d, U = W.random_euler2d(rng, 33, 27)
    d.update(flux=flux)
    _compare(orc, hc, d, U)
    d, U = W.riemann2d_config3(40)
    d.update(flux=flux)
    _compare(orc, hc, d, U)


def test_state_after_steps_with_rounding_noise(orc, hc):
    """After time steps the flat regions carry rounding noise; the cut
    decisions there depend on the last bits, and still agree."""
    d, U = W.riemann2d_config3(32)
    V = orc.solve(orc.problem(d), U, cfl=0.5, max_steps=3)["U"]
    _compare(orc, hc, d, V)
    rng = np.random.default_rng(8)
    d1, U1 = W.random_tube(rng, 80)
    V1 = orc.solve(orc.problem(d1), U1, cfl=0.5, max_steps=5)["U"]
    _compare(orc, hc, d1, V1)


def test_strip_geometry_of_the_1d_kernel(hc):
    """The index map of the 1D stage kernel (one midpoint per lane, cells
    owned by the strip whose midpoints reach them), checked for every strip
    and lane of the launch: each cell once, each midpoint reported once from
    its own stencil, each cell's 2G midpoints on the lanes above it, stencils
    inside the ghost range.  MND (G = 2, 61-cell strips), MD (G = 3, 59) and
    HWCNS (G = 1, 60, node fluxes at stencil node 1)."""
    hc.hc_strip1d_check.argtypes = [ctypes.c_int, ctypes.c_int]
    for md in (0, 1, 2):
        for nx in list(range(5, 200)) + [243, 244, 245, 4096, 16384, 16385]:
            assert hc.hc_strip1d_check(nx, md) == 0, (nx, md)


def test_xcd_order_of_2d_segments(hc):
    """The 2D stage launch's workgroup-to-segment order: within each group of
    equal-height segments a permutation of the group's indices, in which the
    workgroups that share an XCD (launch index mod 8) take one contiguous run
    in launch order.  Group sizes of the 2048^2 launch (34 strips x 30 long
    and x 29 short segments) and others, with every start modulo 8."""
    hc.hc_xcd_order.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    sizes = list(range(0, 40)) + [34 * 30, 34 * 29, 1024, 2006, 4097]
    for n in sizes:
        for base in (0, 1, 5, 7, 1020, 34 * 30):
            out = np.zeros(n, dtype=np.int32)
            hc.hc_xcd_order(base, n, out.ctypes.data)
            assert sorted(out.tolist()) == list(range(base, base + n)), (base, n)
            L = np.arange(base, base + n)
            for x in range(8):
                w = out[L % 8 == x]
                if w.size:
                    assert np.all(np.diff(w) == 1), (base, n, x)
            # runs follow the order of the XCDs' first workgroups
            firsts = [out[L % 8 == (base + k) % 8][0] for k in range(min(n, 8))]
            assert firsts == sorted(firsts), (base, n)


def _plan(hc, b, d, minr):
    hc.hc_plan_strip.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    b = np.ascontiguousarray(b, dtype=np.int32)
    d = np.ascontiguousarray(d, dtype=np.uint32)
    out = np.zeros_like(b)
    hc.hc_plan_strip(b.ctypes.data, d.ctypes.data, len(d), minr, out.ctypes.data)
    return out


def test_segment_planner_keeps_a_partition_and_balances(hc):
    """The planner of the 2D stage launch's adaptive segment rows: every
    plan is a partition of the same rows (ends kept, each segment at least
    minr rows) whatever the durations; equal durations keep the layout; a
    zero duration keeps it too; and, iterated against durations drawn from a
    fixed per-row cost with a heavy band (as a shock gives), the plans
    converge to segments of about equal cost."""
    n, ty, minr = 30, 47, 11
    R = n * ty
    uniform = np.arange(n + 1) * ty
    assert np.array_equal(_plan(hc, uniform, np.full(n, 3000), minr), uniform)
    assert np.array_equal(_plan(hc, uniform, np.r_[np.full(n - 1, 3000), 0], minr), uniform)
    rng = np.random.default_rng(3)
    for _ in range(300):
        cuts = np.sort(rng.choice(np.arange(1, R), size=n - 1, replace=False))
        b = np.r_[0, cuts, R]
        d = rng.integers(1, 100000, size=n)
        out = _plan(hc, b, d, minr)
        assert out[0] == 0 and out[-1] == R
        assert np.all(np.diff(out) >= minr)
    # per-row cost 1, rows 600-700 cost 1.6; a segment also pays 3 rows of overhead
    rho = np.ones(R)
    rho[600:700] = 1.6
    cum = np.r_[0.0, np.cumsum(rho)]

    def seg_costs(b):
        return np.array([cum[b[i + 1]] - cum[b[i]] + 3.0 for i in range(n)])

    b = uniform.copy()
    before = seg_costs(b).max() / seg_costs(b).mean()
    for _ in range(12):
        b = _plan(hc, b, np.round(100 * seg_costs(b)).astype(np.uint32), minr)
    after = seg_costs(b).max() / seg_costs(b).mean()
    assert before > 1.4 and after < 1.06, (before, after)
    assert b[0] == 0 and b[-1] == R and np.all(np.diff(b) >= minr)


def test_ieee_range_predicate(hc):
    """The range test that routes a lane to the ranged reciprocal and root
    (positive x in [2^-767, 2^1022)) at its edges and on special values,
    against the same condition on the IEEE fields of x."""
    hc.hc_in_ieee_range.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lo, hi = 2.0 ** -767, 2.0 ** 1022
    edges = [lo, np.nextafter(lo, 0), np.nextafter(lo, 1), hi, np.nextafter(hi, 0), np.nextafter(hi, np.inf),
             1.0, 0.5, 1e-300, 1e-231, 2e-231, 3e300, 5e307, np.finfo(float).max, np.finfo(float).tiny, 5e-324,
             0.0, -0.0, np.inf, -np.inf, np.nan, -1.0, -lo, -1e-300]
    rng = np.random.default_rng(5)
    bits = rng.integers(0, 2 ** 63, size=100000, dtype=np.int64).astype(np.uint64) | \
        (rng.integers(0, 2, size=100000).astype(np.uint64) << np.uint64(63))
    x = np.concatenate([np.array(edges, dtype=np.float64), bits.view(np.float64)])
    out = np.zeros(x.size, dtype=np.uint8)
    hc.hc_in_ieee_range(x.ctypes.data, out.ctypes.data, x.size)
    with np.errstate(invalid="ignore"):
        want = (x >= lo) & (x < hi)
    assert np.array_equal(out.astype(bool), want)
    assert want[:6].tolist() == [True, False, True, False, True, False]
