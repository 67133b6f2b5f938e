"""GPU (HIP, gfx950) path against the CPU oracle, through the C ABI.

RHS within 1e-12 (per-component inf-norm relative), stencil-cut flags
identical outside the 1e-12 C_T tie band, fields within 1e-10 after 100
steps, at sizes spanning several 61-column strips and row segments with
ragged tails, plus the full 2048^2 four-quadrant case.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

from paper_1810_07806_amd import workloads as W
from cases import CASES_1D, CASES_2D, euler1d_cases, euler2d_cases, extreme_density_cases, scalar_cases
from parity import FIELD_TOL, assert_rhs_close, check_flags, rel_inf_err, rhs_mask_from_flips

pytestmark = pytest.mark.gpu

NTHREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1810_07806_amd import wcnst
    wcnst.lib()
    return T


def _solver(desc):
    from paper_1810_07806_amd.wcnst import Solver
    return Solver(desc)


def _rhs_case(orc, torch, desc, U, name):
    _say(f"rhs {name} {desc.get('system')} {desc.get('ndim')}D nx={desc['nx']} ny={desc.get('ny', 1)} "
         f"flux={desc.get('flux')} scheme={desc.get('scheme')} charwise={desc.get('charwise')}")
    from paper_1810_07806_amd.wcnst import split_flags
    s = _solver(desc)
    Ug = s.new_state(U)
    Rg, fg = s.rhs(Ug, flags=True)
    torch.cuda.synchronize()
    Rg = Rg.cpu().numpy()
    fg = [b.cpu().numpy() for b in split_flags(desc, fg)]
    p = orc.problem(desc)
    Ro, fo, co = orc.rhs(p, U, flags=True, chi=True, nthreads=NTHREADS)
    flips = check_flags(fg, fo, co, desc.get("CT", 1e-5))
    ny, nx = Ro.shape[1], Ro.shape[2]
    keep = rhs_mask_from_flips((ny, nx), flips, desc.get("ndim", 1))
    err = assert_rhs_close(Rg, Ro, keep)
    s.close()
    return err, fo


@pytest.mark.parametrize("kw", CASES_1D, ids=lambda k: "-".join(str(v) for v in k.values()))
def test_rhs_euler1d(orc, torch, kw):
    for name, d, U in euler1d_cases(kw):
        _, fo = _rhs_case(orc, torch, d, U, name)
    # both kept and cut stencils occurred on the last (largest) case
    if kw["scheme"] == "teno":
        assert (fo[0] == 7).any() and (fo[0] != 7).any()


def test_rhs_shu_osher_2048(orc, torch):
    d, U = W.shu_osher(2048)
    _rhs_case(orc, torch, d, U, "shu-osher")


def test_rhs_scalar(orc, torch):
    """Advection (the config 1 state and a 5-cell line) and Burgers (Roe
    speed and local Lax-Friedrichs)."""
    for name, d, U in scalar_cases():
        _, fo = _rhs_case(orc, torch, d, U, name)
        if name == "advection200":
            assert (fo[0] != 7).any()


@pytest.mark.parametrize("kw", CASES_2D, ids=lambda k: "-".join(str(v) for v in k.values()))
def test_rhs_euler2d(orc, torch, kw):
    for name, d, U in euler2d_cases(kw):
        _rhs_case(orc, torch, d, U, name)


def test_rhs_config3_full_size(orc, torch):
    """The 2048^2 four-quadrant state in the launch configuration of the
    benchmark; the whole field is compared."""
    d, U = W.riemann2d_config3(2048)
    _rhs_case(orc, torch, d, U, "config3-2048")


# ------------------------------------------------------------ time stepping

def _solve_case(orc, torch, desc, U, t_final, steps, name, tol=FIELD_TOL):
    _say(f"solve {name} t_final={t_final} steps={steps}")
    s = _solver(desc)
    Ug = s.new_state(U)
    tg, ng = s.solve(Ug, t_final=t_final, cfl=0.5, max_steps=steps)
    Ugh = Ug.cpu().numpy()
    r = orc.solve(orc.problem(desc), U, t_final=t_final, cfl=0.5, max_steps=steps, nthreads=NTHREADS)
    assert r["status"] == 0
    assert ng == r["steps"], (ng, r["steps"])
    assert abs(tg - r["t"]) <= 1e-12 * max(1.0, abs(r["t"]))
    err = rel_inf_err(Ugh, r["U"])
    assert (err <= tol).all(), f"{name}: field error {err}"
    assert np.isfinite(Ugh).all()
    if desc.get("system", "euler") == "euler":
        assert Ugh[0].min() > 0.0
    s.close()
    return Ugh


def test_solve_advection_config1(orc, torch):
    d, U = W.advection_sine_square(200)
    _solve_case(orc, torch, d, U, 2.0, 1 << 40, "advection-t2")


def test_solve_shu_osher_100_steps(orc, torch):
    d, U = W.shu_osher(2048)
    _solve_case(orc, torch, d, U, np.inf, 100, "shu-osher-100")


def test_solve_shu_osher_to_final_time(orc, torch):
    """Config 2 (the Shu-Osher problem of Sec. 3.5, N = 2048) to its final
    time t = 1.8: about 3400 steps, the step count, time and field against
    the oracle."""
    d, U = W.shu_osher(2048)
    _solve_case(orc, torch, d, U, 1.8, 1 << 40, "shu-osher-t1.8")


@pytest.mark.parametrize("kw", [dict(), dict(flux="lf", charwise=0, bc_x="periodic"), dict(flux="vanleer"),
                                dict(scheme="js"), dict(scheme="z", z_q=2), dict(bc_x="reflect")],
                         ids=["roe-teno", "lf-componentwise-periodic", "vanleer", "js", "wcns-z", "walls"])
def test_solve_1d_latency_mode_and_wide_lines(orc, torch, kw):
    """1D Euler stages over at most 256 strips run three wavefronts per
    strip (the latency mode), longer lines one: both through whole solves
    against the oracle, at 5 and 61 cells (one strip), 1000 cells (17
    strips) and 16000 cells (263 strips, the one-wavefront kernel)."""
    rng = np.random.default_rng(11)
    for n, steps in ((5, 40), (61, 40), (1000, 40), (16000, 12)):
        d, U = W.random_tube(rng, n)
        d.update(kw)
        _solve_case(orc, torch, d, U, np.inf, steps, f"tube{n}-{kw}")


def test_solve_tube_to_time(orc, torch):
    rng = np.random.default_rng(3)
    d, U = W.random_tube(rng, 257)
    _solve_case(orc, torch, d, U, 0.05, 1 << 40, "tube-to-t")


def test_solve_vanleer_sod_and_quadrants(orc, torch):
    """The van Leer splitting through whole solves: the Sod tube to t = 0.2
    and 60 steps of the four-quadrant problem at 128^2."""
    d, U = W.sod(300, flux="vanleer")
    _solve_case(orc, torch, d, U, 0.2, 1 << 40, "sod-vanleer")
    d, U = W.riemann2d_config3(128)
    d["flux"] = "vanleer"
    _solve_case(orc, torch, d, U, np.inf, 60, "quadrants-vanleer-128")


def test_solve_config3_100_steps(orc, torch):
    d, U = W.riemann2d_config3(128)
    _solve_case(orc, torch, d, U, np.inf, 100, "config3-128-100")


def test_solve_random2d_periodic_100_steps(orc, torch):
    rng = np.random.default_rng(11)
    d, U = W.random_euler2d(rng, 96, 70)
    d.update(bc_x="periodic", bc_y="periodic")
    _solve_case(orc, torch, d, U, np.inf, 100, "quad-periodic-100")


def test_step_api_matches_oracle_step(orc, torch):
    rng = np.random.default_rng(4)
    d, U = W.random_euler2d(rng, 64, 48)
    _say("step api")
    s = _solver(d)
    Ug = s.new_state(U)
    s.step(Ug, dt=1e-3)
    s.step(Ug, dt=0.0, cfl=0.4)
    st = s.status()
    p = orc.problem(d)
    V, ok, _, _ = orc.rk3_step(p, U, 1e-3)
    dt2 = 0.4 / orc.max_speed(p, V)
    V, ok2, _, _ = orc.rk3_step(p, V, dt2, stage_base=3)
    assert ok == 0 and ok2 == 0 and st["status"] == 0 and st["steps"] == 2
    assert abs(st["t"] - (1e-3 + dt2)) <= 1e-14
    assert (rel_inf_err(Ug.cpu().numpy(), V) <= FIELD_TOL).all()


def test_nonphysical_state_reported_like_oracle(orc, torch):
    from paper_1810_07806_amd.wcnst import WcnstError
    rng = np.random.default_rng(9)
    d, U = W.random_tube(rng, 64)
    U = U.copy()
    U[0, 0, 17] = -0.5
    _say("nonphysical")
    r = orc.solve(orc.problem(d), U, t_final=0.1, cfl=0.5)
    s = _solver(d)
    Ug = s.new_state(U)
    with pytest.raises(WcnstError) as ei:
        s.solve(Ug, t_final=0.1, cfl=0.5)
    assert ei.value.status == 2
    st = s.status()
    assert (st["bad_stage"], st["bad_cell"]) == (r["bad_stage"], r["bad_cell"])


def test_config3_diagonal_symmetry_bitwise(torch):
    """Identical arithmetic in the x and y sweeps keeps the symmetric state
    of Sec. 3.6.1 symmetric bit for bit."""
    d, U = W.riemann2d_config3(256)
    _say("symmetry 256 x 30 steps")
    s = _solver(d)
    Ug = s.new_state(U)
    s.solve(Ug, t_final=np.inf, cfl=0.5, max_steps=30)
    V = Ug.cpu().numpy()
    assert np.array_equal(V[0], V[0].T) and np.array_equal(V[3], V[3].T)
    assert np.array_equal(V[1], V[2].T)


def test_repeat_runs_are_bitwise_identical(torch):
    rng = np.random.default_rng(21)
    d, U = W.random_euler2d(rng, 150, 90)
    _say("determinism")
    outs = []
    for _ in range(2):
        s = _solver(d)
        Ug = s.new_state(U)
        s.solve(Ug, t_final=np.inf, cfl=0.5, max_steps=20)
        outs.append(Ug.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_bitwise_agreement_with_oracle(orc, torch):
    """Both sides evaluate every value in the order of its definition with
    IEEE division and square root, so the RHS and whole trajectories agree
    bit for bit (the stated tolerances are looser than this)."""
    d, U = W.riemann2d_config3(192)
    _say("bitwise rhs config3-192")
    s = _solver(d)
    Ug = s.new_state(U)
    Rg = s.rhs(Ug).cpu().numpy()
    Ro, _, _ = orc.rhs(orc.problem(d), U, nthreads=NTHREADS)
    assert np.array_equal(Rg, Ro)
    _say("bitwise 60 steps config3-192")
    s.solve(Ug, t_final=np.inf, cfl=0.5, max_steps=60)
    r = orc.solve(orc.problem(d), U, cfl=0.5, max_steps=60, nthreads=NTHREADS)
    assert np.array_equal(Ug.cpu().numpy(), r["U"])
    rng = np.random.default_rng(77)
    d1, U1 = W.random_tube(rng, 300)
    _say("bitwise tube to t=0.1")
    s1 = _solver(d1)
    V = s1.new_state(U1)
    s1.solve(V, t_final=0.1, cfl=0.5)
    r1 = orc.solve(orc.problem(d1), U1, t_final=0.1, cfl=0.5)
    assert np.array_equal(V.cpu().numpy(), r1["U"])


def test_launch_shape_does_not_change_results(torch):
    """Segment heights (including ragged last segments and 1-row segments)
    only change the work decomposition: results are bit-identical."""
    rng = np.random.default_rng(5)
    d, U = W.random_euler2d(rng, 140, 75)
    outs = []
    for rows in (35, 1, 2, 3, 16, 75, 200):
        _say(f"launch shape rows={rows}")
        s = _solver(d)
        s.set_tuning(rows)
        Ug = s.new_state(U)
        R = s.rhs(Ug).cpu().numpy()
        s.solve(Ug, t_final=np.inf, cfl=0.5, max_steps=5)
        outs.append((R, Ug.cpu().numpy()))
    for R, V in outs[1:]:
        assert np.array_equal(R, outs[0][0]) and np.array_equal(V, outs[0][1])


def test_rows_autotuner_keeps_state_and_results(torch):
    """The 2D segment-height autotuner times its candidates on a copy of the
    state and restores the solver's step record; the tuned solve gives the
    bits of the default shape, and set_tuning(0) restores that shape."""
    from paper_1810_07806_amd import autotune
    d, U = W.riemann2d_config3(300)
    s = _solver(d)
    default = s.stage_shape()
    Ug = s.new_state(U)
    U_in = Ug.clone()
    _say("rows autotuner on 300^2")
    res = autotune.tune_rows(s, Ug, steps=1, rows=(0, 8, 24, 300))
    assert [r["rows"] for r in res["table"]] == [0, 8, 24, 300]
    assert res["rows"] in (0, 8, 24, 300) and torch.equal(Ug, U_in)
    st = s.status()
    assert st["t"] == 0.0 and st["steps"] == 0 and st["status"] == 0
    s.solve(Ug, t_final=np.inf, cfl=0.5, max_steps=6)
    ref = _solver(d)
    V = ref.new_state(U)
    ref.solve(V, t_final=np.inf, cfl=0.5, max_steps=6)
    assert torch.equal(Ug, V)
    s.set_tuning(0)
    assert s.stage_shape() == default


def test_solve_config3_full_size_100_steps(orc, torch):
    """The 2048^2 benchmark problem in the benchmark's launch configuration:
    100 SSP-RK3 steps against the oracle (run on the host cores) over the
    whole field, the 1e-10 field criterion at the benchmark's size."""
    d, U = W.riemann2d_config3(2048)
    _solve_case(orc, torch, d, U, np.inf, 100, "config3-2048-100-steps")


def test_config3_full_size_200_steps_symmetric(torch):
    """At the full size and step count of the benchmark, where the oracle is
    too slow to follow, a property that holds at any size: the diagonal
    symmetry of the initial state survives bit for bit, and the state stays
    physical with a decreasing-or-bounded CFL speed."""
    d, U = W.riemann2d_config3(2048)
    _say("symmetry 2048 x 200 steps")
    s = _solver(d)
    Ug = s.new_state(U)
    t, n = s.solve(Ug, t_final=np.inf, cfl=0.5, max_steps=200)
    assert n == 200 and s.status()["status"] == 0
    V = Ug.cpu().numpy()
    assert np.array_equal(V[0], V[0].T) and np.array_equal(V[3], V[3].T)
    assert np.array_equal(V[1], V[2].T)
    assert np.isfinite(V).all() and (V[0] > 0).all()


@pytest.mark.parametrize("config", [3, 6])
def test_lax_liu_configurations_to_paper_time(orc, torch, config):
    """Configurations 3 and 6 of Sec. 3.6 run to the paper's final time
    t = 0.3 at 256^2 (a few hundred steps): the GPU state equals the
    oracle's within the field tolerance, stays physical, and the step
    counts agree."""
    d, U = (W.riemann2d_config3 if config == 3 else W.riemann2d_config6)(256)
    _solve_case(orc, torch, d, U, 0.3, 1 << 40, f"lax-liu-{config}-t0.3")


@pytest.mark.parametrize("bc", ["zero_gradient", "periodic", "reflect", "fixed"])
def test_free_stream_rhs_is_exactly_zero(orc, torch, bc):
    """Degenerate input: a uniform state (moving, except against walls) has
    an RHS of exactly zero on every side type, in 1D and 2D, on the GPU as
    in the oracle; with fixed sides holding the same state."""
    g = 1.4
    u = 0.0 if bc == "reflect" else 0.3
    v = 0.0 if bc == "reflect" else -0.2
    st2 = W.conserved_2d(0.9, u, v, 1.1, g)
    st1 = W.conserved_1d(0.9, u, 1.1, g)
    fixed2 = (tuple(st2), tuple(st2))
    fixed1 = (tuple(st1), tuple(st1))
    for d, U in (
        (W.describe(ndim=2, system="euler", nx=70, ny=40, bc_x=bc, bc_y=bc, fixed_x=fixed2, fixed_y=fixed2),
         np.broadcast_to(np.asarray(st2)[:, None, None], (4, 40, 70)).copy()),
        (W.describe(ndim=1, system="euler", nx=130, bc_x=bc, fixed_x=fixed1),
         np.broadcast_to(np.asarray(st1)[:, None, None], (3, 1, 130)).copy()),
    ):
        _say(f"free stream {d['ndim']}D {bc}")
        s = _solver(d)
        Rg = s.rhs(s.new_state(U)).cpu().numpy()
        s.close()
        Ro, _, _ = orc.rhs(orc.problem(d), U)
        assert np.abs(Ro).max() == 0.0
        assert np.abs(Rg).max() == 0.0


@pytest.mark.parametrize("flux", ["roe", "lf"])
@pytest.mark.parametrize("scale", ["crossing-2^-767", "1e-300", "1e150"])
def test_rhs_extreme_density_scales(orc, torch, flux, scale):
    """Densities far from order one, where the kernels' reciprocals and roots
    of the Roe averages and fluxes switch between the hardware sequences and
    the IEEE operations (below 2^-767 only the latter give IEEE results):
    the RHS still equals the oracle's bit for bit, in 1D and 2D."""
    for name, d, U in extreme_density_cases(flux, scale):
        _rhs_case(orc, torch, d, U, name)
        s = _solver(d)
        Rg = s.rhs(s.new_state(U)).cpu().numpy()
        s.close()
        Ro, _, _ = orc.rhs(orc.problem(d), U, nthreads=NTHREADS)
        assert np.isfinite(Ro).all()
        assert np.array_equal(Rg, Ro)


def _host_dt_1d(U, d, cfl):
    """cfl / max over cells of (|u| + c)/dx, in the kernels' order of
    operations (1/rho once; p = (gamma - 1)(E - rho u^2 / 2))."""
    g, dx = d["gamma"], (d["x1"] - d["x0"]) / d["nx"]
    r, m, e = U[0].ravel(), U[1].ravel(), U[2].ravel()
    ir = 1.0 / r
    p = (g - 1.0) * (e - 0.5 * m * m * ir)
    a = np.sqrt(g * p * ir)
    return cfl / ((np.abs(m * ir) + a) / dx).max()


def test_cfl_reduction_over_many_waves(orc, torch):
    """The fused CFL reduction of the third stage on a 2^22-cell line
    (68 760 wavefronts on one step record): the time after two steps is
    t1 + cfl / S(U^1), with S the maximum cell speed of the state after the
    first step, recomputed on the host (the host formula is the oracle's
    step rule: checked on a 2048-cell line first)."""
    ds, Us = W.shu_osher(2048)
    assert orc.solve(orc.problem(ds), Us, cfl=0.5, max_steps=1)["t"] == _host_dt_1d(Us, ds, 0.5)
    d, U = W.shu_osher(1 << 22)
    _say("cfl reduction shu-osher 2^22 cells")
    s = _solver(d)
    V = s.new_state(U)
    t1, n1 = s.solve(V, t_final=np.inf, cfl=0.5, max_steps=1)
    U1 = V.cpu().numpy()
    V2 = s.new_state(U)
    s.reset(0.0, 0)
    t2, n2 = s.solve(V2, t_final=np.inf, cfl=0.5, max_steps=2)
    s.close()
    assert n1 == 1 and n2 == 2
    assert t1 == _host_dt_1d(U, d, 0.5)
    assert t2 == t1 + _host_dt_1d(U1, d, 0.5)


def test_degenerate_solve_calls(orc, torch):
    """Calls that must not advance the state: t_final already reached (zero,
    negative, the current time), zero steps with t_final = inf; zero steps
    short of a finite t_final report WCNST_E_MAX_STEPS; invalid cfl, t_final
    NaN and negative max_steps are refused before any launch.  The state is
    unchanged bit for bit, as in the oracle."""
    from paper_1810_07806_amd.wcnst import WcnstError
    d, U = W.sod(101)
    _say("degenerate solve calls sod101")
    s = _solver(d)
    V = s.new_state(U)
    for tf in (0.0, -1.0):
        assert s.solve(V, t_final=tf, cfl=0.5) == (0.0, 0)
        assert np.array_equal(V.cpu().numpy(), U)
        r = orc.solve(orc.problem(d), U, t_final=tf, cfl=0.5)
        assert r["steps"] == 0 and np.array_equal(r["U"], U)
    assert s.solve(V, t_final=np.inf, cfl=0.5, max_steps=0) == (0.0, 0)
    assert np.array_equal(V.cpu().numpy(), U)
    with pytest.raises(WcnstError) as e:
        s.solve(V, t_final=0.1, cfl=0.5, max_steps=0)
    assert e.value.status == 3
    for kw in (dict(t_final=0.1, cfl=0.0), dict(t_final=0.1, cfl=-0.5), dict(t_final=np.nan, cfl=0.5),
               dict(t_final=0.1, cfl=0.5, max_steps=-1)):
        with pytest.raises(WcnstError) as e:
            s.solve(V, **kw)
        assert e.value.status == 1, kw
    assert np.array_equal(V.cpu().numpy(), U)
    t, n = s.solve(V, t_final=0.05, cfl=0.5)
    Vh = V.cpu().numpy()
    assert n > 0 and abs(t - 0.05) <= 1e-12 * 0.05
    # a second call to the time already reached does nothing
    assert s.solve(V, t_final=0.05, cfl=0.5) == (t, 0)
    assert np.array_equal(V.cpu().numpy(), Vh)
    s.close()
    r = orc.solve(orc.problem(d), U, t_final=0.05, cfl=0.5)
    assert r["steps"] == n and r["t"] == t and np.array_equal(r["U"], Vh)


def test_rhs_16384_squared_sampled_windows(orc, torch):
    """A 16384^2 grid (8.6 GB per state: variable planes start past 2^32
    bytes): the GPU RHS on sampled 32 x 32 windows, at the corners, edges
    and inside, against the oracle run on each window alone.  A cell's RHS
    depends only on the four cells on each side along its x and y lines, so
    window cells at least 4 cells from every window edge that is not a
    domain edge must agree (same spacing, same zero-gradient sides)."""
    n, w = 16384, 32
    _say(f"rhs {n}^2 sampled windows")
    d, U = W.ripples_2d(n, n)
    s = _solver(d)
    Ug = s.new_state(U)
    Rg = s.rhs(Ug)
    torch.cuda.synchronize()
    del Ug
    h = 1.0 / n
    corners = [(0, 0), (0, n - w), (n - w, 0), (n - w, n - w), (8180, 8180), (12345, 3210), (16000, 9000),
               (5000, n - w), (n - w, 7777)]
    for y0, x0 in corners:
        win = np.ascontiguousarray(U[:, y0:y0 + w, x0:x0 + w])
        dw = W.describe(ndim=2, system="euler", nx=w, ny=w, x0=x0 * h, x1=(x0 + w) * h, y0=y0 * h, y1=(y0 + w) * h)
        Ro, _, _ = orc.rhs(orc.problem(dw), win, nthreads=NTHREADS)
        ylo = 0 if y0 == 0 else 4
        yhi = w if y0 + w == n else w - 4
        xlo = 0 if x0 == 0 else 4
        xhi = w if x0 + w == n else w - 4
        got = Rg[:, y0 + ylo:y0 + yhi, x0 + xlo:x0 + xhi].cpu().numpy()
        want = Ro[:, ylo:yhi, xlo:xhi]
        scale = np.abs(want).reshape(4, -1).max(axis=1)[:, None, None]
        assert (np.abs(got - want) <= 1e-12 * scale).all(), (y0, x0)
        assert np.array_equal(got, want), (y0, x0)
    s.close()


def test_rhs_1d_2e28_cells_sampled_windows(orc, torch):
    """A 1D line of 2^28 cells (6.4 GB per state: the third variable plane
    starts past 2^32 bytes): the GPU RHS on sampled 64-cell windows at both
    ends and inside against the oracle run on each window alone, with the
    4-cell margin at window edges that are not domain edges."""
    n, w = 1 << 28, 64
    _say(f"rhs 1D {n} cells sampled windows")
    d, U = W.ripples_1d(n)
    s = _solver(d)
    Ug = s.new_state(U)
    Rg = s.rhs(Ug)
    torch.cuda.synchronize()
    del Ug
    h = 1.0 / n
    for x0 in (0, n - w, n // 2 - 17, 150_000_000, int(0.55 * n) - w // 2, 3 * (n // 4) + 5):
        win = np.ascontiguousarray(U[:, :, x0:x0 + w])
        dw = W.describe(ndim=1, system="euler", nx=w, x0=x0 * h, x1=(x0 + w) * h)
        Ro, _, _ = orc.rhs(orc.problem(dw), win)
        lo = 0 if x0 == 0 else 4
        hi = w if x0 + w == n else w - 4
        got = Rg[:, :, x0 + lo:x0 + hi].cpu().numpy()
        assert np.array_equal(got, Ro[:, :, lo:hi]), x0
    s.close()


@pytest.mark.parametrize("n", [128, 768, 1024, 1536, 2048, 4096])
def test_stage_shape_covers_the_grid(torch, n):
    """The stage launch shape the library reports: its segments tile the
    rows exactly (no empty segment), its wavefronts fit the launch rules,
    and 2048^2 takes the pair-balanced 30 x 47 + 29 x 22 rows."""
    d, U = W.riemann2d_config3(n)
    s = _solver(d)
    sh = s.stage_shape()
    s.close()
    assert sh["strips"] == (n + 60) // 61
    n1, r1, r2, ns = sh["nseg1"], sh["rows1"], sh["rows2"], sh["nseg"]
    assert 1 <= n1 <= ns and r1 >= 1 and r2 >= 1
    rows = n1 * r1
    assert rows < n or n1 == ns
    last_start = rows + (ns - n1 - 1) * r2 if ns > n1 else (n1 - 1) * r1
    assert last_start < n <= (rows + (ns - n1) * r2 if ns > n1 else n1 * r1)
    if n == 2048:
        assert (r1, r2, n1, ns) == (47, 22, 30, 59)


def test_adaptive_segment_rows_move_and_keep_the_results(torch):
    """The first-height segment rows of the 2048^2 stage launch follow the
    flow: after 30 steps of the four-quadrant problem rows have moved from
    the segments where the stencil-cut test runs in full to the others, and
    every strip's boundaries are still a partition of its first 30 x 47 rows.
    The state equals, bit for bit, that of 30 steps with one fixed segment
    height.  A tuning turns the layout off; clearing it starts it afresh."""
    import math
    _say("adaptive layout 2048^2, 30 steps")
    d, U0 = W.riemann2d_config3(2048)
    s = _solver(d)
    R = 30 * 47
    L0 = s.stage_layout()
    assert L0 is not None and L0.shape == (34, 31)
    assert np.array_equal(L0, np.tile(np.arange(31) * 47, (34, 1)))
    U = s.new_state(U0)
    s.solve(U, t_final=math.inf, cfl=0.5, max_steps=30)
    L = s.stage_layout()
    rows = np.diff(L, axis=1)
    assert np.all(L[:, 0] == 0) and np.all(L[:, -1] == R)
    assert rows.min() >= 11 and rows.min() < 47 and rows.max() > 47
    s2 = _solver(d)
    s2.set_tuning(47)
    assert s2.stage_layout() is None
    V = s2.new_state(U0)
    s2.solve(V, t_final=math.inf, cfl=0.5, max_steps=30)
    assert torch.equal(U, V)
    s.set_tuning(0)
    assert np.array_equal(s.stage_layout(), L0)
    s.close()
    s2.close()


def test_randomised_cases_against_the_oracle(orc, torch):
    """A seeded sweep over random 1D and 2D Euler problems: every flux,
    scheme, characteristic or componentwise interpolation, boundary kind,
    TENO power q in {2, 4, 6, 8, 12} and states rescaled by 1e-3 .. 1e4 (the
    same flows in other units), at ragged sizes.  The RHS and its cut flags,
    and a few SSP-RK3 steps, against the oracle (both may fail, then at the
    same stage and cell).  q = 8 and 12 reach the range where plain powers
    of C + tau5 / (beta_k + eps) overflow double."""
    from paper_1810_07806_amd.wcnst import WcnstError, split_flags
    rng = np.random.default_rng(2024)
    for n in range(60):
        ndim = int(rng.integers(1, 3))
        kw = dict(flux=str(rng.choice(["roe", "lf", "vanleer"])),
                  scheme=str(rng.choice(["teno", "teno", "linear", "js", "z"])), charwise=int(rng.integers(0, 2)))
        if kw["scheme"] == "teno" and rng.random() < 0.5:
            kw["q"] = int(rng.choice([2, 4, 8, 12]))
        if kw["scheme"] == "z" and rng.random() < 0.5:
            kw["z_q"] = 2
        sides = ["zero_gradient", "periodic", "reflect"]
        if ndim == 1:
            d, U = W.random_tube(rng, int(rng.choice([5, 17, 61, 62, 122, 200, 777])))
            kw["bc_x"] = str(rng.choice(sides))
        else:
            d, U = W.random_euler2d(rng, int(rng.integers(5, 90)), int(rng.integers(5, 90)))
            kw["bc_x"], kw["bc_y"] = str(rng.choice(sides)), str(rng.choice(sides))
        if rng.random() < 0.3:
            U = U * float(10.0 ** rng.uniform(-3, 4))
        d.update(kw)
        _say(f"random case {n}: ndim={ndim} nx={d['nx']} ny={d.get('ny', 1)} {kw}")
        s = _solver(d)
        Ug = s.new_state(U)
        Rg, fg = s.rhs(Ug, flags=True)
        Rg = Rg.cpu().numpy()
        fg = [b.cpu().numpy() for b in split_flags(d, fg)]
        p = orc.problem(d)
        Ro, fo, co = orc.rhs(p, U, flags=True, chi=True, nthreads=NTHREADS)
        flips = check_flags(fg, fo, co, d.get("CT", 1e-5))
        assert_rhs_close(Rg, Ro, rhs_mask_from_flips((Ro.shape[1], Ro.shape[2]), flips, ndim))
        steps = int(rng.integers(1, 12))
        r = orc.solve(p, U, t_final=np.inf, cfl=0.5, max_steps=steps, nthreads=NTHREADS)
        try:
            s.solve(Ug, t_final=np.inf, cfl=0.5, max_steps=steps)
            g = dict(status=0)
        except WcnstError:
            g = s.status()
        assert (r["status"] == 0) == (g["status"] == 0), (r["status"], g)
        if r["status"] == 0:
            assert np.array_equal(Ug.cpu().numpy(), r["U"])
        else:
            assert (r["bad_stage"], r["bad_cell"]) == (g["bad_stage"], g["bad_cell"])
        s.close()
