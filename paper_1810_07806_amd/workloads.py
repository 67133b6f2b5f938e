"""Seeded synthetic inputs: problem descriptors and initial states.

This module holds none of the scheme's arithmetic.  It turns the initial
conditions of the paper's test problems (Sec. 3) and of the synthetic
benchmark workloads into conserved-variable arrays ``U[v][y][x]`` (FP64, x
fastest) plus a descriptor dict that both the HIP binding and the CPU oracle
understand.  Descriptor keys:

    ndim, system ('advection' | 'burgers' | 'euler'), nx, ny,
    x0, x1, y0, y1, bc_x, bc_y ('periodic' | 'zero_gradient'),
    flux ('roe' | 'lf'), scheme ('teno' | 'linear' | 'js'), diff ('mnd' | 'md'),
    charwise, gamma, adv_speed, CT, C, eps_teno, eps_js, q, grid ('cell' | 'node')

Spacing is always h = (x1 - x0) / nx.  On a 'cell' grid the unknowns sit at
x0 + (i + 1/2) h; on a periodic 'node' grid (the paper's convention of N
points including both ends) the unknowns are the N - 1 distinct nodes
x0 + i h.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULTS = dict(ndim=1, system="euler", nx=64, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                bc_x="zero_gradient", bc_y="zero_gradient", flux="roe", scheme="teno",
                diff="mnd", charwise=1, gamma=1.4, adv_speed=1.0, CT=1e-5, C=1.0,
                eps_teno=1e-40, eps_js=1e-6, q=6, z_q=1, eps_z=1e-40, grid="cell")


def describe(**kw) -> dict:
    d = dict(DEFAULTS)
    d.update(kw)
    if d["ndim"] == 1:
        d["ny"] = 1
    return d


def coords(desc: dict, axis: str = "x") -> np.ndarray:
    n = desc["nx"] if axis == "x" else desc["ny"]
    a, b = (desc["x0"], desc["x1"]) if axis == "x" else (desc["y0"], desc["y1"])
    h = (b - a) / n
    off = 0.5 if desc.get("grid", "cell") == "cell" else 0.0
    return a + (np.arange(n, dtype=np.float64) + off) * h


def conserved_1d(rho, u, p, gamma):
    rho, u, p = (np.asarray(a, dtype=np.float64) for a in (rho, u, p))
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def conserved_2d(rho, u, v, p, gamma):
    rho, u, v, p = (np.asarray(a, dtype=np.float64) for a in (rho, u, v, p))
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def primitive(U: np.ndarray, gamma: float):
    """(rho, u[, v], p) from conserved variables (for checks and plots)."""
    rho = U[0]
    if U.shape[0] == 3:
        u = U[1] / rho
        return rho, u, (gamma - 1.0) * (U[2] - 0.5 * rho * u * u)
    u, v = U[1] / rho, U[2] / rho
    return rho, u, v, (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))


# ---------------------------------------------------------------- scalar cases

def advection_sine_square(nx: int = 200):
    """Linear advection, a = 1, periodic [-1, 1]: sin(pi x) plus a unit square
    pulse on [-0.4, 0.4], sampled at cell centres (no centre lies on the pulse
    edges for even nx not divisible by 5 ... and for nx = 200 the centres sit
    at odd multiples of 1/200)."""
    d = describe(ndim=1, system="advection", nx=nx, x0=-1.0, x1=1.0, bc_x="periodic")
    x = coords(d)
    u = np.sin(np.pi * x) + (np.abs(x) <= 0.4).astype(np.float64)
    return d, u[None, None, :].reshape(1, 1, nx)


def advection_gaussian(n_points: int, scheme: str = "teno", diff: str = "md"):
    """Sec. 3.2: exp(-300 (x - 0.5)^2) on periodic [0, 1], N points including
    both ends (N - 1 unknowns)."""
    nx = n_points - 1
    d = describe(ndim=1, system="advection", nx=nx, x0=0.0, x1=1.0, bc_x="periodic",
                 grid="node", scheme=scheme, diff=diff)
    x = coords(d)
    return d, np.exp(-300.0 * (x - 0.5) ** 2).reshape(1, 1, nx)


def burgers_sine(n_points: int, scheme: str = "teno", diff: str = "md", flux: str = "roe"):
    """Sec. 3.3: u0 = 1/2 + sin(pi x) on periodic [0, 2], N points incl. ends."""
    nx = n_points - 1
    d = describe(ndim=1, system="burgers", nx=nx, x0=0.0, x1=2.0, bc_x="periodic",
                 grid="node", scheme=scheme, diff=diff, flux=flux)
    x = coords(d)
    return d, (0.5 + np.sin(np.pi * x)).reshape(1, 1, nx)


def smooth_periodic(nx: int, system: str = "advection", x0: float = -1.0, x1: float = 1.0):
    d = describe(ndim=1, system=system, nx=nx, x0=x0, x1=x1, bc_x="periodic")
    x = coords(d)
    return d, np.sin(np.pi * x).reshape(1, 1, nx)


# ------------------------------------------------------------------ 1D Euler

def riemann_1d(nx: int, left, right, x_split: float = 0.5, x0: float = 0.0, x1: float = 1.0,
               gamma: float = 1.4, **kw):
    d = describe(ndim=1, system="euler", nx=nx, x0=x0, x1=x1, gamma=gamma, **kw)
    x = coords(d)
    lft = x < x_split
    rho = np.where(lft, left[0], right[0])
    u = np.where(lft, left[1], right[1])
    p = np.where(lft, left[2], right[2])
    return d, conserved_1d(rho, u, p, gamma).reshape(3, 1, nx)


def sod(nx: int = 101, **kw):
    """Sec. 3.4 Sod tube: (1, 0, 1) | (0.125, 0, 0.1) split at 0.5."""
    return riemann_1d(nx, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), **kw)


def lax(nx: int = 101, **kw):
    """Sec. 3.4 Lax tube: (0.445, 0.698, 3.528) | (0.5, 0, 0.571)."""
    return riemann_1d(nx, (0.445, 0.698, 3.528), (0.5, 0.0, 0.571), **kw)


def shu_osher(nx: int = 2048, **kw):
    """Shock / density-wave interaction (Sec. 3.5) on [-5, 5], shock at x = -4:
    x < -4: (3.857143, 2.629369, 10.33333); else (1 + 0.2 sin 5x, 0, 1)."""
    d = describe(ndim=1, system="euler", nx=nx, x0=-5.0, x1=5.0, **kw)
    x = coords(d)
    lft = x < -4.0
    rho = np.where(lft, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(lft, 2.629369, 0.0)
    p = np.where(lft, 10.33333, 1.0)
    return d, conserved_1d(rho, u, p, d["gamma"]).reshape(3, 1, nx)


def random_tube(rng: np.random.Generator, nx: int, gamma: float = 1.4):
    """Piecewise-smooth 1D Euler state with a jump and a smooth wave, for
    parity tests that must exercise both cut and uncut stencils."""
    d = describe(ndim=1, system="euler", nx=nx, gamma=gamma)
    x = coords(d)
    xs = rng.uniform(0.3, 0.7)
    lft = x < xs
    rho = np.where(lft, rng.uniform(0.5, 2.0), rng.uniform(0.1, 1.0)) * (1 + 0.1 * np.sin(7 * x))
    u = np.where(lft, rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5))
    p = np.where(lft, rng.uniform(0.5, 2.0), rng.uniform(0.1, 1.0))
    return d, conserved_1d(rho, u, p, gamma).reshape(3, 1, nx)


# ------------------------------------------------------------------ 2D Euler

CONFIG3_STATES = {  # (rho, u, v, p), Sec. 3.6.1
    "NE": (1.5, 0.0, 0.0, 1.5),
    "NW": (0.5323, 1.206, 0.0, 0.3),
    "SW": (0.138, 1.206, 1.206, 0.029),
    "SE": (0.5323, 0.0, 1.206, 0.3),
}

CONFIG6_STATES = {  # Sec. 3.6.2
    "NE": (1.0, 0.75, -0.5, 1.0),
    "NW": (2.0, 0.75, 0.5, 1.0),
    "SW": (1.0, -0.75, 0.5, 1.0),
    "SE": (3.0, -0.75, -0.5, 1.0),
}


def quadrants(nx: int, ny: int, states: dict, xs: float = 0.5, ys: float = 0.5,
              gamma: float = 1.4, **kw):
    """Four-quadrant Riemann problem on [0, 1]^2 with zero-gradient sides.
    Quadrant membership follows Sec. 3.6: x >= xs is east, y >= ys is north."""
    d = describe(ndim=2, system="euler", nx=nx, ny=ny, gamma=gamma, **kw)
    x = coords(d, "x")[None, :]
    y = coords(d, "y")[:, None]
    east = np.broadcast_to(x >= xs, (ny, nx))
    north = np.broadcast_to(y >= ys, (ny, nx))
    prim = np.zeros((4, ny, nx))
    for key, st in states.items():
        m = (north if key[0] == "N" else ~north) & (east if key[1] == "E" else ~east)
        for v in range(4):
            prim[v][m] = st[v]
    return d, conserved_2d(prim[0], prim[1], prim[2], prim[3], gamma)


def riemann2d_config3(n: int = 2048, **kw):
    return quadrants(n, n, CONFIG3_STATES, **kw)


def riemann2d_config6(n: int = 1024, **kw):
    return quadrants(n, n, CONFIG6_STATES, **kw)


def rayleigh_taylor(nx: int = 128, ny: int = 512, gamma: float = 5.0 / 3.0, **kw):
    """Sec. 3.8 Rayleigh-Taylor instability on [0, 1/4] x [0, 1], gamma = 5/3:
    heavy gas (rho 2, p = 1 + 2y) below y = 1/2, light gas (rho 1,
    p = y + 3/2, the reading of the garbled "1 + 3/2") above, both at rest
    but for v = -0.025 a cos(8 pi x) with a the local sound speed;
    reflecting walls at x = 0 and 1/4, fixed states (2, 0, 0, 1) at y = 0 and
    (1, 0, 0, 2.5) at y = 1; body force rho (in +y) in the momentum and
    rho v in the energy equation."""
    g = gamma
    fixed_y = (tuple(conserved_2d(2.0, 0.0, 0.0, 1.0, g)), tuple(conserved_2d(1.0, 0.0, 0.0, 2.5, g)))
    d = describe(ndim=2, system="euler", nx=nx, ny=ny, x0=0.0, x1=0.25, y0=0.0, y1=1.0, gamma=g,
                 bc_x="reflect", bc_y="fixed", fixed_y=fixed_y, gravity=1.0, **kw)
    x = coords(d, "x")[None, :]
    y = coords(d, "y")[:, None]
    low = np.broadcast_to(y < 0.5, (ny, nx))
    rho = np.where(low, 2.0, 1.0)
    p = np.where(low, 1.0 + 2.0 * y, y + 1.5)
    a = np.sqrt(g * p / rho)
    v = -0.025 * a * np.cos(8.0 * np.pi * x)
    return d, conserved_2d(rho, np.zeros_like(rho), v, p, g)


def ripples_2d(nx: int, ny: int, gamma: float = 1.4, **kw):
    """Analytic 2D Euler state on [0, 1]^2 for parity at any size: ripples in
    every variable, an oblique density and pressure jump and a shear layer,
    so that neighbouring cells differ everywhere and both cut and kept
    stencils occur.  Built a block of rows at a time (large grids)."""
    d = describe(ndim=2, system="euler", nx=nx, ny=ny, gamma=gamma, **kw)
    x = coords(d, "x")[None, :]
    y = coords(d, "y")
    U = np.empty((4, ny, nx))
    tp = 2.0 * np.pi
    for r0 in range(0, ny, 512):
        yy = y[r0:r0 + 512, None]
        jump = (x + 0.4 * yy) > 0.55
        rho = 1.0 + 0.2 * np.sin(tp * (3.0 * x + 2.0 * yy)) + np.where(jump, 0.8, 0.0)
        u = 0.3 * np.cos(tp * (x - yy)) + np.where(yy > 0.7, 0.4, -0.1)
        v = 0.2 * np.sin(tp * (2.0 * x + 5.0 * yy))
        p = 1.0 + 0.1 * np.cos(tp * (5.0 * x + yy)) + np.where(jump, 1.5, 0.0)
        U[:, r0:r0 + 512, :] = conserved_2d(rho, u, v, p, gamma)
    return d, U


def ripples_1d(nx: int, gamma: float = 1.4, **kw):
    """1D counterpart of ripples_2d on [0, 1]: ripples, a density and
    pressure jump and a velocity step, built in chunks (long lines)."""
    d = describe(ndim=1, system="euler", nx=nx, gamma=gamma, **kw)
    x = coords(d)
    U = np.empty((3, 1, nx))
    tp = 2.0 * np.pi
    for c0 in range(0, nx, 1 << 24):
        xx = x[c0:c0 + (1 << 24)]
        jump = xx > 0.55
        rho = 1.0 + 0.2 * np.sin(tp * 7.0 * xx) + np.where(jump, 0.8, 0.0)
        u = 0.3 * np.cos(tp * 3.0 * xx) + np.where(xx > 0.7, 0.4, -0.1)
        p = 1.0 + 0.1 * np.cos(tp * 5.0 * xx) + np.where(jump, 1.5, 0.0)
        U[:, 0, c0:c0 + (1 << 24)] = conserved_1d(rho, u, p, gamma)
    return d, U


def random_euler2d(rng: np.random.Generator, nx: int, ny: int, gamma: float = 1.4, **kw):
    """Random four-quadrant state with smooth ripples: every parity case sees
    shocks, contacts and smooth regions, so both cut and kept stencils occur."""
    d = describe(ndim=2, system="euler", nx=nx, ny=ny, gamma=gamma, **kw)
    x = coords(d, "x")[None, :]
    y = coords(d, "y")[:, None]
    xs, ys = rng.uniform(0.3, 0.7, size=2)
    rho = np.empty((ny, nx)); u = np.empty((ny, nx)); v = np.empty((ny, nx)); p = np.empty((ny, nx))
    for north in (False, True):
        for east in (False, True):
            m = ((y >= ys) == north) & ((x >= xs) == east)
            m = np.broadcast_to(m, (ny, nx))
            rho[m] = rng.uniform(0.2, 2.0)
            u[m] = rng.uniform(-1.0, 1.0)
            v[m] = rng.uniform(-1.0, 1.0)
            p[m] = rng.uniform(0.2, 2.0)
    ripple = 1.0 + 0.05 * np.sin(2 * np.pi * 3 * x) * np.cos(2 * np.pi * 2 * y)
    return d, conserved_2d(rho * ripple, u, v, p, gamma)


# -------------------------------------------------- batched shock tubes

def _vacuum_free(rl, ul, pl, rr, ur, pr, gamma):
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    # pressure-positivity condition of the exact Riemann solution, with a
    # factor 1/2 safety margin
    return (ur - ul) < 0.5 * 2.0 * (cl + cr) / (gamma - 1.0)


def shock_tube_params(rng: np.random.Generator, n_min: int = 256, n_max: int = 8192,
                      gamma: float = 1.4):
    """One random tube: N log-uniform in [n_min, n_max], rho and p
    log-uniform in [0.1, 10], u uniform in [-1, 1], interface uniform in
    [0.3, 0.7] on [0, 1]; redrawn from the same stream while near-vacuum."""
    n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
    while True:
        rl, rr, pl, pr = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=4))
        ul, ur = rng.uniform(-1.0, 1.0, size=2)
        if _vacuum_free(rl, ul, pl, rr, ur, pr, gamma):
            break
    xs = rng.uniform(0.3, 0.7)
    return dict(nx=n, left=(float(rl), float(ul), float(pl)),
                right=(float(rr), float(ur), float(pr)), x_split=float(xs))


def shock_tube_batch(count: int = 4096, seed: int = 0, n_min: int = 256, n_max: int = 8192,
                     t_final: float = 0.15, gamma: float = 1.4):
    """Independent 1D Euler tubes of uneven length (zero-gradient ends)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        prm = shock_tube_params(rng, n_min, n_max, gamma)
        d, U = riemann_1d(prm["nx"], prm["left"], prm["right"], prm["x_split"], gamma=gamma)
        d["t_final"] = t_final
        out.append((d, U))
    return out


def random_quadrants_params(rng: np.random.Generator, side_min: int = 256, side_max: int = 1024,
                            gamma: float = 1.4):
    """Random four-quadrant state: side log-uniform, rounded to 64; rho, p in
    [0.1, 2], u, v in [-1.5, 1.5]; redrawn while any interface is near-vacuum."""
    side = int(round(math.exp(rng.uniform(math.log(side_min), math.log(side_max))) / 64.0)) * 64
    side = max(side_min, min(side_max, side))
    while True:
        st = {}
        for key in ("NE", "NW", "SW", "SE"):
            rho, p = rng.uniform(0.1, 2.0, size=2)
            u, v = rng.uniform(-1.5, 1.5, size=2)
            st[key] = (float(rho), float(u), float(v), float(p))
        ok = True
        # x-interfaces (west | east) use u, y-interfaces (south | north) use v
        for a, b in (("NW", "NE"), ("SW", "SE")):
            ok &= _vacuum_free(st[a][0], st[a][1], st[a][3], st[b][0], st[b][1], st[b][3], gamma)
        for a, b in (("SW", "NW"), ("SE", "NE")):
            ok &= _vacuum_free(st[a][0], st[a][2], st[a][3], st[b][0], st[b][2], st[b][3], gamma)
        if ok:
            return dict(n=side, states=st)


# -------------------------------------------------- serving request stream

def serving_trace(count: int = 200, seed: int = 0, rate: float = 10.0, frac_1d: float = 0.7,
                  n1_min: int = 512, n1_max: int = 16384, side_min: int = 256, side_max: int = 1024,
                  t_1d: float = 0.15, t_2d: float = 0.1, gamma: float = 1.4):
    """Poisson stream of mixed solve requests: exponential inter-arrival
    times of mean 1/rate seconds; with probability frac_1d a 1D shock tube
    (as the batched tubes, N log-uniform in [n1_min, n1_max], to t_1d), else
    a 2D four-quadrant Riemann problem with random states (side log-uniform
    in [side_min, side_max] rounded to 64, to t_2d).  Returns a list of
    dict(rid, arrival, desc, U0, t_final), arrivals increasing."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < frac_1d:
            prm = shock_tube_params(rng, n1_min, n1_max, gamma)
            d, U = riemann_1d(prm["nx"], prm["left"], prm["right"], prm["x_split"], gamma=gamma)
            tf = t_1d
        else:
            prm = random_quadrants_params(rng, side_min, side_max, gamma)
            d, U = quadrants(prm["n"], prm["n"], prm["states"], gamma=gamma)
            tf = t_2d
        d["t_final"] = tf
        out.append(dict(rid=rid, arrival=t, desc=d, U0=U, t_final=tf))
    return out
