"""Right-hand-side cases of the parity tests, shared by the GPU parity tests
and by the CPU check that the oracle's single-rounding build agrees with its
plain build (every case the GPU is compared on is also a case the two
oracle builds are compared on)."""
from __future__ import annotations

import numpy as np

from paper_1810_07806_amd import workloads as W

CASES_1D = []
for _flux in ("roe", "lf"):
    for _scheme in ("teno", "linear", "js"):
        CASES_1D.append(dict(flux=_flux, scheme=_scheme, charwise=1, bc_x="zero_gradient"))
CASES_1D.append(dict(flux="roe", scheme="teno", charwise=0, bc_x="zero_gradient"))
CASES_1D.append(dict(flux="roe", scheme="teno", charwise=1, bc_x="periodic"))
CASES_1D.append(dict(flux="lf", scheme="teno", charwise=0, bc_x="periodic"))
CASES_1D.append(dict(flux="vanleer", scheme="teno", charwise=1, bc_x="zero_gradient"))
CASES_1D.append(dict(flux="vanleer", scheme="js", charwise=0, bc_x="periodic"))
# Eq. (16) with other integer powers than the paper's q = 6
CASES_1D.append(dict(flux="roe", scheme="teno", charwise=1, bc_x="zero_gradient", q=2))
CASES_1D.append(dict(flux="lf", scheme="teno", charwise=1, bc_x="periodic", q=4))
# the WCNS-Z comparison scheme of Sec. 3 (Borges et al. 2008 weights)
CASES_1D.append(dict(flux="roe", scheme="z", charwise=1, bc_x="zero_gradient"))
CASES_1D.append(dict(flux="lf", scheme="z", charwise=0, bc_x="periodic", z_q=2))

CASES_2D = [dict(flux="roe", scheme="teno", charwise=1),
            dict(flux="lf", scheme="teno", charwise=1),
            dict(flux="roe", scheme="linear", charwise=1),
            dict(flux="roe", scheme="teno", charwise=0),
            dict(flux="roe", scheme="js", charwise=1),
            dict(flux="vanleer", scheme="teno", charwise=1),
            dict(flux="roe", scheme="teno", charwise=1, q=4),
            dict(flux="roe", scheme="z", charwise=1),
            dict(flux="lf", scheme="z", charwise=0, z_q=2)]

# ragged strips and segments, one strip / one segment, the minimum, and exact
# multiples of the 61-column strip and the 35-row segment
SIZES_2D = ((133, 97), (61, 33), (5, 5), (130, 65), (122, 70), (62, 36))
SIZES_1D = (245, 61, 62, 5)


def euler1d_cases(kw):
    """(name, desc, U) of the 1D Euler case list entry kw."""
    rng = np.random.default_rng(100)
    for n in SIZES_1D:
        d, U = W.random_tube(rng, n)
        d.update(kw)
        yield f"tube{n}", d, U
    d, U = W.random_tube(np.random.default_rng(7), 300)
    d.update(kw)
    yield "tube300", d, U


def euler2d_cases(kw):
    """(name, desc, U) of the 2D case list entry kw."""
    rng = np.random.default_rng(200)
    for (nx, ny) in SIZES_2D:
        d, U = W.random_euler2d(rng, nx, ny)
        d.update(kw)
        yield f"quad{nx}x{ny}", d, U
    d, U = W.random_euler2d(rng, 70, 40)
    d.update(kw, bc_x="periodic", bc_y="periodic")
    yield "quad-periodic", d, U


def scalar_cases():
    for n in (200, 199, 5):
        d, U = W.advection_sine_square(n) if n >= 8 else W.smooth_periodic(n)
        yield f"advection{n}", d, U
    for flux in ("roe", "lf"):
        rng = np.random.default_rng(5)
        d = W.describe(ndim=1, system="burgers", nx=150, bc_x="periodic", flux=flux)
        yield f"burgers-{flux}", d, rng.normal(size=(1, 1, 150))


EXTREME_DENSITY = {"crossing-2^-767": lambda s: -230.6 + 1.5 * np.sin(2 * np.pi * s),
                   "1e-300": lambda s: -300.0 + 0.2 * np.sin(2 * np.pi * s),
                   "1e150": lambda s: 150.0 + 0.2 * np.sin(2 * np.pi * s)}


def scaled_state(ndim, n, log_rho, gamma=1.4):
    """Smooth state with density 10**log_rho(x) (and pressure of the same
    scale, so the sound speed stays of order one)."""
    if ndim == 1:
        d = W.describe(ndim=1, system="euler", nx=n, bc_x="periodic")
        x = W.coords(d)
        rho = 10.0 ** log_rho(x)
        return d, W.conserved_1d(rho, 0.4 + 0.2 * np.sin(4 * np.pi * x), rho * (1 + 0.3 * np.cos(2 * np.pi * x)),
                                 gamma)[:, None, :]
    d = W.describe(ndim=2, system="euler", nx=n, ny=45, bc_x="periodic", bc_y="periodic")
    x, y = np.meshgrid(W.coords(d, "x"), W.coords(d, "y"))
    rho = 10.0 ** log_rho(x + y)
    return d, W.conserved_2d(rho, 0.4 + 0.2 * np.sin(4 * np.pi * y), -0.3 + 0.1 * np.cos(2 * np.pi * x),
                             rho * (1 + 0.3 * np.cos(2 * np.pi * x)), gamma)


def extreme_density_cases(flux, scale):
    for ndim, n in ((1, 245), (2, 70)):
        d, U = scaled_state(ndim, n, EXTREME_DENSITY[scale])
        d.update(flux=flux, scheme="teno", charwise=1)
        yield f"density-{scale}-{ndim}D", d, U


def all_rhs_cases(full_size: bool = False):
    """Every RHS case of the parity lists (the 2048^2 cases only with
    full_size)."""
    for kw in CASES_1D:
        for name, d, U in euler1d_cases(kw):
            yield f"{name}-{'-'.join(str(v) for v in kw.values())}", d, U
    for kw in CASES_2D:
        for name, d, U in euler2d_cases(kw):
            yield f"{name}-{'-'.join(str(v) for v in kw.values())}", d, U
    yield from scalar_cases()
    for flux in ("roe", "lf"):
        for scale in EXTREME_DENSITY:
            yield from extreme_density_cases(flux, scale)
    d, U = W.shu_osher(2048)
    yield "shu-osher", d, U
    if full_size:
        d, U = W.riemann2d_config3(2048)
        yield "config3-2048", d, U
