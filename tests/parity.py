"""Comparison rules of the GPU-vs-oracle parity tests.

RHS:    per conserved component, ||R_gpu - R_orc||_inf <= 1e-12 ||R_orc||_inf.
Fields: per component, ||U_gpu - U_orc||_inf <= 1e-10 ||U_orc||_inf.
Flags:  identical, except entries where one of the oracle's chi_k lies within
        1e-12 * C_T of C_T (a comparison decided by the last bits); cells whose
        stencil reaches such a flipped midpoint are then left out of the RHS
        comparison.
"""
from __future__ import annotations

import numpy as np

RHS_TOL = 1e-12
FIELD_TOL = 1e-10
BAND = 1e-12


def rel_inf_err(a, b):
    """Per-component ||a - b||_inf / ||b||_inf over the leading axis.  NaN
    entries must sit at the same places on both sides (a non-physical
    intermediate state gives NaN in both); they are then left out."""
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    out = []
    for v in range(a.shape[0]):
        na, nb = np.isnan(a[v]), np.isnan(b[v])
        if not np.array_equal(na, nb):
            out.append(np.inf)
            continue
        ok = ~nb
        if not ok.any():
            out.append(0.0)
            continue
        scale = np.abs(b[v][ok]).max()
        err = np.abs(a[v][ok] - b[v][ok]).max()
        out.append(err / scale if scale > 0 else err)
    return np.array(out)


def flag_mismatch(fg, fo, chi, CT):
    """Returns (mismatch mask, tie mask) over the oracle's flag array shape."""
    fg = np.asarray(fg)
    fo = np.asarray(fo)
    tie = (np.abs(chi - CT) <= BAND * CT).any(axis=-1)
    return fg != fo, tie


def check_flags(fg_blocks, fo_blocks, chi_blocks, CT):
    """Asserts flag identity outside the tie band; returns the flipped-in-band
    positions per direction (lists of (line, slot))."""
    flips = []
    for fg, fo, ch in zip(fg_blocks, fo_blocks, chi_blocks):
        mis, tie = flag_mismatch(fg, fo, ch, CT)
        bad = mis & ~tie
        assert not bad.any(), f"{int(bad.sum())} flags differ outside the tie band, first at {np.argwhere(bad)[:5]}"
        flips.append(np.argwhere(mis))
    return flips


def rhs_mask_from_flips(shape, flips, ndim, diff="mnd"):
    """Boolean mask (ny, nx) of cells whose stencil touches a flipped midpoint
    (MND: midpoints within 3/2 spacings of a cell, slot s = j + 2; MD: within
    5/2 spacings, slot s = j + 3; HWCNS: within 1/2, slot s = j + 1)."""
    ny, nx = shape
    g = {"md": 3, "hwcns": 1}.get(diff, 2)
    keep = np.ones((ny, nx), dtype=bool)
    for d, fl in enumerate(flips):
        for k, line, slot, side in fl:
            j = slot - g  # midpoint j + 1/2
            lo, hi = max(0, j - g + 1), min((nx if d == 0 else ny) - 1, j + g)
            if d == 0:
                keep[line, lo:hi + 1] = False
            else:
                keep[lo:hi + 1, line] = False
    return keep


def assert_rhs_close(Rg, Ro, keep=None, tol=RHS_TOL):
    Rg = np.asarray(Rg, dtype=np.float64)
    Ro = np.asarray(Ro, dtype=np.float64)
    if keep is not None:
        Rg = np.where(keep[None], Rg, Ro)
    err = rel_inf_err(Rg, Ro)
    assert (err <= tol).all(), f"relative RHS error per component {err} exceeds {tol}"
    return err


# ------------------------------------------------- decisions below resolution

FLAT_REL = 1e-12


def _left_eigenvectors(UA, UB, gamma, nv):
    """Rows of the left eigenvector matrix at the Roe average of UA, UB
    (arrays (F, nv), normal momentum first), textbook form, (F, nv, nv).
    Used only to find the characteristic data of each stencil (numpy, no
    attention to rounding)."""
    rA, rB = UA[:, 0], UB[:, 0]
    def prim(U, r):
        u = U[:, 1] / r
        v = U[:, 2] / r if nv == 4 else np.zeros_like(r)
        p = (gamma - 1) * (U[:, nv - 1] - 0.5 * r * (u * u + v * v))
        return u, v, (U[:, nv - 1] + p) / r
    uA, vA, HA = prim(UA, rA)
    uB, vB, HB = prim(UB, rB)
    sA, sB = np.sqrt(rA), np.sqrt(rB)
    u = (sA * uA + sB * uB) / (sA + sB)
    v = (sA * vA + sB * vB) / (sA + sB)
    H = (sA * HA + sB * HB) / (sA + sB)
    q2 = u * u + v * v
    c = np.sqrt((gamma - 1) * (H - 0.5 * q2))
    b1 = (gamma - 1) / c ** 2
    b2 = 0.5 * q2 * b1
    L = np.zeros((UA.shape[0], nv, nv))
    L[:, 0, 0], L[:, 0, 1], L[:, 0, nv - 1] = 0.5 * (b2 + u / c), -0.5 * (b1 * u + 1 / c), 0.5 * b1
    L[:, 1, 0], L[:, 1, 1], L[:, 1, nv - 1] = 1 - b2, b1 * u, -b1
    L[:, nv - 1, 0], L[:, nv - 1, 1], L[:, nv - 1, nv - 1] = 0.5 * (b2 - u / c), -0.5 * (b1 * u - 1 / c), 0.5 * b1
    if nv == 4:
        L[:, 0, 2], L[:, 1, 2], L[:, 3, 2] = -0.5 * b1 * v, b1 * v, -0.5 * b1 * v
        L[:, 2, 0], L[:, 2, 2] = -v, 1.0
    return L


def flat_interpolations(desc, U):
    """Interpolations (flag layout [nv][lines][nfaces][2] per direction, MND
    faces, periodic or zero-gradient sides) in which at least two of the
    three candidate substencils hold values that vary by no more than
    FLAT_REL times the field's magnitude there.  Their smoothness indicators
    are then rounding noise, so the comparison of their measures (Eqs.
    (16)-(18)) is decided by rounding; and whatever the pattern, those
    candidates agree within the tolerance, so the interpolated value does
    not move beyond it.  This happens where a characteristic field is
    constant in exact arithmetic (an acoustic field across a pure density
    wave), also next to a jump in the other fields."""
    nv = U.shape[0]
    ndim = int(desc.get("ndim", 1))
    euler = desc.get("system", "euler") == "euler"
    charwise = euler and int(desc.get("charwise", 1)) == 1
    gamma = float(desc.get("gamma", 1.4))
    out = []
    dirs = [("x", [0, 1, 2, 3][:nv], U)]
    if ndim == 2:
        dirs.append(("y", [0, 2, 1, 3], np.transpose(U, (0, 2, 1))))
    for axis, perm, V in dirs:
        bc = desc.get(f"bc_{axis}", "zero_gradient")
        if bc not in ("periodic", "zero_gradient"):
            raise NotImplementedError(bc)
        lines = V[perm]  # (nv, nlines, n), normal momentum first
        n = lines.shape[2]
        ext = np.pad(lines, ((0, 0), (0, 0), (4, 4)), mode="wrap" if bc == "periodic" else "edge")
        nf = n + 3
        # stencil of face j = s - 2: nodes j-2 .. j+3 = ext columns s .. s+5
        st = np.stack([ext[:, :, m:m + nf] for m in range(6)], axis=-1)  # (nv, lines, nf, 6)
        st = np.moveaxis(st, 0, -1).reshape(-1, 6, nv)  # (F, 6, nv)
        if charwise:
            L = _left_eigenvectors(st[:, 2], st[:, 3], gamma, nv)
        else:
            L = np.broadcast_to(np.eye(nv), (st.shape[0], nv, nv))
        terms = L[:, :, None, :] * st[:, None, :, :]  # (F, k, m, v)
        W = terms.sum(-1)
        scale = np.abs(terms).sum(-1).max(-1)  # (F, k)
        tol = FLAT_REL * scale[..., None]

        def undecided(t):  # t: the four neighbour differences of one side
            small = np.abs(t) <= tol
            sub = small[..., 0:3] & small[..., 1:4]  # substencil k uses t_k, t_{k+1}
            return sub.sum(-1) >= 2

        flatL = undecided(np.diff(W[:, :, 0:5], axis=-1))
        flatR = undecided(np.diff(W[:, :, 1:6][..., ::-1], axis=-1))
        flat = np.stack([flatL, flatR], axis=-1).reshape(lines.shape[1], nf, nv, 2)
        out.append(np.moveaxis(flat, 2, 0))
    return out
