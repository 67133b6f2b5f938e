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
