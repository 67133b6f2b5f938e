"""The oracle's single rounding of each product-plus-sum is a choice of
evaluation order, not a change of method.

The oracle evaluates the differences, candidates and indicators of
Eqs. (9)-(11) and (15), the sum of Eq. (12), the characteristic projections
and the Roe dissipation with one rounding per a * b + c.  The same source
built with -DORC_PLAIN rounds each of them twice, as the formulas read
when evaluated term by term.  On every right-hand-side case the GPU is
compared on, the two builds must agree within the parity tolerance
(1e-12 per component, inf-norm relative) with identical stencil-cut flags
outside the 1e-12 C_T tie band, so the bitwise agreement of the kernels
with the default build carries over to the plain reading of the paper at
the stated tolerances.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

from cases import all_rhs_cases
from parity import assert_rhs_close, flag_mismatch, flat_interpolations

NTHREADS = max(1, min(8, len(os.sched_getaffinity(0))))

CASES = list(all_rhs_cases(full_size=True))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_and_plain_oracle_builds_agree(orc, case):
    name, d, U = case
    p = orc.problem(d)
    Rf, ff, cf = orc.rhs(p, U, flags=True, chi=True, nthreads=NTHREADS)
    Rp, fp, _ = orc.rhs(p, U, flags=True, nthreads=NTHREADS, plain=True)
    CT = d.get("CT", 1e-5)
    # the right-hand sides agree everywhere, flipped cuts or not (a linear
    # interpolation across a jump may leave a state without a real sound
    # speed: both builds give NaN there, at the same places)
    assert_rhs_close(Rp, Rf)
    # cut flags agree outside the tie band and outside stencils whose data
    # are flat to the parity tolerance (there the pattern is decided by
    # rounding and cannot move a value beyond the tolerance)
    flat = flat_interpolations(d, U)
    compared = 0
    for fpb, ffb, cfb, flb in zip(fp, ff, cf, flat):
        mis, tie = flag_mismatch(fpb, ffb, cfb, CT)
        bad = mis & ~tie & ~flb
        assert not bad.any(), f"{name}: {int(bad.sum())} flags differ, first at {np.argwhere(bad)[:4]}"
        compared += int((~flb).sum())
    assert compared > 0


def test_the_two_builds_differ(orc):
    """The comparison above is not vacuous: the builds round differently
    (their right-hand sides are not all bit-identical)."""
    differ = 0
    for name, d, U in CASES[:40]:
        p = orc.problem(d)
        Rf, _, _ = orc.rhs(p, U)
        Rp, _, _ = orc.rhs(p, U, plain=True)
        differ += int(not np.array_equal(Rf, Rp))
    assert differ >= 20
