"""The device reciprocal and square root that the Roe average of the
characteristic projection uses (the hardware's correctly rounded sequences
without their range scaling) against the IEEE division and root, bit for
bit, over the argument range they serve (positive x in [2^-767, 2^1022)):
adversarial mantissas next to all-ones and to zero at every exponent of the
range, and random arguments; the IEEE results on the device also equal the
host's."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "devcheck", "libdevcheck.so")


def _args():
    exps = np.arange(-767, 1022)
    k = np.arange(512, dtype=np.uint64)
    mant = np.concatenate([(np.uint64(1) << np.uint64(52)) - np.uint64(1) - k, k])
    ebits = (exps + 1023).astype(np.uint64) << np.uint64(52)
    adv = (ebits[:, None] | mant[None, :]).ravel()
    rng = np.random.default_rng(17)
    rnd = (rng.integers(256, 2045, size=1 << 21).astype(np.uint64) << np.uint64(52)) | \
        rng.integers(0, 1 << 52, size=1 << 21, dtype=np.uint64)
    return np.concatenate([adv, rnd]).view(np.float64)


def test_ranged_reciprocal_and_root_equal_ieee():
    assert os.path.exists(LIB), "tests/devcheck/libdevcheck.so is missing: run __graft_entry__.build() first"
    L = ctypes.CDLL(LIB)
    L.dc_ranged_math.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    x = np.ascontiguousarray(_args())
    assert ((x >= 2.0 ** -767) & (x < 2.0 ** 1022)).all()
    print(f"[case] ranged math on {x.size} arguments", flush=True)
    out = np.empty((4, x.size), dtype=np.float64)
    assert L.dc_ranged_math(x.ctypes.data, x.size, out.ctypes.data) == 0
    rcp_r, rcp_i, sq_r, sq_i = out
    assert np.array_equal(rcp_i.view(np.uint64), (1.0 / x).view(np.uint64))
    assert np.array_equal(sq_i.view(np.uint64), np.sqrt(x).view(np.uint64))
    assert np.array_equal(rcp_r.view(np.uint64), rcp_i.view(np.uint64))
    assert np.array_equal(sq_r.view(np.uint64), sq_i.view(np.uint64))
