"""wcnst_solve_noalloc (static scratch, no workspace) against wcnst_solve
through the C ABI: the same kernels, so the same bits, on two calls in a
row, the second on a smaller grid (the static scratch keeps the first
call's contents), and at the largest grid the scratch admits."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_1810_07806_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    from paper_1810_07806_amd import wcnst
    wcnst.lib()
    return T


def _both(torch, d, U, **kw):
    from paper_1810_07806_amd.wcnst import Solver, solve_noalloc
    s = Solver(d)
    A = s.new_state(U)
    ta, na = s.solve(A, **kw)
    s.close()
    B = torch.as_tensor(np.ascontiguousarray(U), dtype=torch.float64).reshape(A.shape).cuda().contiguous()
    tb, nb = solve_noalloc(d, B, **kw)
    torch.cuda.synchronize()
    return (A.cpu().numpy(), ta, na), (B.cpu().numpy(), tb, nb)


def test_noalloc_equals_solve_on_two_calls_in_a_row(torch):
    d2, U2 = W.riemann2d_config3(192)
    _say("noalloc call 1: four-quadrant 192^2, 40 steps")
    (a, ta, na), (b, tb, nb) = _both(torch, d2, U2, t_final=np.inf, cfl=0.5, max_steps=40)
    assert na == nb == 40 and ta == tb
    assert np.array_equal(a, b)
    d1, U1 = W.random_tube(np.random.default_rng(77), 300)
    _say("noalloc call 2: tube of 300 cells to t = 0.1 (smaller)")
    (a, ta, na), (b, tb, nb) = _both(torch, d1, U1, t_final=0.1, cfl=0.5)
    assert na == nb and ta == tb and abs(tb - 0.1) <= 1e-12 * 0.1
    assert np.array_equal(a, b)


def test_noalloc_at_the_largest_admitted_grid(torch):
    from paper_1810_07806_amd.wcnst import WcnstError, solve_noalloc
    d, U = W.riemann2d_config3(1024)
    d = dict(d, ny=1023, y1=1023 / 1024)
    U = np.ascontiguousarray(U[:, :1023, :])
    _say("noalloc at 1024 x 1023, 3 steps")
    (a, ta, na), (b, tb, nb) = _both(torch, d, U, t_final=np.inf, cfl=0.5, max_steps=3)
    assert na == nb == 3 and ta == tb and np.array_equal(a, b)
    big, Ub = W.riemann2d_config3(1024)
    B = torch.zeros(Ub.size, dtype=torch.float64, device="cuda")
    with pytest.raises(WcnstError) as e:
        solve_noalloc(big, B, t_final=np.inf, cfl=0.5, max_steps=1)
    assert e.value.status == 1
