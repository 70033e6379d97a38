"""The pressure solve that allocates nothing (dbs_pressure_solve_noalloc):
its work arrays live in the library's static device scratch array.  It is
checked against the handle's dbs_debug_pressure_solve on the same operator
and right-hand side, at the FP64 bar, on two calls in a row with the
second on a smaller mesh (the scratch keeps the first call's contents)."""
from __future__ import annotations

import numpy as np
import pytest

import pin_cases as PC
from paper_2003_08374_amd import workloads as W
from parity_util import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    t.cuda.set_device(0)
    return t


def _system(shape, seed, closed=False):
    c = PC.random_3d(shape, seed=seed)
    if closed:
        c = c.replace(bc=[W.wall()] * 6)
    rng = np.random.default_rng(seed + 100)
    n = int(np.prod(shape))
    rAU = 10 ** rng.uniform(-9, -5, n)
    b = rng.standard_normal(n) * 1e-6
    if closed:
        b -= b.mean()
    x0 = rng.standard_normal(n) * 1e-3
    return c, rAU, b, x0


def _with_handle(c, rAU, b, x0, tol, precision):
    from paper_2003_08374_amd import dbs
    with dbs.Solver(c.replace(p_tol=tol), precision=precision) as s:
        return s.pressure_solve(rAU, b, x0)


def _noalloc(torch, c, rAU, b, x0, tol, precision):
    from paper_2003_08374_amd import dbs
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    tr, tb, tx = dev(rAU), dev(b), dev(x0)
    torch.cuda.synchronize()
    it, rr = dbs.pressure_solve_noalloc(c, tr.data_ptr(), tb.data_ptr(), tx.data_ptr(), tol,
                                        precision=precision)
    return tx.cpu().numpy(), it, rr


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_solve_equals_the_handle_solve_twice(torch, precision):
    """First a 45 x 38 x 21 mesh with an outlet, then a smaller closed
    19 x 14 x 11 box: each equals dbs_debug_pressure_solve to 1e-10."""
    tol = 1e-13
    for shape, seed, closed in [((45, 38, 21), 3, False), ((19, 14, 11), 4, True)]:
        c, rAU, b, x0 = _system(shape, seed, closed)
        xh, ith, rh = _with_handle(c, rAU, b, x0, tol, precision)
        xn, itn, rn = _noalloc(torch, c, rAU, b, x0, tol, precision)
        e = rel_l2(xn, xh)
        print(shape, precision, "its", ith, itn, "relres", rh, rn, "diff", e, flush=True)
        assert rn <= tol and e <= 1e-10
        assert abs(itn - ith) <= 1


def test_noalloc_solve_rejects_meshes_beyond_its_scratch(torch):
    """A mesh above the stated maximum is refused before any GPU work."""
    from paper_2003_08374_amd import dbs
    c = PC.random_3d((100, 80, 70), seed=1)  # 560,000 cells > 2^19
    t = torch.zeros(8, dtype=torch.float64, device="cuda")  # never read: refused first
    with pytest.raises(dbs.DBSError) as e:
        dbs.pressure_solve_noalloc(c, t.data_ptr(), t.data_ptr(), t.data_ptr(), 1e-10)
    assert e.value.code == dbs.EINVAL and "maximum" in str(e.value)
