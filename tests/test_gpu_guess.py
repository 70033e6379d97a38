"""The per-sample choice of the pressure solves' initial guesses (reported by
dbs_stats): a guess changes only the iteration counts, never the solution,
so these tests pin the choice itself on workloads where it is clear-cut.

The first corrector's guess extrapolates p_rgh in time with the order (0 to
3) whose prediction of the last step's p_rgh from the steps before erred
least; a later corrector adds the change of its solve
predicted with the kind (none, its last change, its last two or three
changes extrapolated linearly or quadratically) that best predicted its last
change."""
from __future__ import annotations

import pytest

import oracle as O
from paper_2003_08374_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    O.build(force=False)


def _fractured(n=32):
    return W.fractured_3d(n=n, seed_k=3, seed_phi=4, fractures="planes", frac_seed=5, n_frac=3,
                          name=f"fractured_3d_{n}_planes").replace(p_tol=1e-8, p_maxit=500,
                                                                    mom_tol=1e-8)


def _flume():
    return W.wave_flume(nx=48, ny=20, h=0.02, dt=2e-3, amplitude=0.03, period=1.0, depth=0.2,
                        x_barrier=0.6, crest_height=0.25, crest_width=0.1, slope=1.0,
                        steps=10).replace(p_tol=1e-8)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_smooth_flow_takes_cubic_and_quadratic_change(precision):
    """Flow through the fractured block, smooth in time once the start-up
    transient has passed: cubic extrapolation of p_rgh and quadratic
    extrapolation of the second corrector's change win by step 10 (order 0
    during the first steps, when p_rgh jumps away from its initial field)."""
    from paper_2003_08374_amd import dbs
    with dbs.Solver(_fractured(), precision=precision) as s:
        s.step(1)
        st = s.stats()
        # one stored step: linear at most, the last change by default
        assert (st["p_guess_order"], st["p_guess_change"]) == (1, [0, 1])
        s.step(9)
        st = s.stats()
        assert (st["p_guess_order"], st["p_guess_change"]) == (3, [0, 3])


def test_alternating_flume_takes_p_rgh_itself():
    """In the wave flume p_rgh alternates from step to step, so extrapolating
    it only adds the alternation: order 0 wins."""
    from paper_2003_08374_amd import dbs
    with dbs.Solver(_flume(), precision="mixed") as s:
        for k in range(10):
            s.step(1)
            if k >= 4:
                assert s.stats()["p_guess_order"] == 0, k


def test_reset_restarts_history():
    """A state reset starts the history again: the next step's solves start
    from p_rgh itself, and linear extrapolation is the most the step after
    can take."""
    from paper_2003_08374_amd import dbs
    with dbs.Solver(_fractured(), precision="mixed") as s:
        s.step(10)
        assert s.stats()["p_guess_order"] == 3
        s.set_state(s.state())
        s.step(1)
        assert s.stats()["p_guess_order"] == 1


def test_batch_samples_choose_alone():
    """In a batch every sample takes the choices its own run takes, step by
    step (the choices differ between the two samples at some steps)."""
    from paper_2003_08374_amd import dbs
    cases = [_fractured(32), _fractured(48)]
    n = 10
    alone = []
    for c in cases:
        seq = []
        with dbs.Solver(c, precision="mixed") as s:
            for _ in range(n):
                s.step(1)
                st = s.stats()
                seq.append((st["p_guess_order"], tuple(st["p_guess_change"])))
        alone.append(seq)
    batch = [[] for _ in cases]
    with dbs.BatchSolver(cases, precision="mixed") as B:
        for _ in range(n):
            B.step(1)
            for i in range(len(cases)):
                st = B.stats(i)
                batch[i].append((st["p_guess_order"], tuple(st["p_guess_change"])))
    assert batch == alone
    assert any(a != b for a, b in zip(*alone))
