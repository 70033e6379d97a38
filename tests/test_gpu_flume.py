"""GPU parity of the wave-flume configuration: the time-dependent linear-wave
inlet, the porous barrier with Van Genuchten closures and the open top,
alone and as a batch of amplitudes replayed from captured graphs."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2003_08374_amd import workloads as W
from parity_util import compare_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    O.build(force=False)


def _small_flume(amplitude=0.03, **kw):
    args = dict(nx=48, ny=20, h=0.02, dt=2e-3, amplitude=amplitude, period=1.0, depth=0.2,
                x_barrier=0.6, crest_height=0.25, crest_width=0.1, slope=1.0, steps=10)
    args.update(kw)
    return W.wave_flume(**args).replace(p_tol=1e-13)


def test_flume_matches_oracle():
    """Ten steps against the oracle.  Both sides solve the pressure to a
    relative residual of 1e-14: over ten steps of wave motion through the
    limiter, a solver tolerance of 1e-13 alone leaves alpha and U differences
    of about 1e-10, the size of the bar."""
    from paper_2003_08374_amd import dbs
    c = _small_flume().replace(p_tol=1e-14)
    n = 10
    ref, _ = O.step(c.replace(p_tol=1e-14, p_maxit=200000), O.initial_state(c), n)
    with dbs.Solver(c) as s:
        s.step(n)
        out = s.state()
        assert s.stats()["time"] == pytest.approx(n * c.dt, rel=1e-12)
    compare_states(out, ref, label="flume_48x20")


def test_flume_batch_graph_matches_oracle():
    """Three amplitudes in one batch, steps replayed from captured graphs
    (step 1 eager, 2 and 3 captured, 4 and 5 replayed): the inlet's time must
    advance on the device between replays."""
    from paper_2003_08374_amd import dbs
    cases = [_small_flume(amplitude=a, nx=40 + 4 * i) for i, a in enumerate((0.02, 0.03, 0.04))]
    n = 5
    with dbs.BatchSolver(cases) as B:
        B.set_graph(True)
        for _ in range(n):
            B.step(1)
        outs = [B.state(i) for i in range(len(cases))]
    for c, out in zip(cases, outs):
        ref, _ = O.step(c.replace(p_tol=1e-14, p_maxit=200000), O.initial_state(c), n)
        compare_states(out, ref, label=f"flume graph {c.name}")


def test_flume_restart_time():
    """Stepping 4 + 4 from a restart at t = 4 dt equals 8 steps in one go,
    to the solver tolerance: the restarted run's first pressure solve starts
    from p_rgh itself, the continuous run's from the guess extrapolated from
    the two steps before (a wrong boundary time would differ by far more)."""
    from paper_2003_08374_amd import dbs
    c = _small_flume()
    with dbs.Solver(c) as s:
        s.step(8)
        full = s.state()
    with dbs.Solver(c) as s:
        s.step(4)
        mid = s.state()
    with dbs.Solver(c, state=mid) as s:
        s.set_time(4 * c.dt)
        s.step(4)
        out = s.state()
    compare_states(out, full, tol_l2=1e-10, tol_alpha=1e-10, label="flume restart")
