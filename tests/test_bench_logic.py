"""Host logic of bench.py (CPU only): the timed run is made of segments of at
most `segment` steps from the rest state, and the statistics of every
rbf_step call are summed."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
torch = pytest.importorskip("torch")
import bench  # noqa: E402


class _FakeSolver:
    """Stands in for a solver: advances 'step' and a counter field."""

    def __init__(self, segment):
        self.calls, self.segment = [], segment

    def step(self, st, k):
        assert k >= 1 and st["step"] + k <= self.segment
        self.calls.append((st["step"], k))
        st["step"] += k
        st["u"] += k

        class _S:
            poisson_iters, helmholtz_iters, last_poisson = 3 * k, k, None
        return _S()


def test_run_restores_rest_state_every_segment():
    st = {"u": torch.zeros(4, dtype=torch.float64), "step": 0}
    S = _FakeSolver(400)
    run = bench.Run(S, st, 400)
    run.advance(10)
    run.clear()
    run.advance(1000)
    assert S.calls == [(0, 10), (10, 390), (0, 400), (0, 210)]
    assert run.restarts == 2 and run.poisson_iters == 3000 and run.helmholtz_iters == 1000
    assert st["step"] == 210 and torch.equal(st["u"], torch.full((4,), 210.0, dtype=torch.float64))
    assert run.rest["step"] == 0 and torch.equal(run.rest["u"], torch.zeros(4, dtype=torch.float64))


def test_run_within_one_segment_is_one_call():
    st = {"u": torch.zeros(2, dtype=torch.float64), "step": 0}
    S = _FakeSolver(400)
    run = bench.Run(S, st, 400)
    run.advance(10)
    run.clear()
    run.advance(200)
    assert S.calls == [(0, 10), (10, 200)] and run.restarts == 0
