"""Host logic of solve_recycling (CPU, stand-in problem): which restarts are
redrawn with which seed, how the best assignment is kept, when it stops."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2606_06656_amd import pcls  # noqa: E402


class StandIn:
    """Plays back per-round (iters, unsat) and records every initialisation."""
    device = torch.device("cpu")

    def __init__(self, n, rounds):
        self.n, self.rounds, self.k = n, rounds, 0
        self.calls = []

    def new_state(self, R):
        return torch.zeros((self.n, R), dtype=torch.float32)

    def init_restarts(self, X, R, seed):
        self.calls.append(("all", seed, None))

    def init_restarts_masked(self, X, R, seed, mask):
        self.calls.append(("masked", seed, mask.tolist()))

    def step_ex(self, X, R, lr, n_steps, tol, want_iters):
        return None, torch.tensor(self.rounds[self.k][0], dtype=torch.int32)

    def extract(self, X, R):
        unsat = torch.tensor(self.rounds[self.k][1], dtype=torch.int32)
        assign = torch.full((R, self.n), 10 * self.k, dtype=torch.int8) + torch.arange(R, dtype=torch.int8)[:, None]
        best = torch.tensor([int(torch.argmin(unsat))], dtype=torch.int32)
        self.k += 1
        return assign, unsat, best


def test_converged_restarts_are_redrawn_with_the_next_seed():
    steps = 10
    prob = StandIn(4, [([10, 3, 10], [5, 4, 6]),   # restart 1 converged
                       ([2, 10, 7], [5, 2, 6]),    # restarts 0 and 2 converged; 2 is the new best
                       ([10, 10, 10], [3, 3, 3])])  # nothing converged, no better
    out = pcls.solve_recycling(prob, 3, rounds=3, steps_per_round=steps, seed=40)
    assert prob.calls == [("all", 40, None), ("masked", 41, [0, 1, 0]), ("masked", 42, [1, 0, 1])]
    assert out["unsat"] == 2
    assert np.array_equal(out["assign"], np.full(4, 10 + 1, np.int8))  # round 1, restart 1
    assert [r["converged"] for r in out["rounds"]] == [1, 2, 0]
    assert [r["min_unsat"] for r in out["rounds"]] == [4, 2, 3]
    assert out["rounds"][0]["mean_steps"] == pytest.approx((10 + 3 + 10) / 3)


def test_stops_once_every_constraint_holds():
    prob = StandIn(2, [([1, 1], [3, 1]), ([1, 1], [0, 2]), ([1, 1], [0, 0])])
    out = pcls.solve_recycling(prob, 2, rounds=3, steps_per_round=5, seed=7)
    assert out["unsat"] == 0 and len(out["rounds"]) == 2
    assert prob.calls == [("all", 7, None), ("masked", 8, [1, 1])]  # no redraw after the solution


def test_last_round_redraws_nothing():
    prob = StandIn(2, [([1, 1], [3, 1])])
    out = pcls.solve_recycling(prob, 2, rounds=1, steps_per_round=5, seed=7)
    assert prob.calls == [("all", 7, None)] and out["unsat"] == 1
