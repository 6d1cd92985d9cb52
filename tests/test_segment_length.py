"""Checkpoint spacing within a workspace budget (solver.segment_length_for):
host arithmetic over the library's workspace formula, no device."""
import pytest

from paper_2406_19494_amd import workloads as W
from paper_2406_19494_amd.solver import segment_length_for, workspace_bytes_for


@pytest.mark.parametrize("mode", [2, 3])
def test_longest_segment_that_fits(mode):
    case, _ = W.tgv(16)
    n = 300
    full = workspace_bytes_for(case, mode, n, n)
    assert segment_length_for(case, mode, n, full) == n      # the whole trajectory resident
    prev = 0
    smallest = min(workspace_bytes_for(case, mode, n, S) for S in range(1, n + 1))
    for frac in (0.2, 0.35, 0.5, 0.75, 0.99):
        budget = int(smallest + frac * (full - smallest))
        S = segment_length_for(case, mode, n, budget)
        assert workspace_bytes_for(case, mode, n, S) <= budget
        # no longer segment fits
        assert all(workspace_bytes_for(case, mode, n, T) > budget for T in range(S + 1, n + 1))
        assert S >= prev
        prev = S


def test_budget_below_the_smallest_workspace_is_refused():
    case, _ = W.tgv(16)
    smallest = min(workspace_bytes_for(case, 2, 100, S) for S in range(1, 101))
    with pytest.raises(ValueError):
        segment_length_for(case, 2, 100, smallest - 1)
    assert workspace_bytes_for(case, 2, 100, segment_length_for(case, 2, 100, smallest)) == smallest
