"""Host logic of the tuner: how many steps a timing run may take."""
import pytest
import torch

from paper_2204_03775_amd import autotune


class _Shot:
    def __init__(self, rows, nrec):
        self.traces = torch.zeros(rows, max(nrec, 1)) if rows else None
        self.nrec = nrec


def test_steps_bounded_by_source_and_traces():
    assert autotune.steps_available(_Shot(10, 2), torch.zeros(50)) == 10
    assert autotune.steps_available(_Shot(100, 2), torch.zeros(50)) == 50
    assert autotune.steps_available(_Shot(10, 0), torch.zeros(50)) == 50  # no receivers: no trace bound
    assert autotune.steps_available(_Shot(0, 0), None) >= 1 << 20


def test_timed_steps_capped_over_all_shots():
    shots = [_Shot(40, 1), _Shot(25, 3)]
    srcs = [torch.zeros(100), torch.zeros(30)]
    assert autotune._timed_steps(shots, srcs, 20) == 20
    assert autotune._timed_steps(shots, srcs, 30, before=3) == 22


def test_timed_steps_refuses_short_shots():
    with pytest.raises(ValueError, match="too few"):
        autotune._timed_steps([_Shot(6, 1)], [torch.zeros(100)], 20, before=3)
