"""Host-side checks of the warm-start experiment (no GPU needed)."""

import pytest

import synth


def test_experiment_refuses_test_maps_that_share_training_seeds():
    from paper_1704_00865_amd import warmstart
    trp = [synth.make_problem(16, 16, s) for s in (1, 2, 3)]
    tep = [synth.make_problem(16, 16, s) for s in (3, 4)]
    with pytest.raises(ValueError, match="share seeds"):
        warmstart.experiment(trp, tep, epochs=1)
